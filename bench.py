"""Benchmark: state-updates/s of the batched sparse transfer-matrix sweep.

Headline workload (one GPU): the square-lattice 14 x 15 rectangle, P read out
after every row, at 80 q points x 8 seeded 31-bit primes = 640 instances,
inputs and maps resident in HBM.  One step = one whole sweep: read-out vector
build (T_last), x = e_0, 14 rows of T_14 ... T_1 with the read-out of every
row, launched as a hipGraph row replay with the autotuned launch shape.

A state-update is one target residue written by a factor launch for one
instance.  `value` counts the residues the step's launches actually write:
with single factors, 14 rows x 787 333 targets x 640 instances = 7.05e9;
a launch that applies a precomputed product of two factors writes only the
product's targets, so fused steps write about half as many.  The count of
per-site factor updates the step performs (every T_i's targets, written or
not) is reported beside it under its own key.

Printed: one JSON line with the headline value, the roofline of the factor
kernel (timed alone with HIP events on its launch stream), the plain
per-instance path on the same workload, the CPU oracle on a bounded sample,
and secondary workloads (the m = 2..14 square sweep as one graph, the
triangular m = 12 strip, the continuous-batching server against the plain
path on a Poisson job stream, the coefficient form on the 14 x 15 strip, the
square 18 x 19 strip, and the finite-lattice series at k = 41 on both
lattices, checked against the paper's Table 1, printed series and Baxter's
product).

Usage: python bench.py [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
WORKLOAD = "square_14x15"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def factor_sizes(lat, m, which=0, count=None):
    """Per factor of a family: (|S_in|, |S_out|, nnz) from the maps."""
    from paper_1005_3609_amd import api
    out = []
    for i in range(count if count is not None else m):
        rp, cols, _, ncols = api.map_export(lat, m, which, i)
        out.append((ncols, rp.size - 1, cols.size))
    return out


def split_jobs(I, V):
    """The jobs a strip of I instances runs as, [(instances, lanes_v)]: at
    lanes_v 4 the instances past the last multiple of 256 form a second job at
    lanes_v 2 (1 for at most 64) instead of a padded chunk."""
    if V == 4 and I > 256 and I % 256:
        rest = I % 256
        return [(I - rest, 4), (rest, 1 if rest <= 64 else 2)]
    return [(I, V)]


def padded_instances(I, V):
    """Instance lanes the strip's launches run (chunks of 64 lanes_v)."""
    return sum(-(-i // (64 * v)) * 64 * v for i, v in split_jobs(I, V))


def kernel_name(I, V, U):
    return "+".join(f"k_gather<{v},{U}>" for _, v in split_jobs(I, V))


def row_bytes(sizes, ipad, s_nc, jobs=1):
    """Bytes of one row of factor applications: for every factor each source
    row read once and each target row written once (4 B per residue per
    instance), its CSR row pointers and entry words, and the read-out vector w
    read once by the read-out fused into the last launch.  `jobs`: the launches
    each factor takes (a lanes_v 4 split reads the map once per job)."""
    total = 0
    for k, (s_in, s_out, nnz) in enumerate(sizes):
        total += 4 * ipad * (s_in + s_out) + jobs * (4 * (s_out + 1) + 4 * nnz)
        if k == len(sizes) - 1:
            total += 4 * ipad * s_nc
    return total


def _oracle_row(args):
    """One transfer row T_m ... T_1 of the unchanged oracle applied to a dense
    seeded vector over all NCNNN states, for the given instances; returns
    (seconds, per-site factor updates)."""
    lat, m, inst, seed = args
    import numpy as np

    from oracle import partitions as OP
    from oracle import transfer as OT
    alg = OT.Residues([a for a, _ in inst], [b for _, b in inst])
    rng = np.random.default_rng(seed)
    vec = {s: rng.integers(0, alg.p) for s in OP.ncnnn_in_paper_order(m)}
    factor = OT.factor_square if lat == "square" else OT.factor_triangular
    t0 = time.perf_counter()
    upd = 0
    for i in range(1, m + 1):
        vec = factor(vec, i, m, alg)
        upd += len(vec)
    return time.perf_counter() - t0, upd * len(inst)


def cpu_baseline(lat, m, q_points, primes):
    """The oracle (unchanged) on the host cores: one transfer row of the
    strip for all of the workload's instances, (a) split into one group of
    instances per host core (at most 16, the GPU machine's share), the groups in
    parallel processes, (b) all instances in one process.  Returns the
    cpu_baseline record."""
    import multiprocessing as mp
    import platform
    import subprocess

    import numpy as np

    from paper_1005_3609_amd import workloads as W
    inst = W.instances(q_points, primes)
    procs = max(1, min(os.cpu_count() or 1, 16, len(inst)))
    groups = [inst[len(inst) * k // procs:len(inst) * (k + 1) // procs] for k in range(procs)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_row, [(lat, m, g, W.SEED_BASE + 77) for g in groups])
    wall = time.perf_counter() - t0
    upd_all = sum(u for _, u in res)
    t_one, upd_one = _oracle_row((lat, m, inst, W.SEED_BASE + 77))
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        model = next((ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")), "")
    except (OSError, subprocess.SubprocessError):
        pass
    return {"value": upd_all / wall, "unit": "state-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"one transfer row (T_{m}..T_1) of the {lat} m={m} strip applied to a dense seeded vector over "
                      f"all NCNNN states for all {len(inst)} instances, {procs} processes of about "
                      f"{len(inst) // procs} instances each ({wall:.1f} s wall, pool start-up included)",
            "single_core": {"value": upd_one / t_one, "unit": "state-updates/s", "seconds": t_one,
                            "sample": f"the same row, all {len(inst)} instances in one process"},
            "host": {"cpu_count": os.cpu_count(), "model": model, "python": platform.python_version(),
                     "numpy": np.__version__}}


def timed(torch, stream, fn, reps=1):
    """Milliseconds per call of fn, HIP events on `stream`."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def timed_no_gc(torch, stream, fn, reps=1):
    """timed() with Python's cyclic garbage collector run first and paused
    inside (as timeit does), for legs made of many short host calls: a
    collection over the interpreter's heap stalls the host for tens of
    milliseconds while the device waits for the next call."""
    import gc
    gc.collect()
    gc.disable()
    try:
        return timed(torch, stream, fn, reps)
    finally:
        gc.enable()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "modarith.hpp"):
        with open(os.path.join(ROOT, "paper_1005_3609_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kname, rtune, workload=WORKLOAD):
    """HBM bytes per factor launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration), or None
    when the kernel source or launch shape differs from what was profiled."""
    path = os.path.join(ROOT, "profiles", f"k_gather_{workload}.md")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("bench-traffic:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec["kernel"] == kname and rec["kernel_src"] == kernel_source_hash() and \
                            rec["tuning"] == {k: rtune.get(k) for k in rec["tuning"]}:
                        return rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def updates_of(lat, m, n, n_inst):
    """Per-site factor updates of a strip: every T_i's targets, rows 2..n."""
    return (n - 1) * sum(s for _, s, _ in factor_sizes(lat, m)) * n_inst


def written_of(lat, m, n, n_inst, fuse=1):
    """Residues the strip's factor launches write: the targets of the
    family's factors (single sites, or products of `fuse` of them)."""
    if fuse <= 1:
        return updates_of(lat, m, n, n_inst)
    nf = -(-m // fuse)
    return (n - 1) * sum(s for _, s, _ in factor_sizes(lat, m, fuse, nf)) * n_inst


def bench_sweep(torch, stream, tune, steps):
    """The square m = 2..14 sweep (n = m+1, 640 instances), all widths in one
    hipGraph of grouped launches."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W
    w = W.workload("square_sweep_2_14")
    jobs = [dict(lattice=lat, m=m, n_max=n, q_points=w["q_points"], primes=w["primes"])
            for lat, m, n in w["strips"]]
    for jb in jobs:
        api.prepare(jb["lattice"], jb["m"])
    from paper_1005_3609_amd import tune as tuner
    t = tuner.lookup_tuned_batch("square_sweep_2_14") or dict(tune)
    t = {k: v for k, v in t.items() if k not in ("mode", "ms", "streams")}
    outs, ws = api.batch(jobs, tuning=t, stream=stream)          # capture
    api.batch(jobs, tuning=t, workspace=ws, outs=outs, stream=stream)  # one warm replay, untimed
    ms = timed_no_gc(torch, stream, lambda: api.batch(jobs, tuning=t, workspace=ws, outs=outs, stream=stream), steps)
    I = len(w["q_points"]) * len(w["primes"])
    upd = sum(updates_of(lat, m, n, I) for lat, m, n in w["strips"])
    wr = sum(written_of(lat, m, n, I, t.get("fuse") or 1) for lat, m, n in w["strips"])
    return {"workload": f"square m=2..14, n=m+1, 640 instances, one graph of grouped launches, tuning {t}",
            "ms_per_step": ms, "value": wr / (ms / 1e3), "unit": "state-updates/s (residues written)",
            "per_site_factor_updates_per_s": upd / (ms / 1e3)}


def _strip_leg(torch, stream, lat, m, n, q, p, mode, t, steps):
    """(ms per strip, residues) of one strip in `mode` with tuning t."""
    from paper_1005_3609_amd import api
    ws = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), mode, t), None)
    res = torch.zeros((n, len(q), len(p)), dtype=torch.int32, device=ws.device)

    def run():
        api.strip_async(lat, m, n, q, p, mode=mode, tuning=t, workspace=ws, out=res, stream=stream)
    run()                                     # capture (graph mode)
    run()                                     # one warm replay, untimed
    ms = timed(torch, stream, run, steps)
    return ms, api.to_u32(res).astype("int64").reshape(n, len(q), len(p))


def _tuned(lat, m, I, n, mode=None):
    """The tuned table's entry (its mode, its tuning), or the best entry of
    `mode` recorded in the table's search."""
    from paper_1005_3609_amd import tune as tuner
    t = dict(tuner.lookup_tuned(lat, m, I, n) or {})
    return t.pop("mode", "graph"), {k: v for k, v in t.items() if k != "ms"}


def bench_small_configs(torch, stream, steps):
    """The two plain-method workloads: the square 4x5 rectangle at q = 0..20
    mod 2^31-1 and the square m = 10 strip (rows 1..11) at 80 q x 4 primes:
    one launch sequence per instance (plain), all instances batched in a
    graph row replay, and the resident mode (the whole strip in one launch,
    vectors in LDS) with the tuned shape; residues equal across the three."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W
    out = {}
    for name in ("square_4x5", "square_m10"):
        w = W.workload(name)
        lat, m, n = w["strips"][0]
        q, p = w["q_points"], w["primes"]
        api.prepare(lat, m)
        I = len(q) * len(p)
        tmode, tt = _tuned(lat, m, I, n)
        legs = {"plain": ("plain", None),
                "graph": ("graph", tt if tmode == "graph" else {}),
                "resident": ("resident", tt if tmode == "resident" else dict(lanes_v=1, waves_per_block=16))}
        rows, ref = {}, None
        for key, (mode, t) in legs.items():
            ms, r = _strip_leg(torch, stream, lat, m, n, q, p, mode, t, steps)
            q1, q2 = q.index(1), q.index(2)
            assert (r[:, q1, :] == 0).all() and (r[:, q2, :] == 2).all(), f"{name} {mode}: P(1) = 0, P(2) = 2 failed"
            if ref is None:
                ref = r
            assert (r == ref).all(), f"{name}: {mode} differs from the plain path"
            rows[key] = {"ms_per_step": ms, "value": updates_of(lat, m, n, I) / (ms / 1e3),
                         "unit": "state-updates/s", "tuning": t}
        rows["workload"] = f"square {m}x{n}, {len(q)} q x {len(p)} primes ({I} instances); plain = one launch " \
                           f"sequence per instance, graph = all instances batched, resident = one launch per strip"
        out[name] = rows
    return out


def bench_triangular(torch, stream, steps):
    """The triangular 12x13 strip (48 q x 6 primes): the tuned shape (the
    resident mode's single launch) beside the graph row replay."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W
    w = W.workload("triangular_m12")
    lat, m, n = w["strips"][0]
    q, p = w["q_points"], w["primes"]
    api.prepare(lat, m)
    I = len(q) * len(p)
    mode, t = _tuned(lat, m, I, n)
    ms, r = _strip_leg(torch, stream, lat, m, n, q, p, mode, t, steps)
    assert (r[:, 0, :] == 0).all() and (r[1:, 1, :] == 0).all() and (r[1:, 2, :] == 6).all(), \
        "triangular invariants P(1) = 0, P(2) = 0, P(3) = 6 failed"
    g_ms, g = _strip_leg(torch, stream, lat, m, n, q, p, "graph", {"lanes_v": 1, "unroll": 8}, steps)
    assert (g == r).all(), "graph and tuned paths differ"
    return {"workload": f"triangular 12x13, 48 q x 6 primes, {mode}, tuning {t}", "ms_per_step": ms,
            "value": written_of(lat, m, n, I, t.get("fuse") or 1) / (ms / 1e3),
            "unit": "state-updates/s (residues written)",
            "per_site_factor_updates_per_s": updates_of(lat, m, n, I) / (ms / 1e3),
            "graph_row_replay_ms": g_ms}


def bench_series(torch, stream, tune, steps):
    """The coefficient form (normalised P~ as truncated polynomials in 1/q,
    x^0..x^79, the paper's series order) on the square 14x15 strip for the
    workload's 8 primes: 8 x 80 = 640 useful coefficient lanes, one launch
    chain per row with the T_last read-out applied to every row's state."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W
    w = W.workload("square_14x15")
    lat, m, n = w["strips"][0]
    primes = w["primes"]
    d = 79
    from paper_1005_3609_amd import tune as tuner
    t = tuner.lookup_tuned_series(lat, m, len(primes), d, n)
    if t is None:
        t = {k: v for k, v in tune.items() if k not in ("fuse", "stage")}
    t = {k: v for k, v in t.items() if k not in ("mode", "ms")}
    t["lanes_v"] = 2
    dev = torch.device("cuda", torch.cuda.current_device())
    out, ws = api.series_async(lat, m, n, d, primes, mode="graph", tuning=t, stream=stream, device=dev)
    api.series_async(lat, m, n, d, primes, mode="graph", tuning=t, workspace=ws, out=out, stream=stream)  # warm
    ms = timed(torch, stream, lambda: api.series_async(lat, m, n, d, primes, mode="graph", tuning=t,
                                                       workspace=ws, out=out, stream=stream), steps)
    res = api.to_u32(out).astype("int64").reshape(n, len(primes), d + 1)
    assert (res[:, :, 0] == 1).all(), "constant term of P~ must be 1"
    lanes = len(primes) * (d + 1)
    return {"workload": f"square 14x15, coefficient form x^0..x^{d} (normalised P~), {len(primes)} seeded primes "
                        f"({lanes} coefficient lanes), graph row replay, tuning {t}",
            "ms_per_step": ms, "value": updates_of(lat, m, n, lanes) / (ms / 1e3), "unit": "state-updates/s"}


def copy_calibration(torch, stream, dev, mib):
    """A plain device copy of `mib` MiB, three times: the HBM counters of a
    kernel of known traffic, to scale FETCH_SIZE and WRITE_SIZE by."""
    nel = mib * (1 << 20) // 4
    src = torch.randint(0, 1 << 30, (nel,), dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    c_ms = timed(torch, stream, lambda: dst.copy_(src), 3)
    log(f"copied {mib} MiB x3 (counter calibration); device copy "
        f"{2 * mib * (1 << 20) / (c_ms / 1e3) / 1e9:.0f} GB/s read+write")


def cf_strip_probe(torch, spec, steps, warmup, log):
    """One coefficient-form strip (`lattice,m,n,d`: P~ of the m x r
    rectangles to x^d, r = 1..n) for one seeded prime with the library's
    launch shape for that chunk width, timed on its own.  Prints one JSON
    line: time per strip and the forward factors' own minimum row traffic
    (each source row read once, each target row written once, the maps).
    Used to take kernel traces and HBM counters of the coefficient form."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import tune as tuner
    from paper_1005_3609_amd import workloads as W
    lat, m, n, d = spec.split(",")
    m, n, d = int(m), int(n), int(d)
    primes = W.seeded_primes(1, 1005)
    lanes_v = tuner.series_lanes_v(d)
    t = dict(tuner.SERIES_WIDE_DEFAULT if lanes_v == 8 else tuner.SERIES_DEFAULT, lanes_v=lanes_v)
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(dev)
    api.prepare_series(lat, m)
    out, ws = api.series_async(lat, m, n, d, primes, mode="graph", tuning=t, stream=stream, device=dev)
    for _ in range(warmup):
        api.series_async(lat, m, n, d, primes, mode="graph", tuning=t, workspace=ws, out=out, stream=stream)
    ms = timed(torch, stream, lambda: api.series_async(lat, m, n, d, primes, mode="graph", tuning=t, workspace=ws,
                                                       out=out, stream=stream), steps)
    res = api.to_u32(out).astype("int64").reshape(n, 1, d + 1)
    assert (res[:, :, 0] == 1).all(), "constant term of P~ must be 1"
    row = 4 * 64 * lanes_v
    fwd = [api.series_map_info(lat, m, 4, i) for i in range(m)]
    own = [row * (nc + nr) + 4 * (nr + 1) + 4 * nz for nr, nc, nz in fwd]
    line = {"probe": "coefficient-form strip", "lattice": lat, "m": m, "n": n, "d_max": d, "primes": 1,
            "tuning": t, "ms_per_strip": ms, "row_bytes": row,
            "forward_factors": [dict(rows=nr, cols=nc, entries=nz, own_min_bytes=b) for (nr, nc, nz), b in zip(fwd, own)]}
    log(f"coefficient form {lat} {m}x1..{n}, x^0..x^{d}: {ms:.2f} ms per strip")
    print(json.dumps(line), flush=True)


def bench_finite_lattice(k):
    """The square-lattice free-energy series of Table 1 by the finite-lattice
    method: coefficient-form strips of widths 1..k/2 on the GPU, per-prime
    combination and CRT on the host; for odd k alpha and beta reach z^{2k-3}
    with the polygon term; checked against the paper's Table 1."""
    from paper_1005_3609_amd import finite_lattice as FL
    from paper_1005_3609_amd import workloads as W
    extra = k % 2 == 1
    t0 = time.perf_counter()
    res = FL.square_series(k, W.seeded_primes(5, 2024), mode="graph", extra=extra)
    dt = time.perf_counter() - t0
    tab = FL._read_table(os.path.join(ROOT, "tests", "golden", "table1_square.txt"))
    names = ("alpha", "beta", "gamma")
    match = all(res[name][i] == tab[i][j] for j, name in enumerate(names) for i in range(len(res[name])))
    assert match, "finite-lattice series differ from Table 1"
    N = len(res["alpha"]) - 1
    return {"workload": f"square-lattice bulk and surface series to z^{N}, corner to z^{len(res['gamma']) - 1} "
                        f"(finite-lattice k = {k}: widths 1..{k // 2}, coefficient form x^0..x^{N}, "
                        f"5 seeded primes{', polygon term' if extra else ''})",
            "seconds": dt, "primes_used": res["primes_used"], "matches_table1": match}


def bench_triangular_series(k):
    """The triangular-lattice series of Sec. 4.4 to x^{k-1} by the
    finite-lattice method on the GPU; surface and corner checked against the
    printed series, bulk against Baxter's product."""
    from paper_1005_3609_amd import finite_lattice as FL
    from paper_1005_3609_amd import workloads as W
    t0 = time.perf_counter()
    res = FL.triangular_series(k, W.seeded_primes(3, 2024), mode="graph")
    dt = time.perf_counter() - t0
    tab = FL._read_table(os.path.join(ROOT, "tests", "golden", "triangular_series.txt"))
    N = k - 1
    match = (all(res["surface"][i] == tab[i][0] and res["corner"][i] == tab[i][1] for i in range(N + 1))
             and res["bulk"] == FL.baxter_bulk(N))
    assert match, "triangular series differ from the paper's"
    return {"workload": f"triangular-lattice bulk, surface and corner series to x^{N} (finite-lattice k = {k}: "
                        f"widths 1..{k // 2}, coefficient form, 3 seeded primes)",
            "seconds": dt, "primes_used": res["primes_used"], "matches_paper": match}


def factor_leg(torch, stream, dev, lat, m, n, q, p, rtune, rows, sizes, s_nc, fuse):
    """The factor launches of `rows` transfer rows of the strip over the
    instances (q x p), one launch per fused factor step and job, one stream:
    {ms, launches, avg_us, own_row, per_site_row, achieved, achieved_per_site}."""
    from paper_1005_3609_amd import api
    I = len(q) * len(p)
    V = rtune.get("lanes_v") or 2
    jobs = split_jobs(I, V)
    ipad = padded_instances(I, V)
    out = torch.zeros((n, len(q), len(p)), dtype=torch.int32, device=dev)
    ws = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), "batched", rtune), dev)
    api.strip_async(lat, m, 1, q, p, mode="batched", tuning=rtune, workspace=ws, out=out, stream=stream)
    api.factor_launches(lat, m, q, p, 1, ws, rtune, stream)
    k_ms = timed(torch, stream, lambda: api.factor_launches(lat, m, q, p, rows, ws, rtune, stream))
    del ws, out
    nf = -(-m // fuse)
    per_site_row = row_bytes(sizes, ipad, s_nc, len(jobs))
    own_row = per_site_row if fuse == 1 else row_bytes(factor_sizes(lat, m, fuse, nf), ipad, s_nc, len(jobs))
    launches = rows * nf * len(jobs)
    return {"kernel": kernel_name(I, V, rtune.get("unroll") or 4), "instances": I, "ms": k_ms,
            "launches": launches, "avg_us": k_ms * 1e3 / launches, "own_row": own_row,
            "per_site_row": per_site_row, "achieved": rows * own_row / (k_ms / 1e3) / 1e9,
            "achieved_per_site": rows * per_site_row / (k_ms / 1e3) / 1e9}


def split_legs(torch, stream, dev, lat, m, n, q, p, rtune, rows, sizes, s_nc, fuse):
    """(dominant, others): the factor leg of the kernel that carries the
    strip.  With a lanes_v 4 split (instances past the last multiple of 256
    as a second job), the dominant kernel is the first job's, timed alone on
    its own instances; the second job alone and both one after the other are
    the others."""
    I = len(q) * len(p)
    jobs = split_jobs(I, rtune.get("lanes_v") or 2)
    if len(jobs) == 2 and jobs[0][0] % len(p) == 0:
        na = jobs[0][0] // len(p)
        dom = factor_leg(torch, stream, dev, lat, m, n, q[:na], p, rtune, rows, sizes, s_nc, fuse)
        second = factor_leg(torch, stream, dev, lat, m, n, q[na:], p, dict(rtune, lanes_v=jobs[1][1]), rows,
                            sizes, s_nc, fuse)
        both = factor_leg(torch, stream, dev, lat, m, n, q, p, rtune, rows, sizes, s_nc, fuse)
        return dom, {"second_job": second, "both_jobs_one_stream": both}
    return factor_leg(torch, stream, dev, lat, m, n, q, p, rtune, rows, sizes, s_nc, fuse), {}


def bench_m18(torch, stream, tune, rows):
    """The square 18x19 strip with the workload's 640 instances: one vector is
    8.2 GB, far beyond the 256 MB Infinity Cache, so the factor kernel's
    bandwidth here is HBM bandwidth.  Reports the whole strip (graph mode,
    the tuned 18x19 shape), the factor kernel timed alone over `rows` rows
    (one launch per factor step, all chunks), and one (q, p) instance through
    the plain path (12.8 MB per vector)."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import tune as tuner
    from paper_1005_3609_amd import workloads as W
    w = W.workload("square_18x19")
    lat, m, n = w["strips"][0]
    q, p = w["q_points"], w["primes"]
    I = len(q) * len(p)
    tuned = tuner.lookup_tuned(lat, m, I, n)
    if tuned:
        tune = {k: v for k, v in tuned.items() if k not in ("mode", "ms")}
    dev = torch.device("cuda", torch.cuda.current_device())
    t0 = time.time()
    api.prepare(lat, m)
    sizes = factor_sizes(lat, m)
    s_nc = api.space_size(m)
    maps_s = time.time() - t0
    V = tune.get("lanes_v") or 2
    fuse = tune.get("fuse") or 1
    ipad = padded_instances(I, V)
    nj = len(split_jobs(I, V))
    out = torch.zeros((n, len(q), len(p)), dtype=torch.int32, device=dev)
    ws = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), "graph", tune), dev)

    def strip():
        api.strip_async(lat, m, n, q, p, mode="graph", tuning=tune, workspace=ws, out=out, stream=stream)
    strip()                                   # fused maps, graph capture
    ms = timed(torch, stream, strip)
    res = api.to_u32(out).astype("int64").reshape(n, len(q), len(p))
    assert (res[:, 0, :] == 0).all() and (res[:, 1, :] == 2).all(), "invariants P(1)=0, P(2)=2 failed at m=18"
    del ws
    rtune = dict(tune, streams=1)
    dom, others = split_legs(torch, stream, dev, lat, m, n, q, p, rtune, rows, sizes, s_nc, fuse)
    achieved = dom["achieved"]
    # one (q, p) instance through the plain path, two rows
    q1, p1 = q[:1], p[:1]
    ws_p = api.alloc_workspace(api.workspace_bytes(lat, m, 3, 1, 1, "plain"), dev)
    out_p = torch.zeros((3, 1, 1), dtype=torch.int32, device=dev)

    def plain():
        api.strip_async(lat, m, 3, q1, p1, mode="plain", workspace=ws_p, out=out_p, stream=stream)
    plain()
    p_ms = timed(torch, stream, plain)
    assert (api.to_u32(out_p).astype("int64").reshape(3) == res[:3, 0, 0]).all(), "plain path differs at m=18"
    p_bytes = 2 * row_bytes(sizes, 1, s_nc)
    return {"workload": "square 18x19, 80 q x 8 seeded primes (640 instances), graph row replay, "
                        f"tuning {tune}",
            "maps_build_s": maps_s, "ms_per_strip": ms,
            "value": written_of(lat, m, n, I, fuse) / (ms / 1e3), "unit": "state-updates/s (residues written)",
            "per_site_factor_updates_per_s": updates_of(lat, m, n, I) / (ms / 1e3),
            "factor_kernel": {"kernel": dom["kernel"], "instances": dom["instances"], "rows_timed": rows,
                              "launches": dom["launches"], "avg_launch_us": dom["avg_us"],
                              "achieved_GBs": achieved, "frac_of_hbm_peak": achieved / HBM_PEAK_GBS,
                              "own_min_bytes_per_row": dom["own_row"], "per_site_bytes_per_row": dom["per_site_row"],
                              "frac_per_site": dom["achieved_per_site"] / HBM_PEAK_GBS,
                              **{k: {kk: vv for kk, vv in v.items()} for k, v in others.items()}},
            "plain_single_instance": {"rows": 2, "ms": p_ms,
                                      "value": updates_of(lat, m, 3, 1) / (p_ms / 1e3),
                                      "algorithmic_GBs": p_bytes / (p_ms / 1e3) / 1e9,
                                      "note": "12.8 MB per vector: cache-resident, not an HBM figure"}}


def bench_serving(torch, n_jobs, n_plain):
    """Continuous batching on a seeded Poisson stream (mean 20 jobs/s) against
    the plain per-instance path serving the same arrivals one job at a time."""
    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W
    from paper_1005_3609_amd.server import GpuBackend, Job, Server, fifo_baseline
    stream_jobs = W.serving_stream(n_jobs)

    def jobs(k):
        return [Job(id=j["id"], lattice=j["lattice"], m=j["m"], n_max=j["n_max"], q_points=j["q_points"],
                    primes=j["primes"], arrival=j["arrival"]) for j in stream_jobs[:k]]
    be = GpuBackend(tuning={"unroll": 8})
    for j in stream_jobs:
        be.prepare(j["lattice"], j["m"])          # maps built before the clock starts
    free, _ = torch.cuda.mem_get_info()
    rep = Server(be, budget_bytes=int(0.8 * free), rows_per_tick=1).run(jobs(n_jobs))
    served = rep.summary()
    # every fifth served job, and the widest of each lattice, run again alone
    done = [j for j in rep.jobs if j.state == "done"]
    pick = {j.id for j in done[::5]}
    for lat in ("square", "triangular"):
        wide = [j for j in done if j.lattice == lat]
        if wide:
            pick.add(max(wide, key=lambda j: (j.m, j.instances)).id)
    checked = 0
    for j in done:
        if j.id in pick:
            alone = api.strip(j.lattice, j.m, j.n_max, j.q_points, j.primes, mode="batched")
            assert (alone.reshape(j.result.shape) == j.result).all(), f"served job {j.id} differs from its run alone"
            checked += 1
    dev = torch.device("cuda", torch.cuda.current_device())
    pstream = torch.cuda.Stream(device=dev)

    def run_plain(j):
        out, ws = api.strip_async(j.lattice, j.m, j.n_max, j.q_points, j.primes, mode="plain", stream=pstream)
        pstream.synchronize()
        j.result = api.to_u32(out)
    rep_p = fifo_baseline(run_plain, jobs(n_plain))
    plain = rep_p.summary()
    return {"stream": f"seeded Poisson, mean 20 jobs/s; lattice U{{sq,tri}}, m U{{6..16}}, n=m+1, "
                      f"q=1..U{{16..80}}, 1-4 primes; {n_jobs} jobs served, the first {n_plain} also through "
                      f"the plain path one job at a time",
            "served": {k: served[k] for k in ("done", "failed", "p50_s", "p99_s", "jobs_per_s", "ticks")},
            "checked_against_alone": checked,
            "plain_fifo": {k: plain[k] for k in ("done", "p50_s", "p99_s", "jobs_per_s")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default=None, choices=["batched", "graph", "grouped"])
    for k in ("lanes-v", "targets-per-wave", "waves-per-block", "xcd-order", "unroll", "streams", "fuse", "stage"):
        ap.add_argument("--" + k, type=int, default=None)
    ap.add_argument("--untuned", action="store_true", help="library defaults instead of the tuned table")
    ap.add_argument("--roofline-rows", type=int, default=10)
    ap.add_argument("--plain-instances", type=int, default=16)
    ap.add_argument("--serve-jobs", type=int, default=120)
    ap.add_argument("--serve-plain-jobs", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="headline and roofline only")
    ap.add_argument("--small", action="store_true",
                    help="with --quick: also the small configurations (square 4x5 and m=10, triangular 12x13)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD, choices=["square_14x15", "square_18x19"],
                    help="strip of the headline and roofline legs (the metric is quoted on square_14x15)")
    ap.add_argument("--no-m18", action="store_true", help="skip the square 18x19 leg (about 2 minutes)")
    ap.add_argument("--m18-rows", type=int, default=1, help="rows of factor launches timed at m=18")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--cf-strip", metavar="LATTICE,M,N,D", default=None,
                    help="only time one coefficient-form strip (one prime, x^0..x^D) and print its own JSON line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sweep shards over instances "
                                   "with no communication, and this program drives one GPU",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import tune as tuner
    from paper_1005_3609_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.cf_strip:
        cf_strip_probe(torch, args.cf_strip, args.steps, args.warmup, log)
        if args.copy_mib:
            copy_calibration(torch, torch.cuda.current_stream(dev), dev, args.copy_mib)
        return
    wname = args.workload
    w = W.workload(wname)
    lat, m, n = w["strips"][0]
    q, p = w["q_points"], w["primes"]
    I = len(q) * len(p)

    tuned = None if args.untuned else tuner.lookup_tuned(lat, m, I, n)
    tune = dict(tuned or {})
    mode = args.mode or tune.pop("mode", "graph")
    tune.pop("mode", None)
    tune.pop("ms", None)
    for k in ("lanes_v", "targets_per_wave", "waves_per_block", "xcd_order", "unroll", "streams", "fuse", "stage"):
        v = getattr(args, k)
        if v is not None:
            tune[k] = v
    V = tune.get("lanes_v") or 2
    fuse = tune.get("fuse") or 1
    ipad = padded_instances(I, V)
    nj = len(split_jobs(I, V))

    t0 = time.time()
    api.prepare(lat, m)
    sizes = factor_sizes(lat, m)
    s_nc = api.space_size(m)
    updates_per_step = updates_of(lat, m, n, I)
    written_per_step = written_of(lat, m, n, I, fuse)
    log(f"maps ready in {time.time() - t0:.1f} s; {written_per_step:.3e} residues written per step "
        f"({updates_per_step:.3e} per-site factor updates); "
        f"mode {mode}, tuning {tune} ({'autotuned table' if tuned else 'given or defaults'})")

    stream = torch.cuda.current_stream(dev)
    out = torch.zeros((n, len(q), len(p)), dtype=torch.int32, device=dev)
    ws = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), mode, tune), dev)

    def step():
        api.strip_async(lat, m, n, q, p, mode=mode, tuning=tune, workspace=ws, out=out, stream=stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    t_wall = time.perf_counter()
    ms_per_step = timed(torch, stream, step, args.steps)
    wall = time.perf_counter() - t_wall
    value = written_per_step / (ms_per_step / 1e3)
    per_site = updates_per_step / (ms_per_step / 1e3)
    res = api.to_u32(out).astype("int64").reshape(n, len(q), len(p))
    assert (res[:, 0, :] == 0).all() and (res[:, 1, :] == 2).all(), "invariants P(1)=0, P(2)=2 failed"
    log(f"{mode}: {ms_per_step:.3f} ms/step, {value:.3e} residues written/s, {per_site:.3e} per-site factor "
        f"updates/s (wall {wall:.2f} s)")

    # ---- roofline of the factor kernel, timed alone -----------------------
    # One launch per factor step over all instance chunks (streams = 1), so
    # that a launch's duration is the kernel's own and matches what a
    # kernel trace reports for this launch shape.
    del ws
    rtune = dict(tune, streams=1)
    R = args.roofline_rows
    dom, others = split_legs(torch, stream, dev, lat, m, n, q, p, rtune, R, sizes, s_nc, fuse)
    launches, avg_us, achieved = dom["launches"], dom["avg_us"], dom["achieved"]
    achieved_per_site = dom["achieved_per_site"]
    own_row_all = row_bytes(factor_sizes(lat, m, fuse, -(-m // fuse)) if fuse > 1 else sizes, ipad, s_nc, nj)
    per_site_row, own_row = dom["per_site_row"], dom["own_row"]
    # the headline step itself: every gather launch's own minimum bytes of the
    # n - 1 transfer rows over the timed step (its other kernels included)
    achieved_step = (n - 1) * own_row_all / (ms_per_step / 1e3) / 1e9
    kname = dom["kernel"]
    log(f"factor kernel {kname} ({dom['instances']} instances): {launches} launches, avg {avg_us:.1f} us, "
        f"{achieved:.0f} GB/s of the launches' own minimum traffic ({achieved_per_site:.0f} GB/s counting every "
        f"per-site factor's reads and writes)")
    for k, v in others.items():
        log(f"  {k}: {v['kernel']} ({v['instances']} instances), avg {v['avg_us']:.1f} us per launch, "
            f"{v['achieved']:.0f} GB/s")

    # ---- plain per-instance path on a subset of the instances -------------
    plain = None
    if not args.no_plain and not args.quick:
        k = args.plain_instances
        qs_sub, ps_sub = q[: max(1, k // len(p))], p
        Ik = len(qs_sub) * len(ps_sub)
        ws_p = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(qs_sub), len(ps_sub), "plain"), dev)
        out_p = torch.zeros((n, len(qs_sub), len(ps_sub)), dtype=torch.int32, device=dev)

        def plain_step():
            api.strip_async(lat, m, n, qs_sub, ps_sub, mode="plain", workspace=ws_p, out=out_p, stream=stream)
        plain_step()
        p_ms = timed(torch, stream, plain_step)
        ref = res[:, : len(qs_sub), :]
        assert (api.to_u32(out_p).astype("int64") == ref).all(), "plain path differs from batched"
        plain = {"value": updates_of(lat, m, n, Ik) / (p_ms / 1e3), "unit": "state-updates/s",
                 "instances_timed": Ik, "ms_per_instance": p_ms / Ik,
                 "note": "single factors: every residue written is a per-site factor update"}
        plain["batched_speedup_per_site_updates"] = per_site / plain["value"]
        log(f"plain: {plain['value']:.3e} state-updates/s over {Ik} instances")

    extra = {}
    if not args.quick or args.small:
        extra["plain_configs"] = bench_small_configs(torch, stream, max(5, args.steps // 2))
        log("plain configs: " + ", ".join(f"{k} plain {v['plain']['ms_per_step']:.3f} / graph "
                                          f"{v['graph']['ms_per_step']:.3f} / resident "
                                          f"{v['resident']['ms_per_step']:.3f} ms"
                                          for k, v in extra["plain_configs"].items()))
        extra["triangular_12x13"] = bench_triangular(torch, stream, max(20, args.steps))
        log(f"triangular m=12: {extra['triangular_12x13']['ms_per_step']:.3f} ms "
            f"(graph row replay {extra['triangular_12x13']['graph_row_replay_ms']:.3f} ms)")
    if not args.quick:
        extra["sweep_square_2_14"] = bench_sweep(torch, stream, tune, max(2, args.steps // 4))
        log(f"sweep m=2..14: {extra['sweep_square_2_14']['value']:.3e} state-updates/s")
        extra["serving"] = bench_serving(torch, args.serve_jobs, args.serve_plain_jobs)
        log(f"serving: {extra['serving']}")
        extra["finite_lattice_square"] = bench_finite_lattice(41)
        log(f"finite-lattice series: {extra['finite_lattice_square']}")
        extra["finite_lattice_triangular"] = bench_triangular_series(41)
        log(f"triangular series: {extra['finite_lattice_triangular']}")
        extra["series_square_14x15"] = bench_series(torch, stream, tune, max(2, args.steps // 2))
        log(f"coefficient form m=14: {extra['series_square_14x15']['value']:.3e} state-updates/s, "
            f"{extra['series_square_14x15']['ms_per_step']:.2f} ms/strip")
    if not args.quick and not args.no_m18 and wname != "square_18x19":
        extra["square_18x19"] = bench_m18(torch, stream, tune, args.m18_rows)
        k = extra["square_18x19"]["factor_kernel"]
        log(f"square 18x19: {extra['square_18x19']['value']:.3e} state-updates/s, factor kernel "
            f"{k['avg_launch_us']:.0f} us/launch, {k['achieved_GBs']:.0f} GB/s algorithmic "
            f"({100 * k['frac_of_hbm_peak']:.0f} % of HBM peak)")

    # ---- CPU oracle on a bounded sample -----------------------------------
    cpu = None
    if not args.no_cpu and not args.quick and wname == "square_14x15":
        cpu = cpu_baseline(lat, m, q, p)
        log(f"cpu oracle: {cpu['value']:.3e} state-updates/s on {cpu['cores']} processes, "
            f"{cpu['single_core']['value']:.3e} on one")

    if args.copy_mib:
        copy_calibration(torch, stream, dev, args.copy_mib)

    line = {
        "metric": f"state-updates/s (residues written by the factor launches), square lattice m={m} "
                  f"({m}x{n} strip), batched",
        "value": value,
        "unit": "state-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"square {m}x{n} strip, 80 q x 8 seeded primes (640 instances), "
                               "row-by-row read-out", "lattice": lat, "m": m, "n_max": n,
                   "instances": I, "mode": mode, "tuning": tune, "autotuned": bool(tuned)},
        "per_site_factor_updates": {"value": per_site, "unit": "state-updates/s",
                                    "note": "every per-site factor T_i's targets per step, including the "
                                            "intermediate ones a fused launch never writes"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, rtune, wname),
                     "kernel": kname, "instances": dom["instances"], "avg_launch_us": avg_us,
                     "launches_timed": launches,
                     **({"other_legs": others} if others else {}),
                     "bytes": "each launch's own minimum: its input and output vectors once, its map, "
                              "and the read-out vector with the last launch of a row",
                     "own_min_bytes_per_row": own_row, "per_site_bytes_per_row": per_site_row,
                     "achieved_per_site": achieved_per_site, "frac_per_site": achieved_per_site / HBM_PEAK_GBS,
                     "achieved_step": achieved_step, "frac_step": achieved_step / HBM_PEAK_GBS,
                     "step_note": "the timed headline step (its own launch shape, every kernel of the step): the "
                                  "gather launches' own minimum bytes over ms_per_step"},
        "plain": plain,
        "cpu_baseline": cpu,
        "secondary": extra or None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
