"""Benchmark: state-updates/s of the batched sparse transfer-matrix sweep.

Workload (one GPU): the square-lattice 14 x 15 rectangle, P read out after
every row, at 80 q points x 8 seeded 31-bit primes = 640 instances, inputs
and maps resident in HBM.  One step = one whole sweep: read-out vector build
(T_last), x = e_0, 14 rows of T_14 ... T_1 with the read-out of every row.

A state-update is one target residue written by one forward per-site factor
T_i for one instance; a step performs 14 rows x 787 333 targets x 640
instances = 7.05e9 of them.

Printed: one JSON line with the headline value, the roofline of the factor
kernel (timed alone with HIP events on its launch stream), the plain
per-instance path on the same workload, and the CPU oracle on a bounded
sample.  Usage: python bench.py [--steps K] [--warmup W] [--mode graph]
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


def factor_sizes(lat, m):
    """Per forward factor T_i: (|S_in|, |S_out|, nnz) from the maps."""
    from paper_1005_3609_amd import api
    out = []
    for i in range(m):
        rp, cols, _, ncols = api.map_export(lat, m, 0, i)
        out.append((ncols, rp.size - 1, cols.size))
    return out


def algorithmic_bytes_per_row(sizes, ipad, s_nc):
    """Bytes one row of factor launches must move at minimum: every source
    row read once and every target row written once (4 B per residue per
    instance), the CSR row pointers and entry words, and the read-out vector
    w read once by the fused read-out in T_m."""
    total = 0
    for k, (s_in, s_out, nnz) in enumerate(sizes):
        total += 4 * ipad * (s_in + s_out) + 4 * (s_out + 1) + 4 * nnz
        if k == len(sizes) - 1:
            total += 4 * ipad * s_nc
    return total


def cpu_baseline(lat, m, q_points, primes, n_inst=64):
    """The oracle, unchanged, applying one transfer row T_m ... T_1 to a dense
    seeded state vector over all NCNNN states, for the first n_inst of the
    workload's instances (single process)."""
    import numpy as np

    from oracle import partitions as OP
    from oracle import transfer as OT
    from paper_1005_3609_amd import workloads as W
    inst = W.instances(q_points, primes)[:n_inst]
    alg = OT.Residues([a for a, _ in inst], [b for _, b in inst])
    rng = np.random.default_rng(W.SEED_BASE + 77)
    vec = {s: rng.integers(0, alg.p) for s in OP.ncnnn_in_paper_order(m)}
    factor = OT.factor_square if lat == "square" else OT.factor_triangular
    t0 = time.perf_counter()
    for i in range(1, m + 1):
        vec = factor(vec, i, m, alg)
    dt = time.perf_counter() - t0
    return dt, n_inst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="graph", choices=["batched", "graph", "grouped"])
    ap.add_argument("--lanes-v", type=int, default=0)
    ap.add_argument("--targets-per-wave", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--xcd-order", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--streams", type=int, default=0)
    ap.add_argument("--fuse", type=int, default=0)
    ap.add_argument("--roofline-rows", type=int, default=10)
    ap.add_argument("--plain-instances", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sweep shards over instances "
                                   "with no communication, and multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1005_3609_amd import api
    from paper_1005_3609_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = W.workload(WORKLOAD)
    lat, m, n = w["strips"][0]
    q, p = w["q_points"], w["primes"]
    I = len(q) * len(p)
    tune = {"lanes_v": args.lanes_v, "targets_per_wave": args.targets_per_wave,
            "waves_per_block": args.waves_per_block, "xcd_order": args.xcd_order,
            "unroll": args.unroll, "streams": args.streams, "fuse": args.fuse}
    V = args.lanes_v or 2
    ipad = -(-I // (64 * V)) * 64 * V

    t0 = time.time()
    api.prepare(lat, m)
    sizes = factor_sizes(lat, m)
    s_nc = api.space_size(m)
    updates_per_row = sum(s_out for _, s_out, _ in sizes) * I
    updates_per_step = (n - 1) * updates_per_row
    log(f"maps ready in {time.time() - t0:.1f} s; {updates_per_step:.3e} state-updates per step")

    stream = torch.cuda.current_stream(dev)
    out = torch.zeros((n, len(q), len(p)), dtype=torch.int32, device=dev)
    ws = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), args.mode, tune), dev)
    for _ in range(args.warmup):
        api.strip_async(lat, m, n, q, p, mode=args.mode, tuning=tune, workspace=ws, out=out, stream=stream)
    torch.cuda.synchronize()
    log("warmup done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        api.strip_async(lat, m, n, q, p, mode=args.mode, tuning=tune, workspace=ws, out=out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    value = updates_per_step / (ms_per_step / 1e3)
    res = api.to_u32(out).astype("int64").reshape(n, len(q), len(p))
    assert (res[:, 0, :] == 0).all() and (res[:, 1, :] == 2).all(), "invariants P(1)=0, P(2)=2 failed"
    log(f"{args.mode}: {ms_per_step:.3f} ms/step, {value:.3e} state-updates/s (wall {wall:.2f} s)")

    # ---- roofline of the factor kernel, timed alone -----------------------
    del ws
    ws_b = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(q), len(p), "batched", tune), dev)
    api.strip_async(lat, m, n, q, p, mode="batched", tuning=tune, workspace=ws_b, out=out, stream=stream)
    api.factor_launches(lat, m, q, p, 2, ws_b, tune, stream)
    torch.cuda.synchronize()
    R = args.roofline_rows
    ev0.record(stream)
    api.factor_launches(lat, m, q, p, R, ws_b, tune, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_ms = ev0.elapsed_time(ev1)
    launches = R * m
    avg_us = k_ms * 1e3 / launches
    bytes_row = algorithmic_bytes_per_row(sizes, ipad, s_nc)
    achieved = R * bytes_row / (k_ms / 1e3) / 1e9
    log(f"factor kernel: {launches} launches, avg {avg_us:.1f} us, {achieved:.0f} GB/s algorithmic")
    del ws_b

    # ---- plain per-instance path on a subset of the instances -------------
    plain = None
    if not args.no_plain:
        k = args.plain_instances
        qs_sub, ps_sub = q[: max(1, k // len(p))], p
        Ik = len(qs_sub) * len(ps_sub)
        ws_p = api.alloc_workspace(api.workspace_bytes(lat, m, n, len(qs_sub), len(ps_sub), "plain"), dev)
        out_p = torch.zeros((n, len(qs_sub), len(ps_sub)), dtype=torch.int32, device=dev)
        api.strip_async(lat, m, n, qs_sub, ps_sub, mode="plain", workspace=ws_p, out=out_p, stream=stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        api.strip_async(lat, m, n, qs_sub, ps_sub, mode="plain", workspace=ws_p, out=out_p, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        p_ms = ev0.elapsed_time(ev1)
        ref = res[:, : len(qs_sub), :]
        assert (api.to_u32(out_p).astype("int64") == ref).all(), "plain path differs from batched"
        plain = {"value": (n - 1) * sum(s for _, s, _ in sizes) * Ik / (p_ms / 1e3),
                 "unit": "state-updates/s", "instances_timed": Ik,
                 "ms_per_instance": p_ms / Ik, "batched_speedup": None}
        plain["batched_speedup"] = value / plain["value"]
        log(f"plain: {plain['value']:.3e} state-updates/s over {Ik} instances")

    # ---- CPU oracle on a bounded sample -----------------------------------
    cpu = None
    if not args.no_cpu:
        dt, ninst = cpu_baseline(lat, m, q, p)
        upd = sum(s for _, s, _ in sizes) * ninst
        cpu = {"value": upd / dt, "unit": "state-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"one transfer row (T_14..T_1) of the square m=14 sweep applied to a dense seeded "
                         f"vector over all {s_nc} NCNNN states, first {ninst} of the 640 instances, "
                         f"{dt:.1f} s single-threaded Python"}
        log(f"cpu oracle: {cpu['value']:.3e} state-updates/s")

    if args.copy_mib:
        nel = args.copy_mib * (1 << 20) // 4
        src = torch.randint(0, 1 << 30, (nel,), dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(3):
            dst.copy_(src)
        ev1.record(stream)
        torch.cuda.synchronize()
        c_ms = ev0.elapsed_time(ev1) / 3
        log(f"copied {args.copy_mib} MiB x4 (counter calibration); device copy "
            f"{2 * args.copy_mib * (1 << 20) / (c_ms / 1e3) / 1e9:.0f} GB/s read+write")

    line = {
        "metric": "state-updates/s, square lattice m=14 (14x15 strip), batched",
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
        "config": {"workload": "square 14x15 strip, 80 q x 8 seeded primes (640 instances), "
                               "row-by-row read-out", "lattice": lat, "m": m, "n_max": n,
                   "instances": I, "mode": args.mode, "tuning": tune},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"k_gather<{V}>", "avg_launch_us": avg_us,
                     "algorithmic_bytes_per_row": bytes_row, "launches_timed": launches},
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
