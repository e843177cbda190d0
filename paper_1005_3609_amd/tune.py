"""Autotuner for the batched sweep: launch shape and execution mode.

Searches instances per lane (chunk width W = 64 V), targets per wavefront,
wavefronts per workgroup and the execution mode (hipGraph row replay, the
whole sweep as one graph of grouped launches, or the resident mode's single
launch with the vectors in LDS, where the width fits), timing whole sweeps
with HIP events on the launch stream.  Every candidate must return residues bit-identical to the first
one; a candidate that differs is rejected and reported (the arithmetic is
exact, so a difference is a bug, never rounding).  Results are cached as
JSON keyed by (gfx arch, lattice, m, instances, n_max).

The coefficient form (normalised P~ as truncated polynomials, one chunk per
prime) is tuned the same way over its own space (single factors, no
staging, graph row replay), keyed by (gfx arch, "series", lattice, m,
primes x coefficients, n_max).
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from . import api

DEFAULT_CACHE = os.environ.get("CHROMSTRIP_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "chromstrip", "tune.json"))
SPACE = dict(lanes_v=[1, 2, 4], targets_per_wave=[4, 8, 16], waves_per_block=[2, 4, 8],
             xcd_order=[1, 2], unroll=[4, 8], streams=[1, 2], fuse=[1, 2, 3], stage=[0, 1, 2, 3, 4, 5, 6],
             mode=["graph", "grouped"])


def candidates(space=None) -> list[dict]:
    space = space or SPACE
    out = []
    for v, t, w, x, u, s, f, g, mode in itertools.product(space["lanes_v"], space["targets_per_wave"],
                                                          space["waves_per_block"], space.get("xcd_order", [0]),
                                                          space.get("unroll", [4]), space.get("streams", [1]),
                                                          space.get("fuse", [1]), space.get("stage", [0]),
                                                          space["mode"]):
        if mode == "resident":
            continue            # its own candidates: resident_candidates
        if mode == "grouped" and s != 1:
            continue            # grouped launches already cover every chunk at once
        if g and g not in (4, 6) and (mode == "grouped" or v > 2):
            continue            # staging and op streams apply to graph / batched launches (lanes_v <= 2);
                                # the target orders (4, 6) to every mode
        out.append(dict(lanes_v=v, targets_per_wave=t, waves_per_block=w, xcd_order=x, unroll=u, streams=s,
                        fuse=f, stage=g, mode=mode))
    return out


# Resident mode (one launch per strip, vectors in LDS): instances per
# workgroup, wavefronts per workgroup, fused family.
# stage: 0 = exact double accumulation where its bound holds, 1 = modular
RESIDENT_SPACE = dict(lanes_v=[1, 2, 4], waves_per_block=[8, 16], fuse=[1, 2, 3], stage=[0, 1])


def resident_candidates(lattice, m, n_inst, n_max, space=None) -> list[dict]:
    """Resident-mode candidates whose two state vectors fit a workgroup's LDS."""
    space = space or RESIDENT_SPACE
    out = []
    for v, w, f, g in itertools.product(space["lanes_v"], space["waves_per_block"], space["fuse"],
                                        space.get("stage", [0])):
        t = dict(lanes_v=v, waves_per_block=w, fuse=f, stage=g)
        try:
            api.workspace_bytes(lattice, m, n_max, n_inst, 1, "resident", t)
        except api.ChromError:
            continue
        out.append(dict(t, mode="resident"))
    return out


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(lattice, m, n_inst, n_max):
    return f"{_arch()}|{lattice}|{m}|{n_inst}|{n_max}"


def load(path=DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(lattice, m, n_inst, n_max, path=DEFAULT_CACHE):
    return load(path).get(_key(lattice, m, n_inst, n_max))


PACKAGE_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def lookup_tuned(lattice, m, n_inst, n_max):
    """Best known configuration: the user's tuning cache first, then the
    table shipped with the package.  None if neither has the workload."""
    for path in (DEFAULT_CACHE, PACKAGE_TABLE):
        hit = load(path).get(_key(lattice, m, n_inst, n_max))
        if hit:
            return dict(hit["best"])
    return None


def time_candidate(lattice, m, n_max, q_points, primes, cand, steps=3, stream=None):
    """(ms per sweep, residues) for one candidate."""
    import torch
    tune = {k: v for k, v in cand.items() if k != "mode"}
    mode = cand["mode"]
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream or torch.cuda.current_stream(dev)
    ws = api.alloc_workspace(api.workspace_bytes(lattice, m, n_max, len(q_points), len(primes), mode, tune), dev)
    out = torch.zeros((n_max, len(q_points), len(primes)), dtype=torch.int32, device=dev)
    api.strip_async(lattice, m, n_max, q_points, primes, mode=mode, tuning=tune, workspace=ws, out=out,
                    stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        api.strip_async(lattice, m, n_max, q_points, primes, mode=mode, tuning=tune, workspace=ws, out=out,
                        stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, api.to_u32(out)


def tune(lattice, m, n_max, q_points, primes, space=None, steps=3, path=DEFAULT_CACHE, log=None,
         resident_only=False) -> dict:
    """Times every candidate, keeps the fastest bit-identical one, caches it.
    resident_only: the resident-mode candidates plus the best known entry."""
    table = []
    ref = None
    best = None
    n_inst = len(q_points) * len(primes)
    if resident_only:
        cands = resident_candidates(lattice, m, n_inst, n_max)
        known = lookup_tuned(lattice, m, n_inst, n_max)
        if known:
            known.pop("ms", None)
            cands = [known] + cands
    else:
        cands = candidates(space)
        if "resident" in (space or SPACE)["mode"]:
            cands += resident_candidates(lattice, m, n_inst, n_max)
    for cand in cands:
        ms, res = time_candidate(lattice, m, n_max, q_points, primes, cand, steps)
        if ref is None:
            ref = res
        ok = bool(np.array_equal(res, ref))
        table.append(dict(cand, ms=ms, identical=ok))
        if log:
            log(f"{cand} {ms:.3f} ms {'ok' if ok else 'MISMATCH'}")
        if ok and (best is None or ms < best["ms"]):
            best = dict(cand, ms=ms)
    bad = [t for t in table if not t["identical"]]
    if bad:
        raise RuntimeError(f"tuning candidates disagree with the reference result: {bad}")
    cache = load(path)
    cache[_key(lattice, m, len(q_points) * len(primes), n_max)] = dict(best=best, table=table)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return dict(best=best, table=table)


# Coefficient-form launch shape used where no tuned entry exists: the best of
# SERIES_SPACE for square m = 14, 8 primes x 80 coefficients on the MI355X
# (wider wavefront tiles than the evaluation form's).
SERIES_DEFAULT = dict(targets_per_wave=16, waves_per_block=4, xcd_order=1, unroll=4, streams=3)
# 512-slot rows (lanes_v 8), one prime per call: square m = 18, x^0..x^419,
# swept over targets_per_wave 2..32, waves_per_block 1..8, xcd_order 1..2
# on the MI355X: 115 ms per 3-row strip, against 127 ms at 8 x 4.
SERIES_WIDE_DEFAULT = dict(targets_per_wave=16, waves_per_block=1, xcd_order=1, unroll=4, streams=1)

SERIES_SPACE = dict(targets_per_wave=[4, 8, 16], waves_per_block=[4, 8], xcd_order=[1], unroll=[4, 8],
                    streams=[1, 3])


def _series_key(lattice, m, n_primes, d_max, n_max):
    return f"{_arch()}|series|{lattice}|{m}|{n_primes}x{d_max + 1}|{n_max}"


def series_lanes_v(d_max: int) -> int:
    """Smallest chunk width (64 lanes_v coefficients) that holds x^0..x^d_max."""
    return 1 if d_max < 64 else (2 if d_max < 128 else (4 if d_max < 256 else 8))


def lookup_tuned_series(lattice, m, n_primes, d_max, n_max):
    """Best known coefficient-form launch shape (user cache, then the shipped
    table), or None."""
    for path in (DEFAULT_CACHE, PACKAGE_TABLE):
        hit = load(path).get(_series_key(lattice, m, n_primes, d_max, n_max))
        if hit:
            return dict(hit["best"])
    return None


def tune_series(lattice, m, n_max, d_max, primes, space=None, steps=3, path=DEFAULT_CACHE, log=None) -> dict:
    """Times coefficient-form strips over the launch-shape space; every
    candidate's coefficients must equal the first one's."""
    import torch
    space = space or SERIES_SPACE
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(dev)
    table, ref, best = [], None, None
    lanes_v = series_lanes_v(d_max)
    for t, w, x, u, s in itertools.product(space["targets_per_wave"], space["waves_per_block"],
                                           space["xcd_order"], space["unroll"], space["streams"]):
        if lanes_v == 8 and u != 4:
            continue                    # 512-slot rows run with unroll 4 only
        cand = dict(lanes_v=lanes_v, targets_per_wave=t, waves_per_block=w, xcd_order=x, unroll=u, streams=s)
        out, ws = api.series_async(lattice, m, n_max, d_max, primes, mode="graph", tuning=cand, stream=stream,
                                   device=dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            api.series_async(lattice, m, n_max, d_max, primes, mode="graph", tuning=cand, workspace=ws, out=out,
                             stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res = api.to_u32(out)
        if ref is None:
            ref = res
        ok = bool(np.array_equal(res, ref))
        table.append(dict(cand, ms=ms, identical=ok))
        if log:
            log(f"{cand} {ms:.3f} ms {'ok' if ok else 'MISMATCH'}")
        if ok and (best is None or ms < best["ms"]):
            best = dict(cand, mode="graph", ms=ms)
        del out, ws
    bad = [t for t in table if not t["identical"]]
    if bad:
        raise RuntimeError(f"tuning candidates disagree with the reference result: {bad}")
    cache = load(path)
    cache[_series_key(lattice, m, len(primes), d_max, n_max)] = dict(best=best, table=table)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return dict(best=best, table=table)


BATCH_SPACE = dict(lanes_v=[1, 2], targets_per_wave=[4, 8], waves_per_block=[4, 8], xcd_order=[1], unroll=[4],
                   fuse=[1, 2], stage=[0, 6])


def _batch_key(name: str):
    return f"{_arch()}|batch|{name}"


def lookup_tuned_batch(name: str):
    """Best known grouped-launch shape for a named job list, or None."""
    for path in (DEFAULT_CACHE, PACKAGE_TABLE):
        hit = load(path).get(_batch_key(name))
        if hit:
            return dict(hit["best"])
    return None


def tune_batch(name: str, jobs, space=None, steps=3, path=DEFAULT_CACHE, log=None) -> dict:
    """Times one hipGraph of grouped launches over `jobs` (chromatic_batch)
    for every launch shape of the space; every candidate's residues must
    equal the first one's.  Cached under `name`."""
    import torch
    space = space or BATCH_SPACE
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(dev)
    table, ref, best = [], None, None
    for v, t, w, x, u, f, st, g in itertools.product(space["lanes_v"], space["targets_per_wave"],
                                                     space["waves_per_block"], space["xcd_order"], space["unroll"],
                                                     space["fuse"], space.get("streams", [1]), space.get("stage", [0])):
        cand = dict(lanes_v=v, targets_per_wave=t, waves_per_block=w, xcd_order=x, unroll=u, fuse=f, streams=st,
                    stage=g)
        outs, ws = api.batch(jobs, tuning=cand, stream=stream, device=dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            api.batch(jobs, tuning=cand, workspace=ws, outs=outs, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res = [api.to_u32(o) for o in outs]
        if ref is None:
            ref = res
        ok = all(np.array_equal(a, b) for a, b in zip(res, ref))
        table.append(dict(cand, ms=ms, identical=ok))
        if log:
            log(f"{cand} {ms:.3f} ms {'ok' if ok else 'MISMATCH'}")
        if ok and (best is None or ms < best["ms"]):
            best = dict(cand, mode="grouped", ms=ms)
        del outs, ws
    bad = [t for t in table if not t["identical"]]
    if bad:
        raise RuntimeError(f"tuning candidates disagree with the reference result: {bad}")
    cache = load(path)
    cache[_batch_key(name)] = dict(best=best, table=table)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return dict(best=best, table=table)


def main():
    """python -m paper_1005_3609_amd.tune --workload square_14x15 [--cache PATH] [--series D]"""
    import argparse
    import sys

    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="square_14x15")
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="a reduced search space")
    ap.add_argument("--batch", action="store_true",
                    help="tune the workload's strips as one batch of grouped launches (chromatic_batch)")
    ap.add_argument("--space", default=None, metavar="JSON",
                    help="a search space as JSON (keys of SPACE, each a list)")
    ap.add_argument("--resident", action="store_true",
                    help="the resident mode's candidates against the best known entry")
    ap.add_argument("--medium", action="store_true",
                    help="lanes_v 1-2, fused families 1-3, one or three chunk groups, graph mode (96 candidates)")
    ap.add_argument("--series", type=int, default=None, metavar="D",
                    help="tune the coefficient form to x^D for the workload's strips and primes instead")
    args = ap.parse_args()
    w = W.workload(args.workload)
    if args.batch:
        jobs = [dict(lattice=lat, m=m, n_max=n, q_points=w["q_points"], primes=w["primes"])
                for lat, m, n in w["strips"]]
        for jb in jobs:
            api.prepare(jb["lattice"], jb["m"])
        res = tune_batch(args.workload, jobs, steps=args.steps, path=args.cache,
                         log=lambda s: print(s, file=sys.stderr, flush=True))
        print(json.dumps(dict(workload=args.workload, batch=True, best=res["best"])), flush=True)
        return
    if args.series is not None:
        for lat, m, n in w["strips"]:
            res = tune_series(lat, m, n, args.series, w["primes"], steps=args.steps, path=args.cache,
                              log=lambda s: print(s, file=sys.stderr, flush=True))
            print(json.dumps(dict(workload=args.workload, series_d_max=args.series, lattice=lat, m=m, n_max=n,
                                  best=res["best"])), flush=True)
        return
    space = None
    if args.medium:
        space = dict(lanes_v=[1, 2], targets_per_wave=[4, 8], waves_per_block=[4, 8], xcd_order=[1],
                     unroll=[4, 8], streams=[1, 3], fuse=[1, 2, 3], stage=[0], mode=["graph"])
    if args.quick:
        space = dict(lanes_v=[2], targets_per_wave=[4, 8], waves_per_block=[4, 8], xcd_order=[1],
                     unroll=[4], streams=[3], fuse=[2], stage=[0, 1], mode=["graph"])
    if args.space:
        space = dict(SPACE, **json.loads(args.space))
    for lat, m, n in w["strips"]:
        api.prepare(lat, m)
        res = tune(lat, m, n, w["q_points"], w["primes"], space=space, steps=args.steps, path=args.cache,
                   log=lambda s: print(s, file=sys.stderr, flush=True), resident_only=args.resident)
        print(json.dumps(dict(workload=args.workload, lattice=lat, m=m, n_max=n, best=res["best"])), flush=True)


if __name__ == "__main__":
    main()
