"""Write the stored oracle values that the GPU parity tests compare against.

Calls only the CPU oracle (``oracle.transfer``) and the seeded input
generator; nothing here touches the GPU path.  Run from the repository root:

    python tests/golden/make_golden.py [--jobs 8]

Each output file ``oracle_<lattice>_<m>x<n>.json`` holds P of the m x r
rectangles, r = 1..n, modulo p, for a seeded sample of the workload's
instances (q, p).  Tall rectangles that the oracle cannot sweep directly
(width 18) are stored through transposition symmetry, P(m x r) = P(r x m):
the oracle computes the narrow width r with m rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import transfer as T                       # noqa: E402
from paper_1005_3609_amd import workloads as W         # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _direct(task):
    """Sweep width m to n rows on the sampled instances."""
    name, lat, m, n, sample, seed = task
    w = W.workload(name)
    inst = W.instances(w["q_points"], w["primes"])
    idx = W.sample_instances(len(inst), sample, seed)
    qs = [inst[k][0] for k in idx]
    ps = [inst[k][1] for k in idx]
    t0 = time.time()
    z = T.chromatic_residues(lat, m, n, qs, ps)
    out = dict(workload=name, lattice=lat, m=m, n_max=n, how="direct",
               instance_index=idx, q=qs, p=ps,
               z=[[int(x) for x in row] for row in z], oracle_seconds=time.time() - t0)
    path = os.path.join(HERE, f"oracle_{lat}_{m}x{n}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    return path, out["oracle_seconds"]


def _transposed(task):
    """P(m x r) for r = 1..rmax via P(r x m): width r swept to m rows."""
    name, lat, m, n, rmax, sample, seed = task
    w = W.workload(name)
    inst = W.instances(w["q_points"], w["primes"])
    idx = W.sample_instances(len(inst), sample, seed)
    qs = [inst[k][0] for k in idx]
    ps = [inst[k][1] for k in idx]
    t0 = time.time()
    rows = []
    for r in range(1, rmax + 1):
        z = T.chromatic_residues(lat, r, m, qs, ps)[m - 1]
        rows.append([int(x) for x in z])
    out = dict(workload=name, lattice=lat, m=m, n_max=n, how="transposed",
               rows_present=rmax, instance_index=idx, q=qs, p=ps, z=rows,
               oracle_seconds=time.time() - t0)
    path = os.path.join(HERE, f"oracle_{lat}_{m}x{n}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    return path, out["oracle_seconds"]


def _run(task):
    return _transposed(task[1:]) if task[0] == "T" else _direct(task[1:])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--only", default=None, help="comma list of output stems")
    args = ap.parse_args()
    seed = W.SEED_BASE + 99
    tasks = [
        ("T", "square_18x19", "square", 18, 19, 13, 16, seed),
        ("D", "square_sweep_2_14", "square", 14, 15, 64, seed),
        ("D", "square_sweep_2_14", "square", 13, 14, 64, seed),
        ("D", "triangular_m12", "triangular", 12, 13, 288, seed),
        ("D", "square_sweep_2_14", "square", 12, 13, 64, seed),
        ("D", "square_sweep_2_14", "square", 11, 12, 64, seed),
    ]
    if args.only:
        keep = set(args.only.split(","))
        tasks = [t for t in tasks if f"{t[2]}_{t[3]}x{t[4]}" in keep]
    with Pool(min(args.jobs, len(tasks))) as pool:
        for path, secs in pool.imap_unordered(_run, tasks):
            print(f"{os.path.basename(path)}: oracle {secs:.1f} s", flush=True)


if __name__ == "__main__":
    main()
