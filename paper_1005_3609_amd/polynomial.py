"""Exact chromatic polynomials of rectangles from the GPU coefficient form.

P_G(q) of the m x r rectangles, r = 1..n, as integer coefficient lists
(q^0 .. q^|V|), without interpolation: the coefficient form gives the
normalised P~ = q^{-|V|} P (eq. Z_modified) as coefficients of x^0..x^d mod
each prime, and with d = |V| - 1 (the constant term of P is 0) the whole
polynomial is known mod p: the coefficient of q^{|V| - k} in P is that of
x^k in P~.  Primes are added until the CRT lift stops changing (Sec. 3.5).

    python -m paper_1005_3609_amd.polynomial square 6 7
"""
from __future__ import annotations

from . import api, host
from . import workloads as W


def chromatic_polynomials(lattice, m: int, n: int, primes=None, batch: int = 4, max_primes: int = 64):
    """[P_{m x r}(q) for r = 1..n], each a list of integers c_0..c_{|V|}
    with P = sum c_j q^j.  Needs m n <= 256 (coefficients x^0..x^{mn-1} in
    at most 4 lanes per wavefront lane).  Primes are drawn in groups of
    `batch` from `primes` (default: seeded 31-bit primes) until every row's
    lift is stable; returns (polynomials, primes used)."""
    V = m * n
    if V > 256:
        raise ValueError("m * n must be at most 256 (coefficient slots per state row)")
    d = V - 1
    pool = list(primes) if primes is not None else W.seeded_primes(max_primes, 1005)
    residues = []            # [prime][row][coefficient]
    used = []
    while True:
        group = pool[len(used):len(used) + batch]
        if not group:
            raise RuntimeError("the lift did not stabilise with the primes given")
        res = api.series(lattice, m, n, d, group, mode="graph")          # [n][len(group)][d + 1]
        for b in range(len(group)):
            residues.append([[int(v) for v in res[r, b]] for r in range(n)])
        used += group
        # stable: the lift over every prime so far equals the lift without
        # the last one, for every row
        out, stable = [], len(used) > 1
        for r in range(n):
            rows = [residues[b][r] for b in range(len(used))]
            coef, _ = host.series_exact(rows, used)
            if stable:
                prev, _ = host.series_exact(rows[:-1], used[:-1])
                stable = prev == coef
            Vr = m * (r + 1)
            p = [0] * (Vr + 1)
            for k2, c in enumerate(coef[:Vr]):
                p[Vr - k2] = c
            out.append(p)
        if stable:
            return out, len(used)


def main(argv=None) -> int:
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="Exact chromatic polynomials of the m x r rectangles, r = 1..n")
    ap.add_argument("lattice", choices=["square", "triangular"])
    ap.add_argument("m", type=int)
    ap.add_argument("n", type=int)
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("a GPU is required", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    polys, used = chromatic_polynomials(a.lattice, a.m, a.n)
    for r, p in enumerate(polys, start=1):
        terms = " + ".join(f"({c})*q^{j}" for j, c in enumerate(p) if c)
        print(f"{a.lattice} {a.m}x{r}: {terms}")
    print(f"{used} primes", file=sys.stderr)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
