"""Exact chromatic polynomials of rectangles from the GPU coefficient form.

P_G(q) of the m x r rectangles, r = 1..n, as integer coefficient lists
(q^0 .. q^|V|), without interpolation: the coefficient form gives the
normalised P~ = q^{-|V|} P (eq. Z_modified) as coefficients of x^0..x^d mod
each prime, and with d = |V| - 1 (the constant term of P is 0) the whole
polynomial is known mod p: the coefficient of q^{|V| - k} in P is that of
x^k in P~.  Primes are added until the CRT lift stops changing (Sec. 3.5) and
their product exceeds twice the largest coefficient any of the polynomials
can have (Whitney's broken-circuit theorem bounds |c_{|V|-k}| by C(|E|, k)),
so the symmetric lift is exact, not only stable.

    python -m paper_1005_3609_amd.polynomial square 6 7
"""
from __future__ import annotations

from math import comb

from . import api, host, tune
from . import workloads as W


def graph_counts(lattice, m: int, n: int):
    """(|V|, |E|, triangles, 4-cycles) of the m x n rectangle: the square
    lattice's edges plus, on the triangular lattice, one diagonal per face
    (Sec. 3.3).  Every 4-cycle of the square lattice is a face; the
    triangular lattice's are not counted (None)."""
    faces = max(m - 1, 0) * max(n - 1, 0)
    e = m * (n - 1) + n * (m - 1)
    if lattice == "square":
        return m * n, e, 0, faces
    return m * n, e + faces, 2 * faces, None


def check(lattice, m: int, n: int, c) -> list:
    """Properties every chromatic polynomial P = sum c_j q^j of the m x n
    rectangle has; returns the ones that fail (empty: all hold).

    * degree |V|, monic; c_{|V|-1} = -|E|; c_{|V|-2} = C(|E|, 2) - (triangles);
      on the square lattice (no triangles, every 4-cycle a face, no two faces
      sharing two edges) c_{|V|-3} = -(C(|E|, 3) - faces) and c_{|V|-4} =
      C(|E|, 4) - (faces)(|E| - 3) -- Whitney's broken-circuit expansion;
    * P(0) = P(1) = 0 (at least one edge), and for a connected graph the
      coefficients of q^1..q^|V| are non-zero with alternating signs;
    * the absolute values |c_1|..|c_|V|| are log-concave (Huh);
    * square: P(2) = 2 (connected, bipartite); triangular with m, n >= 2:
      P(2) = 0 and P(3) = 6 (the faces' triangles force a 3-colouring)."""
    V, E, T, F = graph_counts(lattice, m, n)
    bad = []
    c = list(c) + [0] * max(0, V + 1 - len(c))
    if any(c[V + 1:]) or c[V] != 1:
        bad.append("not monic of degree |V|")
    if V >= 2 and c[V - 1] != -E:
        bad.append("c_{|V|-1} != -|E|")
    if V >= 3 and c[V - 2] != comb(E, 2) - T:
        bad.append("c_{|V|-2} != C(|E|,2) - triangles")
    if lattice == "square" and V >= 4 and c[V - 3] != -(comb(E, 3) - F):
        bad.append("c_{|V|-3} != -(C(|E|,3) - faces)")
    if lattice == "square" and V >= 5 and c[V - 4] != comb(E, 4) - F * (E - 3):
        bad.append("c_{|V|-4} != C(|E|,4) - faces (|E| - 3)")
    ev = lambda q: sum(cj * q ** j for j, cj in enumerate(c))
    if c[0] != 0:
        bad.append("P(0) != 0")
    if E and ev(1) != 0:
        bad.append("P(1) != 0")
    if any(c[j] == 0 or (c[j] > 0) != ((V - j) % 2 == 0) for j in range(1, V + 1)):
        bad.append("coefficients of q^1..q^|V| not alternating and non-zero")
    a = [abs(x) for x in c[1:V + 1]]
    if any(a[j] * a[j] < a[j - 1] * a[j + 1] for j in range(1, len(a) - 1)):
        bad.append("|c_j| not log-concave")
    if lattice == "square" and V >= 2 and ev(2) != 2:
        bad.append("P(2) != 2")
    if lattice == "triangular" and m >= 2 and n >= 2 and (ev(2) != 0 or ev(3) != 6):
        bad.append("P(2) != 0 or P(3) != 6")
    return bad


def coefficient_bound(lattice, m: int, n: int) -> int:
    """An upper bound on |c_j| for the chromatic polynomial of the m x n
    rectangle: c_{|V|-k} counts the k-edge subsets with no broken circuit
    (Whitney), at most C(|E|, k), and k runs over 0..|V|-1 (c_0 = 0)."""
    V, E, _, _ = graph_counts(lattice, m, n)
    return max(comb(E, k) for k in range(0, max(min(E, V - 1), 0) + 1))


def primes_per_call(one_prime_bytes: int, free_bytes: int, most: int = 8) -> int:
    """Primes per coefficient-form call: as many as fit in 80 % of the free
    device memory (one prime's workspace each), between 1 and `most`."""
    return max(1, min(most, int(0.8 * free_bytes) // max(one_prime_bytes, 1)))


def chromatic_polynomials(lattice, m: int, n: int, primes=None, batch: int = 0, max_primes: int = 64,
                          log=None):
    """[P_{m x r}(q) for r = 1..n], each a list of integers c_0..c_{|V|}
    with P = sum c_j q^j.  Needs m n <= 512 (coefficients x^0..x^{mn-1} in
    at most 8 slots per wavefront lane).  Primes are drawn in groups of
    `batch` (0: one for 512-slot rows, else as many as the free device
    memory holds, at most 8) from
    `primes` (default: seeded 31-bit primes) until every row's
    lift is stable and the product of the primes exceeds twice
    `coefficient_bound` of the largest rectangle; returns (polynomials,
    primes used).  Raises if a coefficient past a row's degree lifts to a
    non-zero value.  `log(text)`, if
    given, hears of every finished prime group."""
    V = m * n
    if V > 512:
        raise ValueError("m * n must be at most 512 (coefficient slots per state row)")
    d = V - 1
    lanes_v = tune.series_lanes_v(d)
    shape = dict(tune.SERIES_WIDE_DEFAULT if lanes_v == 8 else tune.SERIES_DEFAULT, lanes_v=lanes_v)
    if batch <= 0 and lanes_v == 8:
        batch = 1        # 512-slot rows: two primes per call ran 1.3x slower per prime (triangular 20 x 21)
    elif batch <= 0:
        import torch
        free, _ = torch.cuda.mem_get_info()
        batch = primes_per_call(api.series_workspace_bytes(lattice, m, n, 1, d, "graph", shape), free)
    pool = list(primes) if primes is not None else W.seeded_primes(max_primes, 1005)
    residues = []            # [prime][row][coefficient]
    used = []
    need = 2 * coefficient_bound(lattice, m, n)
    modulus = 1
    while True:
        group = pool[len(used):len(used) + batch]
        if not group:
            raise RuntimeError("the lift did not stabilise with the primes given")
        res = api.series(lattice, m, n, d, group, mode="graph", tuning=shape)   # [n][len(group)][d + 1]
        for b in range(len(group)):
            residues.append([[int(v) for v in res[r, b]] for r in range(n)])
        used += group
        for p_ in group:
            modulus *= p_
        if log:
            log(f"{lattice} {m}x{n}: {len(used)} primes done")
        # stable: the lift over every prime so far equals the lift without
        # the last one, for every row
        out, stable = [], len(used) > 1 and modulus > need
        for r in range(n):
            rows = [residues[b][r] for b in range(len(used))]
            coef, _ = host.series_exact(rows, used)
            if stable:
                prev, _ = host.series_exact(rows[:-1], used[:-1])
                stable = prev == coef
            Vr = m * (r + 1)
            if stable and any(coef[Vr:]):
                raise RuntimeError(f"{lattice} {m}x{r + 1}: a coefficient past x^{Vr - 1} lifted to a non-zero value")
            p = [0] * (Vr + 1)
            for k2, c in enumerate(coef[:Vr]):
                p[Vr - k2] = c
            out.append(p)
        if stable:
            return out, len(used)


def evaluate(c, q: int) -> int:
    """P(q) for P = sum c_j q^j."""
    v = 0
    for cj in reversed(c):
        v = v * q + cj
    return v


def read_values(path, lattice, m: int, n: int):
    """[(r, q, P(q))] from lines 'lattice m r q value' of `path` for the
    given lattice and width and r <= n ('#' starts a comment line)."""
    out = []
    with open(path) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            lat, mm, r, q, v = ln.split()
            if lat == lattice and int(mm) == m and int(r) <= n:
                out.append((int(r), int(q), int(v)))
    return out


def main(argv=None) -> int:
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="Exact chromatic polynomials of the m x r rectangles, r = 1..n")
    ap.add_argument("lattice", choices=["square", "triangular"])
    ap.add_argument("m", type=int)
    ap.add_argument("n", type=int)
    ap.add_argument("--batch", type=int, default=0,
                    help="primes per coefficient-form call (0: one for |V| > 256, else as many as fit in device "
                         "memory, at most 8)")
    ap.add_argument("--max-primes", type=int, default=64)
    ap.add_argument("--transposed", type=int, default=0, metavar="K",
                    help="also compute P of the r x m rectangles, r = 1..K, by strips of width r, and compare "
                         "(P is symmetric under transposition)")
    ap.add_argument("--values", metavar="FILE",
                    help="file of 'lattice m r q value' lines: P(q) of each listed m x r rectangle must equal value")
    ap.add_argument("--out", help="write the polynomials here instead of standard output")
    a = ap.parse_args(argv)
    import time
    import torch
    if not torch.cuda.is_available():
        print("a GPU is required", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    t0 = time.time()
    say = lambda text: print(f"[{time.time() - t0:7.1f} s] {text}", file=sys.stderr, flush=True)
    polys, used = chromatic_polynomials(a.lattice, a.m, a.n, batch=a.batch, max_primes=a.max_primes, log=say)
    say(f"{a.lattice} {a.m}x1..{a.n}: {used} primes")
    rc = 0
    for r, p in enumerate(polys, start=1):
        bad = check(a.lattice, a.m, r, p)
        if bad:
            rc = 1
            say(f"{a.m}x{r}: FAILED " + "; ".join(bad))
    say(f"properties of all {a.n} polynomials: " + ("FAILED" if rc else "hold"))
    if a.values:
        want = read_values(a.values, a.lattice, a.m, a.n)
        bad = [(r, q) for r, q, v in want if evaluate(polys[r - 1], q) != v]
        rc = rc or (1 if bad or not want else 0)
        say(f"values from {a.values}: {len(want) - len(bad)} of {len(want)} equal"
            + (f"; DIFFERENT at (r, q) = {bad}" if bad else ""))
    for r in range(1, min(a.transposed, a.n) + 1):
        tp, _ = chromatic_polynomials(a.lattice, r, a.m, max_primes=a.max_primes)
        same = tp[-1] == polys[r - 1]
        rc = rc or (0 if same else 1)
        say(f"{a.m}x{r} against {r}x{a.m} by width-{r} strips: " + ("equal" if same else "DIFFERENT"))
    lines = []
    for r, p in enumerate(polys, start=1):
        terms = " + ".join(f"({c})*q^{j}" for j, c in enumerate(p) if c)
        lines.append(f"{a.lattice} {a.m}x{r}: {terms}")
    if a.out:
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")
    else:
        print("\n".join(lines))
    return rc


if __name__ == "__main__":
    raise SystemExit(main())
