"""Finite-lattice series of the chromatic polynomial (Sec. 4.1, 4.2, 4.4),
from the coefficient form computed on the GPU.

The free energies are combinations, with integer finite-lattice weights, of
log P~_{G(r,s)}(z) over the rectangles of B(k) = {r <= s, r + s <= k}, in
z = 1/(q-1), correct to O(z^{2k-3}).  Exponentiated they are products of
powers of power series with constant term 1:
    A(z) = (1+z)^2 prod P~^{alpha_k(r,s)}   (Table 1: exp f_b = (q-1)^2/q A)
    B(z) = prod P~^{beta_k(r,s)}             (exp f_s)
    C(z) = prod P~^{gamma_k(r,s)}            (exp f_c)
Only ring operations occur (products, inverses of series with constant term
1), so every prime is combined on its own, straight from the GPU residues
of P~ (no lift of P~ itself, whose coefficients are far larger), and only
the final coefficients are lifted by CRT; primes are added until they stop
changing (Sec. 3.5).

Surface weights: the last term of the printed beta_k(r,s) reads
(r+s-2)/2; the one weight of that shape that extracts the (r+s) part of
rs f_b + (r+s) f_s + f_c has (r+s+2)/2, which is used here.

The triangular lattice takes the same weights (Sec. 4.4) with the series in
Baxter's variable x, q = 2 - x - 1/x (so 1/q = -x/(1-x)^2), correct to
x^{k-1}; its bulk series is (1-x)^2 prod P~^alpha = -x exp(f_b).
"""
from __future__ import annotations

from . import api, host
from . import tune as tuner

SQUARE = "square"
TRIANGULAR = "triangular"


def rectangles(k: int):
    """B(k) as (r, s) pairs, r <= s, r + s <= k."""
    out = []
    for r in range(1, k // 2 + 1):
        for s in range(r, k - r + 1):
            out.append((r, s))
    return out


def weights(k: int, r: int, s: int) -> tuple[int, int, int]:
    """(alpha_k, beta_k, gamma_k)(r, s): finite-lattice weights for the bulk,
    surface and corner free energies (integers; zero unless k-3 <= r+s <= k)."""
    j = k - (r + s)
    if j < 0 or j > 3:
        return 0, 0, 0
    n, rs = r + s, r * s
    mult = 1 if r == s else 2
    a = (1, -3, 3, -1)[j]
    twice_b = (2 - n, 3 * n - 2, -(3 * n + 2), n + 2)[j]
    c = ((r - 1) * (s - 1), 1 + n - 3 * rs, 3 * rs + n - 1, -(r + 1) * (s + 1))[j]
    b = mult * twice_b
    assert b % 2 == 0
    return mult * a, b // 2, mult * c


# ---------------------------------------------------------------------------
# Power series mod p, truncated after z^N (lists of N + 1 residues)
# ---------------------------------------------------------------------------
def _mul(a, b, N, p):
    """a b mod p by one big-integer product (Kronecker substitution: the
    coefficients become digits of 2^bits-ary numbers wide enough for the
    exact convolution sums)."""
    bits = 2 * p.bit_length() + (N + 1).bit_length() + 1
    A = int.from_bytes(b"".join(int(x).to_bytes((bits + 7) // 8, "little") for x in a[: N + 1]), "little")
    B = int.from_bytes(b"".join(int(x).to_bytes((bits + 7) // 8, "little") for x in b[: N + 1]), "little")
    step = 8 * ((bits + 7) // 8)
    prod = A * B
    mask = (1 << step) - 1
    out = []
    for _ in range(N + 1):
        out.append((prod & mask) % p)
        prod >>= step
    return out


def _inv(a, N, p):
    """1 / a mod p for a[0] = 1 (coefficient recurrence)."""
    out = [1] + [0] * N
    for n in range(1, N + 1):
        acc = 0
        for i in range(1, min(n, len(a) - 1) + 1):
            acc += a[i] * out[n - i]
        out[n] = (-acc) % p
    return out


def _pow(a, e: int, N, p):
    base = _inv(a, N, p) if e < 0 else [x % p for x in a[: N + 1]]
    e = abs(e)
    out = [1] + [0] * N
    while e:
        if e & 1:
            out = _mul(out, base, N, p)
        e >>= 1
        if e:
            base = _mul(base, base, N, p)
    return out


def _in_z(px, N, p):
    """P~(x) with x = z/(1+z), by Horner's rule on series mod p."""
    X = [0] + [(1 if i % 2 else p - 1) for i in range(1, N + 1)]   # z - z^2 + z^3 - ...
    acc = [0] * (N + 1)
    for j in range(min(len(px), N + 1) - 1, -1, -1):
        acc = _mul(acc, X, N, p)
        acc[0] = (acc[0] + int(px[j])) % p
    return acc


def _in_baxter_x(pu, N, p):
    """P~(u), u = 1/q, with q = 2 - x - 1/x, i.e. u = -x/(1-x)^2 =
    -(x + 2x^2 + 3x^3 + ...), by Horner's rule on series mod p."""
    U = [0] + [(-i) % p for i in range(1, N + 1)]
    acc = [0] * (N + 1)
    for j in range(min(len(pu), N + 1) - 1, -1, -1):
        acc = _mul(acc, U, N, p)
        acc[0] = (acc[0] + int(pu[j])) % p
    return acc


def polygon_mu(p_max: int) -> list[int]:
    """mu_0 .. mu_{p_max} of the generating function sum_{p>=4} mu_p x^{2p}
    quoted in Sec. 4.2, by coefficient recurrences in y = x^2: the two terms
    y^4 (2 - 2y - y S) / ((1 - 4y)(2 + y)) and y^6 (3 - 4y - 4S) / (1 - 4y)^2
    with S = sqrt(1 - 4y), whose coefficients are -2 C(2j-2, j-1)/j for
    j >= 1.  Division by (1 - 4y) is u_j = a_j + 4 u_{j-1}, by (2 + y) is
    v_j = (u_j - v_{j-1}) / 2."""
    from fractions import Fraction
    from math import comb

    n = max(p_max, 0)
    S = [1] + [-2 * comb(2 * j - 2, j - 1) // j for j in range(1, n + 1)]

    def over_1m4y(a):
        out, prev = [], 0
        for x in a:
            prev = x + 4 * prev
            out.append(prev)
        return out

    num1 = [(2 if j == 0 else 0) - (2 if j == 1 else 0) - (S[j - 1] if j >= 1 else 0) for j in range(n + 1)]
    u = over_1m4y(num1)
    v, prev = [], Fraction(0)
    for x in u:
        prev = (x - prev) / 2
        v.append(prev)
    num2 = [(3 if j == 0 else 0) - (4 if j == 1 else 0) - 4 * S[j] for j in range(n + 1)]
    w = over_1m4y(over_1m4y(num2))
    mu = []
    for q in range(n + 1):
        c = (v[q - 4] if q >= 4 else 0) + (w[q - 6] if q >= 6 else 0)
        if Fraction(c).denominator != 1:
            raise ArithmeticError("non-integer polygon coefficient")
        mu.append(int(c))
    return mu[: p_max + 1]


def default_order(lattice, k: int) -> int:
    """Highest order the finite-lattice formulas fix: z^{2k-4} on the square
    lattice, x^{k-1} on the triangular one."""
    return 2 * k - 4 if lattice == SQUARE else k - 1


def combine_mod(ptilde, k: int, p: int, N: int | None = None, lattice=SQUARE):
    """(A, B, C) mod p from P~_{r,s}(1/q) mod p, ptilde[(r, s)] = coefficient
    list of (1/q)^0 .. (at least) (1/q)^N.  Square: series in z = 1/(q-1),
    A = (1+z)^2 prod P~^alpha.  Triangular: series in Baxter's x,
    A = (1-x)^2 prod P~^alpha.  B, C = prod P~^beta, prod P~^gamma.  N
    defaults to default_order(lattice, k)."""
    if N is None:
        N = default_order(lattice, k)
    lead, subst = ([1, 2, 1], _in_z) if lattice == SQUARE else ([1, p - 2, 1], _in_baxter_x)
    A = (lead + [0] * (N + 1))[: N + 1]
    B = [1] + [0] * N
    C = [1] + [0] * N
    for (r, s) in rectangles(k):
        wa, wb, wc = weights(k, r, s)
        if not (wa or wb or wc):
            continue
        pz = subst(ptilde[(r, s)], N, p)
        if wa:
            A = _mul(A, _pow(pz, wa, N, p), N, p)
        if wb:
            B = _mul(B, _pow(pz, wb, N, p), N, p)
        if wc:
            C = _mul(C, _pow(pz, wc, N, p), N, p)
    return A, B, C


def prime_groups(r: int, n: int, N: int, primes, mode: str, tuning, limit: int, lattice=SQUARE):
    """Splits the primes into consecutive groups whose strip workspace
    (series_workspace_bytes, which grows linearly with the group size)
    stays within `limit` bytes; one prime per group at the least."""
    one = api.series_workspace_bytes(lattice, r, n, 1, N, mode, tuning)
    per = max(1, min(len(primes), limit // max(one, 1)))
    return [list(primes[i:i + per]) for i in range(0, len(primes), per)]


def _strips(lattice, k: int, N: int, primes, mode, tuning, lanes_v, workspace_limit, log):
    """P~ residues of every rectangle of B(k): one coefficient-form strip per
    width r = 1..k/2 (rows 1..k-r, coefficients to N), all primes at once or
    in groups that keep the workspace within workspace_limit.  Returns one
    dict {(r, s): coefficients} per prime."""
    if lanes_v is None:
        lanes_v = 1 if N < 64 else (2 if N < 128 else 4)
    t = dict(tuning) if tuning else dict(tuner.SERIES_DEFAULT)
    t["lanes_v"] = lanes_v
    per_prime = [dict() for _ in primes]
    for r in range(1, k // 2 + 1):
        n = k - r
        b0 = 0
        for group in prime_groups(r, n, N, primes, mode, t, workspace_limit, lattice):
            res = api.series(lattice, r, n, N, group, mode=mode, tuning=t)   # [n][len(group)][N+1]
            for s in range(r, n + 1):
                for b in range(len(group)):
                    per_prime[b0 + b][(r, s)] = [int(v) for v in res[s - 1, b]]
            b0 += len(group)
            if log is not None:
                log(f"width {r}: rows 1..{n}, {len(group)} prime(s) done")
    return per_prime


def _lift(mods, primes, N):
    """CRT of the three series coefficient by coefficient over the first u
    primes, u = 1, 2, ...; stops when two successive lifts agree.  Returns
    (series, primes_used, stable)."""
    prev = None
    for u in range(1, len(primes) + 1):
        cur = []
        for which in range(3):
            col = []
            for i in range(N + 1):
                x, M = host.crt([mods[b][which][i] for b in range(u)], primes[:u])
                col.append(host.symmetric(x, M))
            cur.append(col)
        if cur == prev:
            return cur, u, True
        prev = cur
    return prev, len(primes), False


def square_series(k: int, primes, mode: str = "graph", tuning=None, lanes_v: int | None = None,
                  workspace_limit: int = 96 << 30, log=None, extra: bool = False):
    """Table 1's series A, B, C to z^{2k-4} from the GPU coefficient form.

    Runs one coefficient-form strip per width r = 1..k/2 (rows up to k - r,
    d_max = 2k - 4), all primes at once or, where the workspace would pass
    `workspace_limit` bytes, in groups of primes; combines every prime, and
    lifts the final coefficients by CRT, adding primes until two successive
    lifts agree.  `log(msg)`, if given, is called once per strip.

    extra (odd k): A and B one order further, to z^{2k-3} = z^{4 m_max - 1}
    (m_max = (k-1)/2, the widest strip): the strips and products run to that
    order and the missing polygon term of Sec. 4.2 is added, mu_{2 m_max} to
    A's and -m_max mu_{2 m_max} to B's last coefficient (their logarithms
    gain those terms and both series start with 1); C stays at z^{2k-4}.

    Returns dict(alpha, beta, gamma, primes_used, stable)."""
    if extra and k % 2 == 0:
        raise ValueError("the extra order needs odd k (4 m_max - 1 = 2k - 3)")
    N = 2 * k - 4 + (1 if extra else 0)
    per_prime = _strips(SQUARE, k, N, primes, mode, tuning, lanes_v, workspace_limit, log)
    mods = [list(combine_mod(per_prime[b], k, int(p), N)) for b, p in enumerate(primes)]
    if extra:
        m_max = (k - 1) // 2
        mu = polygon_mu(2 * m_max)[2 * m_max]
        for b, p in enumerate(primes):
            p = int(p)
            mods[b][0][N] = (mods[b][0][N] + mu) % p
            mods[b][1][N] = (mods[b][1][N] - m_max * mu) % p
    out, used, stable = _lift(mods, primes, N)
    gamma = out[2][: 2 * k - 3]
    return {"alpha": out[0], "beta": out[1], "gamma": gamma, "primes_used": used, "stable": stable}


def triangular_series(k: int, primes, mode: str = "graph", tuning=None, lanes_v: int | None = None,
                      workspace_limit: int = 96 << 30, log=None):
    """The triangular-lattice series of Sec. 4.4 to x^{k-1} (Baxter's x,
    q = 2 - x - 1/x) from the GPU coefficient form: strips of widths
    1..k/2 with rows 1..k-r and coefficients to (1/q)^{k-1}, the square
    lattice's weights, per-prime combination and CRT as in square_series.
    Returns dict(bulk, surface, corner, primes_used, stable): bulk =
    (1-x)^2 prod P~^alpha = -x exp(f_b), surface = exp(f_s), corner =
    exp(f_c)."""
    N = k - 1
    per_prime = _strips(TRIANGULAR, k, N, primes, mode, tuning, lanes_v, workspace_limit, log)
    mods = [combine_mod(per_prime[b], k, int(p), N, TRIANGULAR) for b, p in enumerate(primes)]
    out, used, stable = _lift(mods, primes, N)
    return {"bulk": out[0], "surface": out[1], "corner": out[2], "primes_used": used, "stable": stable}


def baxter_bulk(N: int) -> list[int]:
    """-x exp(f_b) of the triangular lattice from Baxter's product (Sec. 4.4,
    eq. efb) to x^N: prod over j >= 1 of (1-x^{6j-3})(1-x^{6j-2})^2(1-x^{6j-1})
    divided by (1-x^{6j-5})(1-x^{6j-4})(1-x^{6j})(1-x^{6j+1}); exact
    integers (each factor 1/(1 - x^e) is a geometric series)."""
    out = [1] + [0] * N

    def times(e, sign):
        nonlocal out
        if e > N:
            return
        if sign > 0:               # multiply by (1 - x^e)
            out = [out[i] - (out[i - e] if i >= e else 0) for i in range(N + 1)]
        else:                      # divide by (1 - x^e): running sums with stride e
            for i in range(e, N + 1):
                out[i] += out[i - e]

    for j in range(1, N // 6 + 2):
        for e in (6 * j - 3, 6 * j - 2, 6 * j - 2, 6 * j - 1):
            times(e, +1)
        for e in (6 * j - 5, 6 * j - 4, 6 * j, 6 * j + 1):
            times(e, -1)
    return out


def _read_table(path):
    """k -> tuple of ints (None for '-') from a whitespace table whose first
    column is k ('#' comment lines)."""
    tab = {}
    with open(path) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, *vals = ln.split()
                tab[int(k)] = tuple(None if x == "-" else int(x) for x in vals)
    return tab


def main(argv=None) -> int:
    import argparse
    import sys
    import time

    import numpy as np

    from . import workloads as W

    ap = argparse.ArgumentParser(description="Bulk, surface and corner series by the finite-lattice method on the "
                                             "GPU: square lattice to z^(2k-4) in z = 1/(q-1), triangular to "
                                             "x^(k-1) in q = 2 - x - 1/x")
    ap.add_argument("k", type=int)
    ap.add_argument("--lattice", default=SQUARE, choices=[SQUARE, TRIANGULAR])
    ap.add_argument("--primes", type=int, default=5, help="number of seeded 31-bit primes")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--mode", default="graph", choices=["graph", "batched"])
    ap.add_argument("--workspace-gib", type=int, default=96, help="largest strip workspace per call")
    ap.add_argument("--check", default=None,
                    help="table to compare with: columns k alpha beta gamma (square) or k surface corner "
                         "(triangular)")
    ap.add_argument("--extra", action="store_true", help="square, odd k: alpha and beta to z^(2k-3) (polygon term)")
    ap.add_argument("--baxter", action="store_true", help="triangular: compare the bulk with Baxter's product")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("a GPU is required", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    kw = dict(mode=a.mode, workspace_limit=a.workspace_gib << 30,
              log=lambda msg: print(f"[{time.perf_counter() - t0:7.1f} s] {msg}", flush=True))
    primes = W.seeded_primes(a.primes, a.seed)
    if a.lattice == SQUARE:
        res = square_series(a.k, primes, extra=a.extra, **kw)
        names, checked, var = ("alpha", "beta", "gamma"), ("alpha", "beta", "gamma"), "z"
    else:
        res = triangular_series(a.k, primes, **kw)
        names, checked, var = ("bulk", "surface", "corner"), ("surface", "corner"), "x"
    dt = time.perf_counter() - t0
    N = len(res[names[0]]) - 1
    for i in range(N + 1):
        print(i, *(res[n][i] if i < len(res[n]) else "-" for n in names))
    ok = True
    if a.check:
        tab = _read_table(a.check)
        cells = [(i, j) for i in range(N + 1) for j in range(len(checked)) if i < len(res[checked[j]])]
        bad = [(i, j) for i, j in cells if i not in tab or tab[i][j] is None or res[checked[j]][i] != tab[i][j]]
        ok = not bad
        print(f"check against {a.check}: {f'all {len(cells)} coefficients equal' if ok else bad[:10]}")
    if a.baxter and a.lattice == TRIANGULAR:
        same = res["bulk"] == baxter_bulk(N)
        ok = ok and same
        print(f"bulk against Baxter's product to x^{N}: {'equal' if same else 'DIFFERENT'}")
    print(f"{a.lattice} k = {a.k}: {var}^0..{var}^{N}, widths 1..{a.k // 2}, {res['primes_used']} of {a.primes} "
          f"primes to stabilise ({'stable' if res['stable'] else 'NOT stable'}), {dt:.1f} s; "
          f"torch {torch.__version__}, numpy {np.__version__}", flush=True)
    return 0 if (ok and res["stable"]) else 1


if __name__ == "__main__":
    raise SystemExit(main())
