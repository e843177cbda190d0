"""Oracle of the finite-lattice series (Sec. 4.1) -- test infrastructure only.

Plain, slow and exact (Python integers).  Follows the paper's definitions:

* B(k): the r x s rectangles with r <= s and r + s <= k (square lattice);
* the finite-lattice weights alpha_k(r,s), beta_k(r,s), gamma_k(r,s)
  (eqs. fb - fc and the weight formulas that follow them);
* the free energies as sums of weight x log P~_{G(r,s)}(z) in the variable
  z = 1/(q-1) (eq. def_z), correct to O(z^{2k-3}).

Every weight is an integer, so exponentiating gives products of integer
power series:
    exp(f_b) = q prod P~^{alpha},   exp(f_s) = prod P~^{beta},
    exp(f_c) = prod P~^{gamma},
and Table 1 lists the coefficients alpha_k of exp(f_b) = (q-1)^2/q *
sum alpha_k z^k, and those of exp(f_s) and exp(f_c).  With q = (1+z)/z,
q^2/(q-1)^2 = (1+z)^2, so sum alpha_k z^k = (1+z)^2 prod P~^{alpha}.

P~_{G(r,s)} (eq. Z_modified, a polynomial in x = 1/q with constant term 1)
comes from the oracle's transfer matrix in the normalised form
(transfer.projected_strip with transfer.ExactX); x = z/(1+z).
"""
from __future__ import annotations

from fractions import Fraction

from . import transfer as T


def rectangles(k: int) -> list[tuple[int, int]]:
    """B(k): (r, s) with 1 <= r <= s and r + s <= k."""
    return [(r, s) for r in range(1, k) for s in range(r, k - r + 1)]


def _delta(a: int, b: int) -> int:
    return 1 if a == b else 0


def alpha_weight(k: int, r: int, s: int) -> int:
    n = r + s
    return (2 - _delta(r, s)) * (_delta(n, k) - 3 * _delta(n, k - 1) + 3 * _delta(n, k - 2) - _delta(n, k - 3))


def beta_weight(k: int, r: int, s: int) -> int:
    """Surface weights.  The printed formula's last term reads (r+s-2)/2;
    the weights of this shape that extract the (r+s) part of
    rs f_b + (r+s) f_s + f_c (sum w = 0, sum w (r+s) = 1, sum w rs = 0 over
    B(k), the conditions the alpha weights meet for f_b) are unique and
    have (r+s+2)/2 there -- the reading taken here, which reproduces the
    beta column of Table 1."""
    n = r + s
    w = (Fraction(2 - n, 2) * _delta(n, k) + Fraction(3 * n - 2, 2) * _delta(n, k - 1)
         - Fraction(3 * n + 2, 2) * _delta(n, k - 2) + Fraction(n + 2, 2) * _delta(n, k - 3))
    w *= 2 - _delta(r, s)
    assert w.denominator == 1
    return int(w)


def gamma_weight(k: int, r: int, s: int) -> int:
    n = r + s
    return (2 - _delta(r, s)) * ((r - 1) * (s - 1) * _delta(n, k) + (1 + n - 3 * r * s) * _delta(n, k - 1)
                                 + (3 * r * s + n - 1) * _delta(n, k - 2) - (r + 1) * (s + 1) * _delta(n, k - 3))


# --------------------------------------------------------------------------
# Integer power series, truncated after z^N (lists of N + 1 coefficients)
# --------------------------------------------------------------------------
def ps_mul(a, b, N):
    out = [0] * (N + 1)
    for i, ai in enumerate(a[: N + 1]):
        if ai:
            for j, bj in enumerate(b[: N + 1 - i]):
                out[i + j] += ai * bj
    return out


def ps_inv(a, N):
    """1 / a for a[0] = 1."""
    assert a[0] == 1
    out = [0] * (N + 1)
    out[0] = 1
    for n in range(1, N + 1):
        out[n] = -sum(a[i] * out[n - i] for i in range(1, min(n, len(a) - 1) + 1))
    return out


def ps_pow(a, e: int, N):
    """a^e for an integer e (negative: powers of 1/a)."""
    base = ps_inv(a, N) if e < 0 else list(a[: N + 1]) + [0] * (N + 1 - len(a[: N + 1]))
    out = [1] + [0] * N
    for _ in range(abs(e)):
        out = ps_mul(out, base, N)
    return out


def x_to_z(px, N):
    """A polynomial in x = 1/q rewritten in z = 1/(q-1): x = z / (1 + z),
    so x^j = z^j (1+z)^-j = sum_i (-1)^i C(j+i-1, i) z^{j+i}."""
    out = [0] * (N + 1)
    for j, c in enumerate(px):
        if j > N or not c:
            continue
        binom = 1                                   # C(j+i-1, i) for i = 0
        for i in range(0, N - j + 1):
            if i > 0:
                binom = binom * (j + i - 1) // i
            out[j + i] += c * (-1) ** i * (binom if j > 0 else (1 if i == 0 else 0))
    return out


def ptilde_x(lattice: str, r: int, s_max: int, dmax: int) -> list[list[int]]:
    """P~ of the r x s rectangles, s = 1..s_max, as lists of coefficients of
    x^0 .. x^dmax (eq. Z_modified; oracle transfer matrix, normalised)."""
    res = T.projected_strip(lattice, r, s_max, T.ExactX(dmax=dmax))
    out = []
    for z in res:
        z = list(z)[: dmax + 1]
        out.append(z + [0] * (dmax + 1 - len(z)))
    return out


def square_series(k: int):
    """(alpha, beta, gamma) coefficient lists of Table 1's three series,
    from the rectangles of B(k), each to order z^{2k-4} (the orders the
    finite-lattice formulas fix)."""
    N = 2 * k - 4
    rects = rectangles(k)
    pz = {}
    for r in sorted({r for r, _ in rects}):
        s_max = max(s for rr, s in rects if rr == r)
        rows = ptilde_x(T.SQUARE, r, s_max, N)
        for s in range(r, s_max + 1):
            pz[(r, s)] = x_to_z(rows[s - 1], N)
    series = []
    for wfun, lead in ((alpha_weight, [1, 2, 1]), (beta_weight, [1]), (gamma_weight, [1])):
        acc = lead + [0] * (N + 1 - len(lead))
        for (r, s) in rects:
            e = wfun(k, r, s)
            if e:
                acc = ps_mul(acc, ps_pow(pz[(r, s)], e, N), N)
        series.append(acc)
    return tuple(series)
