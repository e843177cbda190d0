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

The triangular lattice takes the same weights (Sec. 4.4) with the series
written in Baxter's variable x, q = 2 - x - 1/x, to x^{k-1}.

P~_{G(r,s)} (eq. Z_modified, a polynomial in x = 1/q with constant term 1)
comes from the oracle's transfer matrix in the normalised form
(transfer.projected_strip with transfer.ExactX); x = z/(1+z).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

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


def inverse_q_to_baxter_x(pu, N):
    """A polynomial in u = 1/q rewritten in the variable x of Sec. 4.4,
    q = 2 - x - 1/x = -(1-x)^2/x, so u = -x (1-x)^{-2} and
    u^j = (-1)^j x^j (1-x)^{-2j} = (-1)^j sum_i C(2j+i-1, i) x^{j+i}."""
    out = [0] * (N + 1)
    for j, c in enumerate(pu):
        if j > N or not c:
            continue
        for i in range(0, N - j + 1):
            binom = comb(2 * j + i - 1, i) if j > 0 else (1 if i == 0 else 0)
            out[j + i] += c * (-1) ** j * binom
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


def mu_coefficients(n: int) -> list[Fraction]:
    """mu_0 .. mu_n of the polygon generating function quoted in Sec. 4.2
    (sum over p >= 4 of mu_p x^{2p}), as exact series in y = x^2:
        y^4 (2 - 2y - y S) / ((1 - 4y)(2 + y)) + y^6 (3 - 4y - 4S) / (1 - 4y)^2,
    S = sqrt(1 - 4y) = 1 - 2 sum_{j>=1} Cat(j-1) y^j (Catalan numbers)."""
    def mul(a, b):
        out = [Fraction(0)] * (n + 1)
        for i, x in enumerate(a[: n + 1]):
            if x:
                for j, y in enumerate(b[: n + 1 - i]):
                    out[i + j] += x * y
        return out

    def inv(a):
        out = [Fraction(0)] * (n + 1)
        out[0] = 1 / Fraction(a[0])
        for t in range(1, n + 1):
            out[t] = -sum(a[i] * out[t - i] for i in range(1, min(t, len(a) - 1) + 1)) / a[0]
        return out

    def catalan(j):
        c = 1
        for i in range(j):
            c = c * 2 * (2 * i + 1) // (i + 2)
        return c

    def shifted(a, e):
        return [Fraction(0)] * e + a[: n + 1 - e]

    pad = [Fraction(0)] * (n + 1)
    S = [Fraction(1)] + [Fraction(-2 * catalan(j - 1)) for j in range(1, n + 1)]
    one_m4y = ([Fraction(1), Fraction(-4)] + pad)[: n + 1]
    num1 = ([Fraction(2), Fraction(-2)] + pad)[: n + 1]
    num1 = [a - b for a, b in zip(num1, shifted(S, 1))]
    den1 = mul(one_m4y, ([Fraction(2), Fraction(1)] + pad)[: n + 1])
    num2 = ([Fraction(3), Fraction(-4)] + pad)[: n + 1]
    num2 = [a - 4 * b for a, b in zip(num2, S)]
    den2 = mul(one_m4y, one_m4y)
    t1 = shifted(mul(num1, inv(den1)), 4)
    t2 = shifted(mul(num2, inv(den2)), 6)
    return [a + b for a, b in zip(t1, t2)]


def square_series(k: int, extra: bool = False):
    """(alpha, beta, gamma) coefficient lists of Table 1's three series,
    from the rectangles of B(k), each to order z^{2k-4} (the orders the
    finite-lattice formulas fix).

    extra (odd k only): alpha and beta one order further, to z^{2k-3}: the
    finite-lattice products are taken to that order and the missing polygon
    term of Sec. 4.2 is added to the logarithms, mu_{2 m_max} z^{4 m_max - 1}
    to f_b and -m_max mu_{2 m_max} z^{4 m_max - 1} to f_s, with m_max =
    (k - 1)/2 the widest strip (so 4 m_max - 1 = 2k - 3).  As the series start
    with 1, adding c z^N to the logarithm adds c z^N to the series mod
    z^{N+1}.  gamma stays at z^{2k-4}."""
    if extra and k % 2 == 0:
        raise ValueError("the extra order needs odd k (4 m_max - 1 = 2k - 3)")
    N = 2 * k - 4 + (1 if extra else 0)
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
    if extra:
        m_max = (k - 1) // 2
        mu = mu_coefficients(2 * m_max)[2 * m_max]
        assert mu.denominator == 1
        series[0][N] += int(mu)
        series[1][N] -= m_max * int(mu)
        series[2] = series[2][:N]
    return tuple(series)


def triangular_series(k: int):
    """(bulk, surface, corner) series of the triangular lattice in Baxter's
    variable x (q = 2 - x - 1/x, Sec. 4.4), to x^{k-1}: the same
    finite-lattice weights over B(k), error O(z^k) = O(x^k) there.
        bulk    = (1-x)^2 prod P~^alpha   (exp f_b = q prod P~^alpha = -(1/x) bulk)
        surface = prod P~^beta            (exp f_s)
        corner  = prod P~^gamma           (exp f_c)"""
    N = k - 1
    rects = rectangles(k)
    px = {}
    for r in sorted({r for r, _ in rects}):
        s_max = max(s for rr, s in rects if rr == r)
        rows = ptilde_x(T.TRIANGULAR, r, s_max, N)
        for s in range(r, s_max + 1):
            px[(r, s)] = inverse_q_to_baxter_x(rows[s - 1], N)
    series = []
    for wfun, lead in ((alpha_weight, [1, -2, 1]), (beta_weight, [1]), (gamma_weight, [1])):
        acc = (lead + [0] * (N + 1))[: N + 1]
        for (r, s) in rects:
            e = wfun(k, r, s)
            if e:
                acc = ps_mul(acc, ps_pow(px[(r, s)], e, N), N)
        series.append(acc)
    return tuple(series)
