"""Pins of the oracle's finite-lattice series (Sec. 4.1) against what the
paper fixes: the coefficients Table 1 prints for the square lattice, and
the identities the finite-lattice weights must satisfy (each weight set
extracts exactly its own term of rs f_b + (r+s) f_s + f_c)."""
import os

import pytest

from oracle import series as S
from oracle import transfer as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table1():
    """tests/golden/table1_square.txt: the paper's Table 1 (k, alpha, beta, gamma)."""
    rows = {}
    with open(os.path.join(GOLDEN, "table1_square.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, a, b, c = ln.split()
            rows[int(k)] = (int(a), int(b), None if c == "-" else int(c))
    return rows


def test_table1_fixture_is_whole():
    t = table1()
    assert sorted(t) == list(range(80))
    assert t[0] == (1, 1, 1) and t[8] == (3, -8, 12) and t[79][2] is None


@pytest.mark.parametrize("k", [5, 8, 11])
def test_series_reproduce_table1(k):
    t = table1()
    N = 2 * k - 4
    al, be, ga = S.square_series(k)
    assert al == [t[i][0] for i in range(N + 1)]
    assert be == [t[i][1] for i in range(N + 1)]
    assert ga == [t[i][2] for i in range(N + 1)]


@pytest.mark.parametrize("k", [5, 7, 9, 11])
def test_extra_order_reproduces_table1(k):
    # one order past the finite-lattice truncation, alpha and beta only
    t = table1()
    N = 2 * k - 3
    al, be, ga = S.square_series(k, extra=True)
    assert len(al) == len(be) == N + 1 and len(ga) == N
    assert al == [t[i][0] for i in range(N + 1)]
    assert be == [t[i][1] for i in range(N + 1)]
    assert ga == [t[i][2] for i in range(N)]


def test_extra_order_needs_the_polygon_term():
    # without the mu term the z^{2k-3} coefficients are those of the plain
    # products (planted mistake: the correction dropped)
    k = 9
    mu = S.mu_coefficients(k - 1)
    assert all(x.denominator == 1 for x in mu) and mu[:4] == [0, 0, 0, 0] and mu[4] == 1
    al, be, _ = S.square_series(k, extra=True)
    t = table1()
    assert al[-1] - int(mu[k - 1]) != t[2 * k - 3][0]
    assert be[-1] + (k - 1) // 2 * int(mu[k - 1]) != t[2 * k - 3][1]
    with pytest.raises(ValueError):
        S.square_series(8, extra=True)


@pytest.mark.parametrize("k", range(4, 26))
def test_weights_extract_their_term(k):
    # sum over B(k) of w * F for F = 1, r+s, rs: (0, 0, 1) for alpha (bulk),
    # (0, 1, 0) for beta (surface), (1, 0, 0) for gamma (corner)
    for wfun, want in ((S.alpha_weight, (0, 0, 1)), (S.beta_weight, (0, 1, 0)), (S.gamma_weight, (1, 0, 0))):
        got = [0, 0, 0]
        for r, s in S.rectangles(k):
            w = wfun(k, r, s)
            got[0] += w
            got[1] += w * (r + s)
            got[2] += w * r * s
        assert tuple(got) == want, (wfun.__name__, k)


def test_printed_surface_weight_fails_the_pins():
    # planted mistake: the printed last term (r+s-2)/2 of beta_k
    from fractions import Fraction

    def printed(k, r, s):
        n = r + s
        d = lambda a, b: 1 if a == b else 0  # noqa: E731
        w = (Fraction(2 - n, 2) * d(n, k) + Fraction(3 * n - 2, 2) * d(n, k - 1)
             - Fraction(3 * n + 2, 2) * d(n, k - 2) + Fraction(n - 2, 2) * d(n, k - 3)) * (2 - d(r, s))
        return int(w)
    k = 8
    assert sum(printed(k, r, s) * (r + s) for r, s in S.rectangles(k)) != 1
    orig = S.beta_weight
    try:
        S.beta_weight = printed
        _, be, _ = S.square_series(k)
    finally:
        S.beta_weight = orig
    assert be != [table1()[i][1] for i in range(2 * k - 3)]


def test_x_to_z_substitution():
    N = 10
    # x = z/(1+z) = z - z^2 + z^3 - ...
    assert S.x_to_z([0, 1], N) == [0] + [(-1) ** (i + 1) for i in range(1, N + 1)]
    # 1/(1-x) = 1 + z in z: (1 - x) (1 + z) = 1
    one_minus_x = S.x_to_z([1, -1], N)
    assert S.ps_mul(one_minus_x, [1, 1] + [0] * (N - 1), N) == [1] + [0] * N


def test_power_series_inverse_and_powers():
    N = 12
    a = [1, 3, -2, 5] + [0] * (N - 3)
    assert S.ps_mul(a, S.ps_inv(a, N), N) == [1] + [0] * N
    assert S.ps_pow(a, 3, N) == S.ps_mul(S.ps_mul(a, a, N), a, N)
    assert S.ps_mul(S.ps_pow(a, -2, N), S.ps_pow(a, 2, N), N) == [1] + [0] * N


def test_ptilde_of_a_path_in_z():
    # 1 x s rectangle = path of s vertices: P = q (q-1)^(s-1), so
    # P~ = q^-s P = (1 - x)^(s-1) and, in z, (1+z)^-(s-1)
    N = 8
    rows = S.ptilde_x(T.SQUARE, 1, 4, N)
    for s in range(1, 5):
        pz = S.x_to_z(rows[s - 1], N)
        assert S.ps_mul(pz, S.ps_pow([1, 1] + [0] * (N - 1), s - 1, N), N) == [1] + [0] * N


# ---------------------------------------------------------------------------
# Triangular lattice (Sec. 4.4): Baxter's variable x, q = 2 - x - 1/x
# ---------------------------------------------------------------------------
def triangular_golden():
    """tests/golden/triangular_series.txt: the printed exp(f_s), exp(f_c)."""
    fs, fc = [], []
    with open(os.path.join(GOLDEN, "triangular_series.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, a, b = ln.split()
            assert int(k) == len(fs)
            fs.append(int(a))
            fc.append(int(b))
    return fs, fc


def _one_minus_power(e, power, N):
    """(1 - x^e)^power as a series to x^N (power may be negative)."""
    f = [1] + [0] * N
    if e <= N:
        f[e] = -1
    base = f if power > 0 else S.ps_inv(f, N)
    out = [1] + [0] * N
    for _ in range(abs(power)):
        out = S.ps_mul(out, base, N)
    return out


def _periodic_product(period, exps, N):
    """prod_{j>=1} prod_k (1 - x^{period j - k})^{exps[k]} to x^N."""
    out = [1] + [0] * N
    for j in range(1, N // period + 2):
        for k, pw in exps.items():
            e = period * j - k
            if 1 <= e <= N:
                out = S.ps_mul(out, _one_minus_power(e, pw, N), N)
    return out


def baxter_bulk(N):
    """-x exp(f_b) from Baxter's product (eq. efb): the product over j of
    (1-x^{6j-3})(1-x^{6j-2})^2(1-x^{6j-1}) / ((1-x^{6j-5})(1-x^{6j-4})(1-x^{6j})(1-x^{6j+1}))."""
    return _periodic_product(6, {3: 1, 2: 2, 1: 1, 5: -1, 4: -1, 0: -1, -1: -1}, N)


def test_triangular_golden_matches_the_printed_products():
    # the transcribed series against the paper's own product forms of
    # exp(f_s) and exp(f_c) (eqs. efs, efc), which it reports agree to x^40
    fs, fc = triangular_golden()
    assert len(fs) == len(fc) == 41
    assert fs == _periodic_product(12, {11: 2, 6: 2, 5: 2, 4: 2, 9: -2, 8: -2, 7: -2, 2: -2}, 40)
    assert fc == _periodic_product(12, {11: -1, 10: 1, 9: 3, 8: 2, 7: 4, 6: -3, 5: 1, 4: -3, 3: 5, 2: 2, 1: 2, 0: 1},
                                   40)


def test_baxter_to_x_substitution():
    # u = 1/q with q = 2 - x - 1/x: u = -x/(1-x)^2 = -x - 2x^2 - 3x^3 - ...;
    # a polynomial in u and its series in x agree at a rational point inside
    # the disc of convergence (exact rationals, truncation far below 1e-40)
    N = 12
    assert S.inverse_q_to_baxter_x([0, 1], N) == [0] + [-i for i in range(1, N + 1)]
    from fractions import Fraction
    x = Fraction(1, 9)
    u = -x / (1 - x) ** 2
    poly = [3, -1, 4, 1, -5]
    lhs = sum(c * u ** j for j, c in enumerate(poly))
    ser = S.inverse_q_to_baxter_x(poly, 60)
    rhs = sum(c * x ** i for i, c in enumerate(ser))
    assert abs(float(lhs - rhs)) < 1e-40


@pytest.mark.parametrize("k", [5, 8, 11, 12])
def test_triangular_series_match_paper(k):
    fs, fc = triangular_golden()
    N = k - 1
    bulk, surf, corner = S.triangular_series(k)
    assert bulk == baxter_bulk(N)
    assert surf == fs[: N + 1]
    assert corner == fc[: N + 1]


def test_triangular_bulk_needs_its_prefactor():
    # planted mistake: exp(f_b) without q = -(1-x)^2/x (the bulk product alone)
    k = 9
    bulk, _, _ = S.triangular_series(k)
    alone = S.ps_mul(bulk, S.ps_inv([1, -2, 1] + [0] * (k - 1), k - 1), k - 1)
    assert alone != baxter_bulk(k - 1)
