"""Host finish of the finite-lattice series (paper_1005_3609_amd.finite_lattice):
its weights equal the oracle's, and combining P~ residues computed without
the GPU (the normalised maps run by a test interpreter) reproduces the
paper's Table 1 after the CRT lift."""
import pytest

from mapinterp import run_series, table1
from oracle import series as S
from paper_1005_3609_amd import finite_lattice as FL
from paper_1005_3609_amd import host
from paper_1005_3609_amd import workloads as W


@pytest.mark.parametrize("k", range(3, 30))
def test_weights_match_oracle(k):
    assert sorted(FL.rectangles(k)) == sorted(S.rectangles(k))
    for r, s in FL.rectangles(k):
        assert FL.weights(k, r, s) == (S.alpha_weight(k, r, s), S.beta_weight(k, r, s), S.gamma_weight(k, r, s))


def test_series_helpers_mod_p():
    p = 998244353
    N = 9
    a = [1, 4, p - 3, 7, 0, 2, 0, 0, 0, 0]
    inv = FL._inv(a, N, p)
    assert FL._mul(a, inv, N, p) == [1] + [0] * N
    assert FL._mul(FL._pow(a, -3, N, p), FL._pow(a, 3, N, p), N, p) == [1] + [0] * N
    # x -> z agrees with the oracle's integer substitution, reduced mod p
    px = [1, -5, 9, -2, 4]
    assert FL._in_z([c % p for c in px], N, p) == [c % p for c in S.x_to_z(px, N)]


def test_combination_reproduces_table1():
    k = 10
    N = 2 * k - 4
    primes = [2147483647, 998244353, 1000000007]
    mods = []
    for p in primes:
        pt = {}
        for r in range(1, k // 2 + 1):
            res = run_series("square", r, k - r, N, p)
            for s in range(r, k - r + 1):
                pt[(r, s)] = [int(v) for v in res[s - 1]]
        mods.append(FL.combine_mod(pt, k, p))
    t = table1()
    for which in range(3):
        got = []
        for i in range(N + 1):
            x, M = host.crt([mods[b][which][i] for b in range(len(primes))], primes)
            got.append(host.symmetric(x, M))
        assert got == [t[i][which] for i in range(N + 1)], which


def test_prime_groups_bound_the_workspace():
    from paper_1005_3609_amd import api
    primes = W.seeded_primes(5, 2024)
    one = api.series_workspace_bytes("square", 6, 8, 1, 30, "graph", dict(lanes_v=1))
    assert api.series_workspace_bytes("square", 6, 8, 3, 30, "graph", dict(lanes_v=1)) <= 3 * one
    for limit, sizes in ((10 * one, [5]), (2 * one + 1, [2, 2, 1]), (one, [1] * 5), (1, [1] * 5)):
        g = FL.prime_groups(6, 8, 30, primes, "graph", dict(lanes_v=1), limit)
        assert [len(x) for x in g] == sizes
        assert sum(g, []) == primes


def test_polygon_mu_matches_oracle():
    assert FL.polygon_mu(44) == [int(x) for x in S.mu_coefficients(44)]


@pytest.mark.parametrize("k,extra", [(9, True), (10, False), (11, True)])
def test_square_series_host_pipeline(monkeypatch, k, extra):
    # the whole host side of square_series (prime groups, per-prime
    # combination, polygon term, CRT stabilisation) with the strips run by
    # the map interpreter instead of the GPU
    import numpy as np

    def cpu_series(lat, m, n, d, primes, mode="graph", tuning=None):
        return np.stack([run_series(lat, m, n, d, int(p)) for p in primes], axis=1)
    monkeypatch.setattr(FL.api, "series", cpu_series)
    res = FL.square_series(k, W.seeded_primes(4, 7), workspace_limit=1, extra=extra)
    t = table1()
    N = 2 * k - 4 + extra
    assert res["stable"]
    assert res["alpha"] == [t[i][0] for i in range(N + 1)]
    assert res["beta"] == [t[i][1] for i in range(N + 1)]
    assert res["gamma"] == [t[i][2] for i in range(2 * k - 3)]
    if extra:
        monkeypatch.setattr(FL, "polygon_mu", lambda n: [0] * (n + 1))   # planted: the polygon term dropped
        bad = FL.square_series(k, W.seeded_primes(4, 7), extra=True)
        assert bad["alpha"][N] != t[N][0] and bad["beta"][N] != t[N][1]
    else:
        with pytest.raises(ValueError):
            FL.square_series(k, W.seeded_primes(4, 7), extra=True)


def _triangular_golden():
    import os
    fs, fc = [], []
    with open(os.path.join(os.path.dirname(__file__), "golden", "triangular_series.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                _, a, b = ln.split()
                fs.append(int(a))
                fc.append(int(b))
    return fs, fc


def test_baxter_bulk_matches_the_oracle_pin():
    from test_oracle_series_pins import baxter_bulk
    assert FL.baxter_bulk(40) == baxter_bulk(40)


@pytest.mark.parametrize("k", [9, 12])
def test_triangular_series_host_pipeline(monkeypatch, k):
    # host side of triangular_series with the strips run by the map interpreter
    import numpy as np

    def cpu_series(lat, m, n, d, primes, mode="graph", tuning=None):
        assert lat == "triangular"
        return np.stack([run_series(lat, m, n, d, int(p)) for p in primes], axis=1)
    monkeypatch.setattr(FL.api, "series", cpu_series)
    res = FL.triangular_series(k, W.seeded_primes(3, 11), workspace_limit=1)
    fs, fc = _triangular_golden()
    N = k - 1
    assert res["stable"] and res["primes_used"] == 2
    assert res["bulk"] == FL.baxter_bulk(N)
    assert res["surface"] == fs[: N + 1]
    assert res["corner"] == fc[: N + 1]
    assert res == dict(zip(("bulk", "surface", "corner"), S.triangular_series(k)), primes_used=2, stable=True)


def test_triangular_substitution_mod_p():
    p = 998244353
    pu = [1, -7, 3, 0, 12, -1]
    N = 11
    assert FL._in_baxter_x([c % p for c in pu], N, p) == [c % p for c in S.inverse_q_to_baxter_x(pu, N)]
