"""Host checks of exact chromatic polynomials (paper_1005_3609_amd.polynomial.check):
every property holds on the oracle's polynomials, and each planted mistake of
the kinds a broken lift or transfer would make is caught."""
import itertools

import pytest

from oracle import graphs as OG
from oracle import transfer as OT
from paper_1005_3609_amd import polynomial as PL

SQ, TRI = "square", "triangular"


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_graph_counts_match_the_graph(lat):
    for m, n in itertools.product(range(1, 6), range(1, 6)):
        vs, es = OG.lattice_graph(lat, m, n)
        adj = {frozenset(e) for e in es}
        tri = sum(1 for a, b, c in itertools.combinations(range(len(vs)), 3)
                  if {frozenset((a, b)), frozenset((b, c)), frozenset((a, c))} <= adj)
        V, E, T, F = PL.graph_counts(lat, m, n)
        assert (V, E, T) == (len(vs), len(es), tri), (lat, m, n)
        if lat == SQ:
            four = sum(1 for a, b, c, d in itertools.permutations(range(len(vs)), 4)
                       if a == min(a, b, c, d) and b < d
                       and {frozenset((a, b)), frozenset((b, c)), frozenset((c, d)), frozenset((d, a))} <= adj)
            assert F == four, (m, n)


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_properties_hold_on_oracle_polynomials(lat):
    for m in range(1, 7):
        polys = OT.chromatic_exact(lat, m, 8)
        for r, p in enumerate(polys, start=1):
            assert PL.check(lat, m, r, p) == [], (lat, m, r)
    # one polynomial by deletion-contraction-free brute force over subsets
    vs, es = OG.lattice_graph(lat, 3, 3)
    assert PL.check(lat, 3, 3, OG.chromatic_by_subsets(vs, es)) == []
    # and one long strip of degree past 256
    assert PL.check(lat, 4, 70, OT.chromatic_exact(lat, 4, 70)[-1]) == []


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_planted_mistakes_are_caught(lat):
    m, n = 5, 6
    good = OT.chromatic_exact(lat, m, n)[-1]
    V = m * n
    M = (2 ** 31 - 1) * 998244353          # a lift that wrapped once
    plants = {
        "wrapped lift": lambda c: c.__setitem__(V // 2, c[V // 2] - M),
        "one coefficient off by one": lambda c: c.__setitem__(V // 3, c[V // 3] + 1),
        "sign of one coefficient": lambda c: c.__setitem__(V - 5, -c[V - 5]),
        "top term lost": lambda c: c.pop(),
        "two neighbours swapped": lambda c: c.__setitem__(slice(10, 12), [c[11], c[10]]),
        "constant term": lambda c: c.__setitem__(0, 1),
    }
    for name, plant in plants.items():
        c = list(good)
        plant(c)
        assert PL.check(lat, m, n, c), name
    # the right polynomial for the wrong rectangle
    assert PL.check(lat, m, n + 1, good)
    assert PL.check(SQ if lat == TRI else TRI, m, n, good)


def test_evaluate_and_read_values(tmp_path):
    assert PL.evaluate([0, -1, 1], 3) == 6 and PL.evaluate([5], 7) == 5 and PL.evaluate([], 2) == 0
    f = tmp_path / "v.txt"
    f.write_text("# comment\nsquare 4 2 3 162\nsquare 4 9 3 1\ntriangular 4 2 3 6\nsquare 5 1 3 48\n")
    assert PL.read_values(str(f), "square", 4, 5) == [(2, 3, 162)]
    # the stored 3-colouring counts agree with the oracle's exact polynomials where both exist
    p = OT.chromatic_exact(SQ, 4, 2)[-1]
    assert PL.evaluate(p, 3) == 162


def test_primes_per_call():
    GiB = 1 << 30
    assert PL.primes_per_call(119 * GiB, 287 * GiB) == 1       # square 20 x 21 on one MI355X
    assert PL.primes_per_call(6 * GiB, 287 * GiB) == 8         # capped
    assert PL.primes_per_call(100 * GiB, 10 * GiB) == 1        # never below one
    assert PL.primes_per_call(30 * GiB, 100 * GiB) == 2
