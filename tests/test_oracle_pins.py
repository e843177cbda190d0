"""Pins for the oracle: each check ties it to something other than itself --
brute force, closed forms, invariants, printed lists and counts, and
agreement between methods that share no code path."""
import itertools
import os
from math import comb

import numpy as np
import pytest

from oracle import graphs as g
from oracle import partitions as P
from oracle import transfer as T

SQ, TRI = T.SQUARE, T.TRIANGULAR


def _read_lines(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]


# ---------------------------------------------------------------------------
# Definition: brute-force colourings
# ---------------------------------------------------------------------------
SMALL_RECTS = [(lat, m, n) for lat in (SQ, TRI) for m in range(1, 5) for n in range(1, 5)
               if m * n <= 12]


@pytest.mark.parametrize("lat,m,n", SMALL_RECTS)
def test_projected_tm_counts_colourings(lat, m, n):
    """Sec. 1: P_G(q) is the number of proper q-colourings."""
    V, E = g.lattice_graph(lat, m, n)
    poly = T.chromatic_exact(lat, m, n)[-1]
    for q in range(0, 5 if m * n <= 9 else 4):
        assert g.poly_eval(poly, q) == g.count_colourings(V, E, q)


def test_backtracking_matches_full_listing():
    """The backtracking count agrees with listing all q^|V| assignments."""
    for lat, m, n in [(SQ, 2, 3), (TRI, 2, 3), (SQ, 3, 3), (TRI, 3, 2)]:
        V, E = g.lattice_graph(lat, m, n)
        for q in range(0, 4):
            assert g.count_colourings(V, E, q) == g.count_colourings_product(V, E, q)


def test_colour_class_dp_matches_brute_force():
    for lat, m, n in [(SQ, 3, 4), (TRI, 3, 4), (SQ, 4, 3), (TRI, 4, 3)]:
        V, E = g.lattice_graph(lat, m, n)
        poly = g.chromatic_by_colour_classes(lat, m, n)
        for q in range(0, 5):
            assert g.poly_eval(poly, q) == g.count_colourings(V, E, q)


# ---------------------------------------------------------------------------
# FK: the spin sum (eq. Z1) equals the subset sum (eq. Z2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("v", [-1, 1, 2])
def test_spin_sum_equals_subset_expansion(v):
    for lat, m, n in [(SQ, 2, 2), (TRI, 2, 3), (SQ, 3, 2)]:
        V, E = g.lattice_graph(lat, m, n)
        poly = g.potts_by_subsets(V, E, v)
        for q in range(1, 4):
            assert g.poly_eval(poly, q) == g.potts_by_spins(V, E, q, v)


# ---------------------------------------------------------------------------
# Independent methods agree on whole polynomials
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [SQ, TRI])
def test_methods_agree(lat):
    for m in range(1, 5):
        for n in range(1, 5):
            V, E = g.lattice_graph(lat, m, n)
            tm = T.chromatic_exact(lat, m, n)[-1]
            assert tm == g.chromatic_by_colour_classes(lat, m, n)
            if len(E) <= 17:
                assert tm == g.poly_trim(g.chromatic_by_subsets(V, E))


def test_rowwise_readout_is_every_length():
    """The strip reads out P of m x r for every r = 1..n_max."""
    for lat in (SQ, TRI):
        rows = T.chromatic_exact(lat, 3, 5)
        for r, poly in enumerate(rows, start=1):
            assert poly == g.chromatic_by_colour_classes(lat, 3, r)


def test_cfg_4x5_against_colour_classes_at_q_0_to_20():
    """The 4 x 5 square rectangle at q = 0..20 mod 2^31-1, two methods."""
    p = 2 ** 31 - 1
    exact = g.chromatic_by_colour_classes(SQ, 4, 5)
    res = T.chromatic_residues(SQ, 4, 5, list(range(21)), [p] * 21)[-1]
    assert [int(x) for x in res] == [g.poly_eval(exact, q) % p for q in range(21)]


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [SQ, TRI])
def test_paths(lat):
    for k in range(1, 9):
        assert T.chromatic_exact(lat, 1, k)[-1] == g.closed_form_path(k)
        assert T.chromatic_exact(lat, k, 1)[-1] == g.closed_form_path(k)


def test_square_ladder():
    rows = T.chromatic_exact(SQ, 2, 8)
    for n, poly in enumerate(rows, start=1):
        assert poly == g.closed_form_square_ladder(n)


def test_triangular_ladder():
    rows = T.chromatic_exact(TRI, 2, 8)
    for n, poly in enumerate(rows, start=1):
        assert poly == g.closed_form_triangular_ladder(n)


def test_square_2x2_is_four_cycle():
    assert T.chromatic_exact(SQ, 2, 2)[-1] == g.closed_form_cycle(4)


def test_cycles_and_complete_graphs_generic_routines():
    for k in range(3, 9):
        V, E = g.cycle_graph(k)
        assert g.poly_trim(g.chromatic_by_subsets(V, E)) == g.closed_form_cycle(k)
        for q in range(0, 4):
            assert g.count_colourings(V, E, q) == g.poly_eval(g.closed_form_cycle(k), q)
    for k in range(1, 6):
        V, E = g.complete_graph(k)
        assert g.poly_trim(g.chromatic_by_subsets(V, E)) == g.closed_form_complete(k)


def test_k4_containing_graphs_have_no_3_colouring():
    """Graphs containing K4 have P(3) = 0 (checked on tiny graphs; the
    triangular lattice itself contains no K4)."""
    V, E = g.complete_graph(4)
    assert g.count_colourings(V, E, 3) == 0
    # K4 plus a pendant path and an extra vertex adjacent to two of its vertices
    E2 = E + [(3, 4), (4, 5), (5, 0), (1, 5)]
    V2 = list(range(6))
    assert g.poly_eval(g.chromatic_by_subsets(V2, E2), 3) == 0
    assert g.count_colourings(V2, E2, 3) == 0
    assert g.count_colourings(V2, E2, 4) > 0


# ---------------------------------------------------------------------------
# Invariants at any size
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [SQ, TRI])
def test_small_q_invariants(lat):
    for m in range(1, 6):
        for n in range(1, 6):
            poly = T.chromatic_exact(lat, m, n)[-1]
            assert g.poly_eval(poly, 0) == 0
            assert g.poly_eval(poly, 1) == (1 if m * n == 1 else 0)
            if lat == SQ or min(m, n) == 1:
                # connected bipartite: exactly two 2-colourings
                assert g.poly_eval(poly, 2) == 2
            else:
                assert g.poly_eval(poly, 2) == 0
                # triangles sharing edges force a unique 3-colouring up to S_3
                assert g.poly_eval(poly, 3) == 6


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_polynomial_coefficients(lat):
    """Degree |V|, leading 1, next coefficient -|E|, then
    C(|E|,2) - #triangles; alternating signs."""
    for m, n in [(3, 3), (3, 4), (4, 4), (2, 5)]:
        V, E = g.lattice_graph(lat, m, n)
        poly = T.chromatic_exact(lat, m, n)[-1]
        nv = len(V)
        assert len(poly) == nv + 1 and poly[nv] == 1
        assert poly[nv - 1] == -len(E)
        triangles = 0 if lat == SQ else 2 * (m - 1) * (n - 1)
        assert poly[nv - 2] == comb(len(E), 2) - triangles
        for k in range(1, nv + 1):
            assert poly[k] == 0 or (poly[k] > 0) == ((nv - k) % 2 == 0)
        assert poly[0] == 0


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_transposition_symmetry(lat):
    for m in range(1, 6):
        for n in range(1, 6):
            assert T.chromatic_exact(lat, m, n)[-1] == T.chromatic_exact(lat, n, m)[-1]


# ---------------------------------------------------------------------------
# The projector trick (Sec. 3.2): generic TM over all non-crossing
# partitions equals the projected sparse factorisation at v = -1
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [SQ, TRI])
def test_generic_equals_projected(lat):
    for m in range(1, 7):
        gen = T.generic_strip(lat, m, 4, -1, T.ExactQ())
        proj = T.projected_strip(lat, m, 4, T.ExactQ())
        for a, b in zip(gen, proj):
            assert g.poly_trim(list(a)) == g.poly_trim(list(b))


def test_generic_tm_any_v_matches_subsets():
    """The generic TM at v != -1 reproduces eq. Z2 (the projector trick is
    not used there)."""
    for lat, m, n in [(SQ, 3, 3), (TRI, 3, 3), (SQ, 2, 4), (TRI, 4, 2)]:
        V, E = g.lattice_graph(lat, m, n)
        for v in (1, 2, -2):
            tm = g.poly_trim(list(T.generic_strip(lat, m, n, v, T.ExactQ())[-1]))
            assert tm == g.poly_trim(g.potts_by_subsets(V, E, v))


# ---------------------------------------------------------------------------
# Normalised (eq. Z_modified) vs un-normalised bookkeeping
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [SQ, TRI])
def test_normalised_form(lat):
    """Sec. 3.5: P-tilde = q^{-|V|} P is a polynomial of degree |V|-1 in
    1/q with constant term 1."""
    for m, n in [(1, 3), (2, 3), (3, 3), (4, 3), (3, 4)]:
        nv = m * n
        ptil = T.projected_strip(lat, m, n, T.ExactX())[-1]
        ptil = g.poly_trim(list(ptil))
        p = T.chromatic_exact(lat, m, n)[-1]
        assert ptil[0] == 1 and len(ptil) <= nv
        # P(q) = q^{|V|} Ptilde(1/q): coefficient of q^{|V|-k} is ptil[k]
        assert [p[nv - k] if nv - k < len(p) else 0 for k in range(nv)] == \
            ptil + [0] * (nv - len(ptil))


def test_truncated_normalised_form():
    """Truncating every weight at degree d gives the first d+1 terms."""
    full = g.poly_trim(list(T.projected_strip(SQ, 4, 4, T.ExactX())[-1]))
    cut = g.poly_trim(list(T.projected_strip(SQ, 4, 4, T.ExactX(dmax=6))[-1]))
    assert cut == full[:7]


# ---------------------------------------------------------------------------
# Residues
# ---------------------------------------------------------------------------
def test_residues_match_exact_polynomials():
    rng = np.random.default_rng(7)
    ps = [2 ** 31 - 1, 2147483629, 1000000007, 998244353]
    for lat in (SQ, TRI):
        exact = T.chromatic_exact(lat, 4, 5)
        qs = [int(x) for x in rng.integers(0, 200, size=8)]
        for p in ps:
            res = T.chromatic_residues(lat, 4, 5, qs, [p] * len(qs))
            for r in range(5):
                assert [int(x) for x in res[r]] == [g.poly_eval(exact[r], q) % p for q in qs]


# ---------------------------------------------------------------------------
# States and counts (Sec. 3.2, 3.4)
# ---------------------------------------------------------------------------
def test_printed_partition_lists(golden_dir):
    nc3 = [P.from_paper(s, 3) for s in _read_lines(golden_dir, "noncrossing_m3.txt")]
    assert sorted(nc3) == sorted(P.noncrossing_partitions(3))
    m4 = [P.from_paper(s, 4) for s in _read_lines(golden_dir, "ncnnn_m4.txt")]
    assert P.ncnnn_in_paper_order(4) == m4
    m5 = [P.from_paper(s, 5) for s in _read_lines(golden_dir, "ncnnn_m5.txt")]
    assert P.ncnnn_in_paper_order(5) == m5


def test_printed_counts(golden_dir):
    rows = {ln.split()[0]: [int(x) for x in ln.split()[1:]]
            for ln in _read_lines(golden_dir, "counts.txt")}
    assert [P.catalan(m) for m in range(1, 7)] == rows["catalan"]
    assert [len(P.noncrossing_partitions(m)) for m in range(1, 7)] == rows["catalan"]
    assert [P.motzkin(k) for k in range(6)] == rows["motzkin"]
    assert [P.motzkin_by_recursion(k) for k in range(6)] == rows["motzkin"]
    assert P.motzkin(19) + P.motzkin(18) == rows["dim_square_m20"][0]
    assert P.motzkin(19) == rows["dim_triangular_m20"][0]


def test_ncnnn_order_is_a_bijection():
    for m in range(1, 10):
        order = P.ncnnn_in_paper_order(m)
        assert len(order) == len(set(order)) == P.motzkin(max(m - 1, 0))
        assert sorted(order) == sorted(P.ncnnn_partitions_by_filter(m))


def test_square_intermediate_spaces():
    """After the square factor T_i the states are the NCNNN ones plus those
    with i ~ i+1 (Sec. 3.2), M_{m-1} + M_{m-2} in number (Sec. 3.4)."""
    for m in range(3, 8):
        for i in range(1, m):
            space = P.square_intermediate_in_paper_order(m, i)
            assert len(space) == len(set(space)) == P.motzkin(m - 1) + P.motzkin(m - 2)
            expect = [p for p in P.noncrossing_partitions(m) if P.is_nnn(p, allowed=i)]
            assert sorted(space) == sorted(expect)
        # the states actually produced by T_i lie in that space
        for lat in (SQ, TRI):
            trace = []
            T.projected_strip(lat, m, 4, T.ExactQ(), trace=trace)
            for r, i, vec in trace:
                for s in vec:
                    assert P.is_noncrossing(s)
                    if lat == SQ and i < m:
                        assert P.is_nnn(s, allowed=i)
                    else:
                        assert P.is_nnn(s)


# ---------------------------------------------------------------------------
# Operator identities (Sec. 3.1, eq. projector)
# ---------------------------------------------------------------------------
def _random_vector(m, rng):
    alg = T.ExactQ()
    vec = {}
    for s in P.noncrossing_partitions(m):
        c = int(rng.integers(-3, 4))
        if c:
            vec[s] = (c, int(rng.integers(-2, 3)))
    return vec, alg


def _same(a, b):
    a = {k: g.poly_trim(list(v)) for k, v in a.items() if any(v)}
    b = {k: g.poly_trim(list(v)) for k, v in b.items() if any(v)}
    return a == b


def test_projector_identity():
    rng = np.random.default_rng(1)
    for m in (3, 4, 5):
        vec, alg = _random_vector(m, rng)
        for i in range(1, m):
            h = T.op_H(vec, i, i + 1, -1, alg)
            assert _same(T.op_H(T.op_P(vec, [i]), i, i + 1, -1, alg), h)    # H P = H
            assert _same(T.op_H(h, i, i + 1, -1, alg), h)                  # H^2 = H
            joined = {k: w for k, w in vec.items() if k[i - 1] == k[i]}
            assert T.op_H(joined, i, i + 1, -1, alg) == {}                 # H kills i~i+1


def test_vertical_edge_is_not_a_projector():
    rng = np.random.default_rng(2)
    vec, alg = _random_vector(4, rng)
    v1 = T.op_V(vec, 2, -1, alg)
    assert not _same(T.op_V(v1, 2, -1, alg), v1)


def test_last_layer_weights_are_contracted_paths():
    """T_last applied to a single state s gives the chromatic polynomial of
    the m-vertex path with the blocks of s identified (the last layer's
    horizontal edges on top of the connections s records)."""
    for m in range(2, 7):
        for s in P.ncnnn_in_paper_order(m):
            w = T.projected_readout({s: (1,)}, m, T.ExactQ())
            blocks = sorted(set(s))
            V = list(range(len(blocks)))
            E = sorted({(min(s[i], s[i + 1]), max(s[i], s[i + 1])) for i in range(m - 1)})
            assert g.poly_trim(list(w)) == g.poly_trim(g.chromatic_by_subsets(V, E))


# ---------------------------------------------------------------------------
# Planted mistakes: a plausible slip in the oracle fails a pin
# ---------------------------------------------------------------------------
def _fails_pins(monkeypatch_ctx):
    bad = False
    for lat, m, n in [(SQ, 3, 3), (TRI, 3, 3), (SQ, 4, 2), (TRI, 2, 3)]:
        V, E = g.lattice_graph(lat, m, n)
        poly = T.chromatic_exact(lat, m, n)[-1]
        for q in range(0, 4):
            if g.poly_eval(poly, q) != g.count_colourings(V, E, q):
                bad = True
    return bad


def test_planted_mistakes_are_caught(monkeypatch):
    # 1. the closure factor q forgotten
    with monkeypatch.context() as mp:
        orig = T.op_D

        def no_closure(vec, i, alg):
            out = {}
            for s, w in vec.items():
                T._acc(out, s if T.alone(s, i) else T.detach(s, i), w, alg)
            return out
        mp.setattr(T, "op_D", no_closure)
        assert _fails_pins(mp)
    # 2. the diagonal laid in the other direction is isomorphic; laying the
    # triangular diagonal after V_i instead of before it is not
    with monkeypatch.context() as mp:
        def late_diagonal(vec, i, m, alg):
            if i < m:
                vec = T.op_H(vec, i, i + 1, -1, alg)
            vec = T.op_V(vec, i, -1, alg)
            if i > 1:
                vec = T.op_H(vec, i - 1, i, -1, alg)
            return T.op_P(vec, list(range(1, m)))
        mp.setattr(T, "factor_triangular", late_diagonal)
        assert _fails_pins(mp)
    # 3. projector on the pair the square factor must leave open
    with monkeypatch.context() as mp:
        def over_projected(vec, i, m, alg):
            if i < m:
                vec = T.op_H(vec, i, i + 1, -1, alg)
            vec = T.op_V(vec, i, -1, alg)
            return T.op_P(vec, list(range(1, m)))
        mp.setattr(T, "factor_square", over_projected)
        assert _fails_pins(mp)
    # 4. wrong sign of the vertical edge (v = +1 instead of -1)
    with monkeypatch.context() as mp:
        orig_V = T.op_V
        mp.setattr(T, "op_V", lambda vec, i, v, alg: orig_V(vec, i, -v, alg))
        assert _fails_pins(mp)
    assert not _fails_pins(None)
