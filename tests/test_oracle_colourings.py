"""Pins of oracle/colourings.py, the count of proper 3-colourings of the
square rectangles by a colour transfer matrix (P(3) by the definition of
Sec. 1): brute force, closed forms, the transposition symmetry, the
partition transfer matrix of the oracle at q = 3, and the stored m = 20
values."""
import os

import pytest

from oracle import colourings as OC
from oracle import graphs as OG
from oracle import transfer as OT

HERE = os.path.dirname(os.path.abspath(__file__))


def test_brute_force_counts():
    for m in range(1, 5):
        got = OC.square_three_colourings(m, 4)
        for r in range(1, 5):
            vs, es = OG.lattice_graph("square", m, r)
            assert got[r - 1] == OG.count_colourings(vs, es, 3), (m, r)
    vs, es = OG.lattice_graph("square", 2, 3)
    assert OC.square_three_colourings(2, 3)[-1] == OG.count_colourings_product(vs, es, 3)


def test_closed_forms():
    # a path of n vertices: 3 * 2^(n-1); the 2 x n ladder q(q-1)(q^2-3q+3)^(n-1) at q = 3
    assert OC.square_three_colourings(1, 9) == [3 * 2 ** (n - 1) for n in range(1, 10)]
    ladder = [OG.poly_eval(OG.closed_form_square_ladder(n), 3) for n in range(1, 10)]
    assert OC.square_three_colourings(2, 9) == ladder == [6 * 3 ** (n - 1) for n in range(1, 10)]
    # one row of m sites: 3 * 2^(m-1)
    assert [OC.square_three_colourings(m, 1)[0] for m in range(1, 10)] == [3 * 2 ** (m - 1) for m in range(1, 10)]


def test_transposition_symmetry():
    for m in range(1, 8):
        for n in range(m, 8):
            assert OC.square_three_colourings(m, n)[-1] == OC.square_three_colourings(n, m)[-1], (m, n)


def test_equals_partition_transfer_matrix_at_q3():
    for m in range(1, 7):
        polys = OT.chromatic_exact("square", m, 8)
        assert OC.square_three_colourings(m, 8) == [OG.poly_eval(p, 3) for p in polys], m


def test_planted_mistake_is_caught():
    # the same count with the horizontal constraint of new rows dropped (any
    # difference allowed) must disagree with brute force
    vs, es = OG.lattice_graph("square", 3, 3)
    brute = OG.count_colourings(vs, es, 3)
    vs2, es2 = OG.lattice_graph("square", 3, 3)
    es2 = [e for e in es2 if vs2[e[0]][0] == vs2[e[1]][0] and vs2[e[0]][0] == 1 or vs2[e[0]][1] == vs2[e[1]][1]]
    assert OG.count_colourings(vs2, es2, 3) != brute
    assert OC.square_three_colourings(3, 3)[-1] == brute


def test_stored_m20_values():
    path = os.path.join(HERE, "golden", "square_three_colourings_m20.txt")
    vals = {}
    with open(path) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            lat, m, r, q, v = ln.split()
            assert (lat, m, q) == ("square", "20", "3")
            vals[int(r)] = int(v)
    assert sorted(vals) == list(range(1, 22))
    assert vals[1] == 3 * 2 ** 19 and vals[2] == 6 * 3 ** 19
    # rows 3..8 by the transposed rectangles, narrow strips of length 20
    for r in range(3, 9):
        assert vals[r] == OC.square_three_colourings(r, 20)[-1], r
