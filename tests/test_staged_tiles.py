"""Host logic of the staged-tile form of the factor maps (the `stage`
tuning): every tile respects its limits, its source list is exactly the set
of sources its rows read, and each re-encoded entry points back at the
source and code of the plain map."""
import numpy as np
import pytest

from paper_1005_3609_amd import api


@pytest.mark.parametrize("lattice,m,fuse", [("square", 6, 1), ("square", 7, 2), ("triangular", 6, 1),
                                            ("triangular", 5, 3), ("square", 9, 2)])
@pytest.mark.parametrize("slots,rows", [(1, 1), (8, 4), (24, 16), (96, 32)])
def test_staged_tiles_reproduce_the_map(lattice, m, fuse, slots, rows):
    nfac = -(-m // fuse)
    for idx in range(nfac):
        rp, cols, codes, _ = api.map_export(lattice, m, 0 if fuse == 1 else fuse, idx)
        st = api.stage_export(lattice, m, fuse, idx, slots, rows)
        tr, ts, src = st["tile_row0"], st["tile_src0"], st["src"]
        n_rows = len(rp) - 1
        assert tr[0] == 0 and tr[-1] == n_rows and ts[0] == 0 and ts[-1] == len(src)
        assert np.all(np.diff(tr) >= 1) and np.all(np.diff(tr) <= rows)
        np.testing.assert_array_equal(st["codes"], codes)
        widest = 0
        for t in range(len(tr) - 1):
            e0, e1 = rp[tr[t]], rp[tr[t + 1]]
            lst = src[ts[t]:ts[t + 1]]
            assert np.all(np.diff(lst) > 0)                       # ascending, distinct
            np.testing.assert_array_equal(lst, np.unique(cols[e0:e1]))
            np.testing.assert_array_equal(lst[st["slots"][e0:e1]], cols[e0:e1])
            if tr[t + 1] - tr[t] > 1:                               # several rows: within the slot limit
                assert len(lst) <= slots
            widest = max(widest, len(lst))
        assert st["max_slots"] == widest


def test_staged_tiles_are_greedy():
    # a tile stops only when the next row would break a limit
    rp, cols, _, _ = api.map_export("square", 8, 2, 1)
    st = api.stage_export("square", 8, 2, 1, 24, 8)
    tr = st["tile_row0"]
    for t in range(len(tr) - 2):
        nxt = tr[t + 1]
        rows_ok = nxt - tr[t] < 8
        union = np.unique(cols[rp[tr[t]]:rp[nxt + 1]])
        assert not (rows_ok and len(union) <= 24), f"tile {t} could have taken row {nxt}"


def test_stage_export_rejects_bad_arguments():
    with pytest.raises(api.ChromError):
        api.stage_export("square", 6, 4, 0, 8, 4)
    with pytest.raises(api.ChromError):
        api.stage_export("square", 6, 1, 6, 8, 4)
    with pytest.raises(api.ChromError):
        api.stage_export("square", 6, 1, 0, 0, 4)


@pytest.mark.parametrize("lattice,m,fuse", [("square", 6, 1), ("square", 9, 2), ("triangular", 6, 1),
                                            ("triangular", 7, 2), ("square", 8, 3)])
@pytest.mark.parametrize("slots,rows", [(1, 1), (12, 8), (48, 16), (96, 64)])
def test_clustered_tiles_reproduce_the_map(lattice, m, fuse, slots, rows):
    # every target row appears once; each tile's source list is exactly the
    # set its targets read; each entry's slot points back at the plain
    # map's source, with the plain map's code, in the row's order
    nfac = -(-m // fuse)
    for idx in range(nfac):
        rp, cols, codes, _ = api.map_export(lattice, m, 0 if fuse == 1 else fuse, idx)
        st = api.cluster_export(lattice, m, fuse, idx, slots, rows)
        tr, ts, src, tgt, crp = st["tile_row0"], st["tile_src0"], st["src"], st["tgt"], st["row_ptr"]
        n_rows = len(rp) - 1
        assert tr[0] == 0 and tr[-1] == n_rows and ts[-1] == len(src)
        assert np.all(np.diff(tr) >= 1) and np.all(np.diff(tr) <= rows)
        np.testing.assert_array_equal(np.sort(tgt), np.arange(n_rows))
        np.testing.assert_array_equal(np.diff(crp), np.diff(rp)[tgt])
        widest = 0
        for t in range(len(tr) - 1):
            lst = src[ts[t]:ts[t + 1]]
            assert np.all(np.diff(lst) > 0)
            reads = []
            for k in range(tr[t], tr[t + 1]):
                r = tgt[k]
                np.testing.assert_array_equal(lst[st["slots"][crp[k]:crp[k + 1]]], cols[rp[r]:rp[r + 1]])
                np.testing.assert_array_equal(st["codes"][crp[k]:crp[k + 1]], codes[rp[r]:rp[r + 1]])
                reads.append(cols[rp[r]:rp[r + 1]])
            np.testing.assert_array_equal(lst, np.unique(np.concatenate(reads)))
            if tr[t + 1] - tr[t] > 1:
                assert len(lst) <= slots
            widest = max(widest, len(lst))
        assert st["max_slots"] == widest


def test_clustered_tiles_share_sources():
    # at 64 targets and 96 slots the last fused pair's clustered tiles stage
    # well under two source rows per target, against about 2.8 for runs of
    # consecutive rows (its targets, the NCNNN states, keep the paper's order)
    rp, cols, _, _ = api.map_export("square", 12, 2, 5)
    n_rows = len(rp) - 1
    cl = api.cluster_export("square", 12, 2, 5, 96, 64)
    run = api.stage_export("square", 12, 2, 5, 10 ** 6, 64)
    assert len(cl["src"]) / n_rows < 1.8
    assert len(run["src"]) / n_rows > 2.3


# ---------------------------------------------------------------------------
# Op streams (tuning stage 5): the kernel's words decoded against the maps
# ---------------------------------------------------------------------------
def _shifted(poly, s):
    """Coefficients of sum_j c_j q^j in powers of t = q - s."""
    from math import comb
    return [sum(poly[j] * comb(j, k) * s ** (j - k) for j in range(k, 4)) for k in range(4)]


@pytest.mark.parametrize("lat,m,fuse", [("square", 7, 1), ("square", 7, 2), ("triangular", 6, 1),
                                        ("square", 11, 2)])
def test_op_streams_encode_the_maps(lat, m, fuse):
    codes = api.family_info(lat, m, fuse)["codes"]
    nf = api.family_info(lat, m, fuse)["n_factors"]
    for idx in range(nf):
        rp, cols, cc, _ = api.map_export(lat, m, 0 if fuse == 1 else fuse, idx)
        ox = api.op_export(lat, m, fuse, idx)
        w, first = ox["words"].astype(np.int64), ox["row_first"]
        assert (w[-64:] == 0).all() and first[-1] == len(w) - 64
        digits = {}
        for c, poly in enumerate(codes):
            d = _shifted(poly, ox["shift"])
            digits[c] = (d[3] == 0 and all(abs(x) <= 1 for x in d[:3]),
                         sum((1 << (24 + 2 * k)) if d[k] == 1 else (1 << (25 + 2 * k)) if d[k] == -1 else 0
                             for k in range(3)))
        for r in range(len(rp) - 1):
            row = w[first[r]:first[r + 1]]
            ents = range(rp[r], rp[r + 1])
            if len(ents) == 0:
                assert list(row) == [1 << 31]
                continue
            assert len(row) == len(ents)
            np.testing.assert_array_equal(row & ((1 << 23) - 1), cols[rp[r]:rp[r + 1]])
            np.testing.assert_array_equal(row >> 31, [0] * (len(ents) - 1) + [1])
            for word, e in zip(row, ents):
                ok, bits = digits[int(cc[e])]
                assert ok and (int(word) & 0x3F000000) == bits


def test_op_streams_refuse_other_coefficients():
    for lat, fuse in (("square", 3), ("triangular", 2)):
        with pytest.raises(api.ChromError, match="unit coefficients"):
            api.op_export(lat, 7, fuse, 1)
