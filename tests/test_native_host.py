"""CPU tests of the native library's host side: the C ABI loads and exports
what the header declares, the ranking reproduces the paper's order, and the
factor maps, executed by a small numpy interpreter below (test code, not a
product path), give the oracle's residues exactly."""
import ctypes as C

import numpy as np
import pytest

from oracle import partitions as OP
from oracle import transfer as OT
from paper_1005_3609_amd import _lib, api

SQ, TRI = "square", "triangular"
P31 = 2 ** 31 - 1


def test_library_exports_every_header_function():
    L = api.lib()
    names = _lib.header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_lib._SIGS)


def test_version_and_motzkin():
    assert b"gfx950" in api.lib().chromatic_version()
    assert [api.motzkin(k) for k in range(10)] == [OP.motzkin(k) for k in range(10)]
    assert api.motzkin(19) + api.motzkin(18) == 24735666
    assert api.motzkin(41) == -1


@pytest.mark.parametrize("m", range(1, 12))
def test_ncnnn_ranking_is_paper_order(m):
    order = OP.ncnnn_in_paper_order(m)
    assert api.space_size(m) == len(order)
    for r, part in enumerate(order):
        assert api.unrank(m, r) == part
        assert api.rank(m, part) == r


def test_ranking_large_m_roundtrip():
    rng = np.random.default_rng(0)
    for m in (14, 18, 20):
        n = api.space_size(m)
        for r in [0, 1, n - 1] + [int(x) for x in rng.integers(0, n, size=200)]:
            assert api.rank(m, api.unrank(m, r)) == r


@pytest.mark.parametrize("m", range(2, 9))
def test_square_intermediate_order(m):
    for i in range(1, m):
        order = OP.square_intermediate_in_paper_order(m, i)
        assert api.space_size(m, _lib.SPACE_SQ_INTER, i) == len(order)
        for r, part in enumerate(order):
            assert api.unrank(m, r, _lib.SPACE_SQ_INTER, i) == part
            assert api.rank(m, part, _lib.SPACE_SQ_INTER, i) == r


@pytest.mark.parametrize("m", range(1, 9))
def test_last_spaces(m):
    for i in range(0, m + 1):
        expect = [p for p in OP.noncrossing_partitions(m)
                  if all(sum(1 for y in p if y == p[x]) == 1 for x in range(i)) and OP.is_nnn(p)]
        n = api.space_size(m, _lib.SPACE_LAST, i)
        assert n == len(expect)
        got = [api.unrank(m, r, _lib.SPACE_LAST, i) for r in range(n)]
        assert sorted(got) == sorted(expect)
        for r, part in enumerate(got):
            assert api.rank(m, part, _lib.SPACE_LAST, i) == r


def test_rank_rejects_states_outside_the_space():
    assert api.rank(4, (0, 0, 1, 2)) == -1            # (12)(3)(4): neighbours joined
    assert api.rank(4, (0, 1, 0, 1)) == -1            # (13)(24): crossing
    assert api.rank(4, (0, 0, 1, 2), _lib.SPACE_SQ_INTER, 1) == api.space_size(4)
    assert api.rank(4, (0, 1, 1, 2), _lib.SPACE_SQ_INTER, 1) == -1
    assert api.rank(4, (0, 1, 0, 2), _lib.SPACE_LAST, 1) == -1


# ---------------------------------------------------------------------------
# numpy interpreter of the exported maps (test code)
# ---------------------------------------------------------------------------
def _apply(csr, cvals, x, p):
    rp, cols, codes, _ = csr
    nrows = rp.size - 1
    out = np.zeros((nrows, x.shape[1]), dtype=np.int64)
    if cols.size:
        contrib = (cvals[codes] * x[cols]) % p
        rows = np.repeat(np.arange(nrows), np.diff(rp))
        np.add.at(out, rows, contrib)
    return out % p


def _eval_codes(codes, qs, ps):
    """coefficient polynomial of every code at every instance, mod p (Horner)"""
    out = []
    for c in codes:
        acc = np.zeros_like(qs)
        for k in range(len(c) - 1, -1, -1):
            acc = (acc * (qs % ps) + (c[k] % ps)) % ps
        out.append(acc)
    return np.stack(out)


def _run_maps(lat, m, n_max, qs, ps, fuse=1):
    qs = np.asarray(qs, dtype=np.int64)
    ps = np.asarray(ps, dtype=np.int64)
    fam = api.family_info(lat, m, fuse)
    cvals = _eval_codes(fam["codes"], qs, ps)
    which = 0 if fuse == 1 else fuse
    fwd = [api.map_export(lat, m, which, i) for i in range(fam["n_factors"])]
    last = [api.map_export(lat, m, 1, i) for i in range(m)]
    u = np.ones((1, qs.size), dtype=np.int64)
    for i in range(m, 0, -1):
        u = _apply(last[i - 1], cvals, u, ps)
    w = u
    x = np.zeros((w.shape[0], qs.size), dtype=np.int64)
    x[0] = 1
    rows = [(w * x % ps).sum(axis=0) % ps]
    for _ in range(1, n_max):
        for f in fwd:
            x = _apply(f, cvals, x, ps)
        rows.append((w * x % ps).sum(axis=0) % ps)
    return np.stack(rows)


@pytest.mark.parametrize("lat", [SQ, TRI])
@pytest.mark.parametrize("m", range(1, 9))
def test_maps_reproduce_oracle(lat, m):
    qs = [0, 1, 2, 3, 7, 100, P31 - 1, 5]
    ps = [P31, P31, P31, P31, P31, 1000000007, P31, 998244353]
    n_max = 6 if m <= 6 else 4
    got = _run_maps(lat, m, n_max, qs, ps)
    want = OT.chromatic_residues(lat, m, n_max, qs, ps)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_map_structure(lat):
    for m in range(1, 11):
        info = api.maps_info(lat, m)
        assert info["codes"][:2] == [(1, 0, 0, 0), (-1, 0, 0, 0)]
        for i in range(m):
            rp, cols, codes, ncols = api.map_export(lat, m, 0, i)
            assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == cols.size
            assert cols.size == 0 or (cols.min() >= 0 and cols.max() < ncols)
            assert codes.size == 0 or codes.max() < info["n_codes"]
            # fan-out per source: <= 4 (square), <= 8 (triangular)
            fan = np.bincount(cols, minlength=ncols)
            assert fan.max() <= (4 if lat == SQ else 8)
            # entries of a row are sorted by source
            for r in range(rp.size - 1):
                seg = cols[rp[r]:rp[r + 1]]
                assert np.all(np.diff(seg) > 0)
        # spaces: square intermediate M_{m-1}+M_{m-2}, else M_{m-1}
        for i in range(m):
            rp, _, _, ncols = api.map_export(lat, m, 0, i)
            nout = rp.size - 1
            if lat == SQ and i + 1 < m:
                assert nout == OP.motzkin(m - 1) + OP.motzkin(m - 2)
            else:
                assert nout == OP.motzkin(m - 1)
        # the read-out chain ends in the single state e_0
        rp, _, _, ncols = api.map_export(lat, m, 1, m - 1)
        assert ncols == 1


def test_coefficient_tables():
    sq = api.maps_info(SQ, 6)["codes"]
    # +-1, q-2, q-1, q
    assert set(sq) == {(1, 0, 0, 0), (-1, 0, 0, 0), (-2, 1, 0, 0), (-1, 1, 0, 0), (0, 1, 0, 0)}
    tri = api.maps_info(TRI, 6)["codes"]
    assert (-3, 1, 0, 0) in tri and (0, 1, 0, 0) in tri
    for lat in (SQ, TRI):
        base = api.family_info(lat, 9, 1)["codes"]
        for k in (2, 3):
            fam = api.family_info(lat, 9, k)
            assert fam["codes"][:len(base)] == base           # extends the single-factor table
            assert fam["n_factors"] == -(-9 // k)
            assert max(max(i for i in range(4) if c[i] or i == 0) for c in fam["codes"]) <= k


@pytest.mark.parametrize("lat", [SQ, TRI])
@pytest.mark.parametrize("fuse", [2, 3])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 7])
def test_fused_families_reproduce_oracle(lat, fuse, m):
    qs = [0, 1, 2, 3, 7, 100, P31 - 1, 5]
    ps = [P31, P31, P31, P31, P31, 1000000007, P31, 998244353]
    got = _run_maps(lat, m, 5, qs, ps, fuse=fuse)
    np.testing.assert_array_equal(got, OT.chromatic_residues(lat, m, 5, qs, ps))


def test_bad_arguments_are_errors_without_touching_a_gpu():
    L = api.lib()
    q = np.arange(3, dtype=np.uint32)
    p = np.array([P31], dtype=np.uint32)
    out = np.zeros(30, dtype=np.uint32)
    args = (q.ctypes.data_as(C.c_void_p), 3, p.ctypes.data_as(C.c_void_p), 1, out.ctypes.data_as(C.c_void_p))
    assert L.chromatic_strip(0, 0, 5, *args) == -1
    assert L.chromatic_strip(0, 21, 5, *args) == -1
    assert L.chromatic_strip(7, 4, 5, *args) == -1
    assert b"lattice" in L.chromatic_last_error()
    bad = np.array([2 ** 31 + 11], dtype=np.uint32)
    assert L.chromatic_strip(0, 4, 5, q.ctypes.data_as(C.c_void_p), 3, bad.ctypes.data_as(C.c_void_p), 1,
                             out.ctypes.data_as(C.c_void_p)) == -1
    even = np.array([1000], dtype=np.uint32)
    assert L.chromatic_strip(0, 4, 5, q.ctypes.data_as(C.c_void_p), 3, even.ctypes.data_as(C.c_void_p), 1,
                             out.ctypes.data_as(C.c_void_p)) == -1
    assert L.chromatic_strip(0, 4, 0, *args) == 0          # n_max = 0: nothing to do
    assert api.lib().chromatic_workspace_bytes(0, 0, 5, 3, 1, 1, None) == 0
    with pytest.raises(api.ChromError):
        api.strip("square", 4, 3, [1, 2], [P31], mode="batched", tuning={"lanes_v": 3})
    # resident mode: widths whose two state vectors do not fit a workgroup's
    # 160 KiB of LDS are refused before any device work
    with pytest.raises(api.ChromError, match="LDS"):
        api.strip("square", 13, 3, [1, 2], [P31], mode="resident")
    with pytest.raises(api.ChromError, match="LDS"):
        api.strip("triangular", 12, 3, [1, 2], [P31], mode="resident", tuning={"lanes_v": 4})
    assert api.lib().chromatic_workspace_bytes(0, 4, 3, 2, 1, 3, None) > 0
    assert api.lib().chromatic_workspace_bytes(0, 13, 3, 2, 1, 3, None) == 0
    with pytest.raises(api.ChromError, match="waves_per_block"):
        api.strip("square", 4, 3, [1, 2], [P31], mode="batched", tuning={"waves_per_block": 16})
    # op-stream gathers (stage 5) take lanes_v 1 or 2
    with pytest.raises(api.ChromError, match="stage 5"):
        api.strip("square", 4, 3, [1, 2], [P31], mode="batched", tuning={"lanes_v": 4, "stage": 5})
    with pytest.raises(api.ChromError, match="stage must be"):
        api.strip("square", 4, 3, [1, 2], [P31], mode="batched", tuning={"stage": 7})
    # resident mode's stage picks the arithmetic: 0 or 1 only
    with pytest.raises(api.ChromError, match="resident mode takes stage"):
        api.strip("square", 4, 3, [1, 2], [P31], mode="resident", tuning={"stage": 2})
    # lanes_v 4 at 640 instances: a job of 512 at lanes_v 4 and one of 128 at
    # lanes_v 2, each with its own workspace region (no padded chunk)
    w4 = api.workspace_bytes("square", 8, 5, 80, 8, "graph", {"lanes_v": 4})
    w2 = api.workspace_bytes("square", 8, 5, 16, 8, "graph", {"lanes_v": 2})
    w4a = api.workspace_bytes("square", 8, 5, 64, 8, "graph", {"lanes_v": 4})
    assert w4 == -(-w4a // 256) * 256 + -(-w2 // 256) * 256
    # a batch's grouped gathers take the target orders (4, 6) but no LDS staging or op streams
    job = dict(lattice="square", m=4, n_max=3, q_points=[1, 2], primes=[P31])
    assert api.batch_workspace_bytes([job], tuning={"stage": 6}) == api.batch_workspace_bytes([job])
    for st in (1, 2, 3, 5):
        with pytest.raises(api.ChromError, match="stage 0, 4 or 6"):
            api.batch_workspace_bytes([job], tuning={"stage": st})
