"""GPU parity of the coefficient form (normalised chromatic polynomial
P~ = q^-|V| P as truncated polynomials in x = 1/q, Sec. 3.5): bit-exact
against the oracle's truncated P~, and at full width against the
evaluation form's polynomial recovered by interpolation."""
import numpy as np
import pytest

from oracle import transfer as OT
from paper_1005_3609_amd import api, host
from paper_1005_3609_amd import workloads as W

pytestmark = pytest.mark.gpu
SQ, TRI = "square", "triangular"
P31 = 2 ** 31 - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    yield


def _oracle(lat, m, n_max, d, primes):
    res = OT.projected_strip(lat, m, n_max, OT.ExactX(dmax=d))
    out = np.zeros((n_max, len(primes), d + 1), dtype=np.int64)
    for r, z in enumerate(res):
        z = list(z)[: d + 1]
        for b, p in enumerate(primes):
            out[r, b, : len(z)] = [c % p for c in z]
    return out


@pytest.mark.parametrize("lat", [SQ, TRI])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_series_matches_oracle(lat, m):
    primes = [P31, 998244353]
    for d, tune in ((20, dict(lanes_v=1)), (63, dict(lanes_v=1, targets_per_wave=3, waves_per_block=2)),
                    (100, dict(lanes_v=2, unroll=8, streams=2))):
        want = _oracle(lat, m, 5, d, primes)
        for mode in ("batched", "graph"):
            got = api.series(lat, m, 5, d, primes, mode=mode, tuning=tune).astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"{lat} m={m} d={d} {mode} {tune}")


def test_series_tunings_identical():
    primes = W.seeded_primes(3, 11)
    ref = api.series(SQ, 7, 6, 120, primes, mode="graph", tuning=dict(lanes_v=2))
    for tune in (dict(lanes_v=4, targets_per_wave=16, waves_per_block=8, xcd_order=3),
                 dict(lanes_v=2, targets_per_wave=1, waves_per_block=1, unroll=8),
                 dict(lanes_v=2, targets_per_wave=33, waves_per_block=4, streams=3, xcd_order=2)):
        for mode in ("batched", "graph"):
            got = api.series(SQ, 7, 6, 120, primes, mode=mode, tuning=tune)
            np.testing.assert_array_equal(got, ref, err_msg=f"{mode} {tune}")


def test_series_lifts_to_exact_polynomial():
    primes = W.seeded_primes(4, 12)
    d = 25
    res = api.series(SQ, 4, 6, d, primes, mode="graph", tuning=dict(lanes_v=1))
    exact = OT.chromatic_exact(SQ, 4, 6)
    for r in range(6):
        V = 4 * (r + 1)
        want = [exact[r][V - k] if 0 <= V - k < len(exact[r]) else 0 for k in range(d + 1)]
        coef, used = host.series_stabilised(res[r].astype(np.int64), primes)
        assert coef == want, r


@pytest.mark.parametrize("lat,m", [(SQ, 14), (TRI, 12)])
def test_series_full_width_matches_evaluation_form(lat, m):
    # m x 1 .. m x 5 rectangles: |V| = m (r+1) <= 70 < 80 coefficients kept, so
    # the coefficient form holds P~ exactly; the evaluation form at q = 0..70
    # gives P itself by interpolation (mod p): P~_k = P_{|V|-k}.
    primes = W.seeded_primes(2, 13)
    n = 5
    d = 79
    ser = api.series(lat, m, n, d, primes, mode="graph", tuning=dict(lanes_v=2))
    qs = list(range(0, 71))
    ev = api.strip(lat, m, n, qs, primes, mode="graph")
    for r in range(n):
        V = m * (r + 1)
        if V > 70:
            continue
        for b, p in enumerate(primes):
            poly = host.interp_mod_p(qs, [int(ev[r, a, b]) for a in range(len(qs))], p)
            want = [poly[V - k] if V - k >= 0 else 0 for k in range(d + 1)]
            np.testing.assert_array_equal(ser[r, b].astype(np.int64), want, err_msg=f"{lat} m={m} r={r} p={p}")


def test_series_edge_cases():
    # d_max = 0: only the constant term, 1 for every rectangle
    got = api.series(SQ, 5, 4, 0, [P31, 3], mode="graph")
    assert got.shape == (4, 2, 1) and (got == 1).all()
    # n_max = 0: nothing to compute
    assert api.series(TRI, 4, 0, 10, [P31]).shape == (0, 1, 11)
    # the largest truncation of each chunk width, extreme primes (3, 5 and
    # 2^31 - 19), one row, one prime
    for d, lanes_v in ((63, 1), (127, 2), (255, 4), (511, 8)):
        primes = [3, 5, 2147483629]
        want = _oracle(TRI, 3, 6, d, primes)
        for mode in ("batched", "graph"):
            got = api.series(TRI, 3, 6, d, primes, mode=mode, tuning=dict(lanes_v=lanes_v)).astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"d={d} {mode}")
    want = _oracle(SQ, 6, 1, 40, [2147483629])
    np.testing.assert_array_equal(api.series(SQ, 6, 1, 40, [2147483629]).astype(np.int64), want)


@pytest.mark.parametrize("lat,m,n", [(SQ, 5, 6), (TRI, 4, 7), (SQ, 4, 66)])
def test_series_lanes_v8_matches_oracle(lat, m, n):
    # 512 coefficient slots per row (two 16-byte accesses per lane); 4 x 66
    # has 264 vertices, so coefficients past x^255 are non-zero
    primes = [P31, 998244353, 3]
    for d in (255, 300, 511):
        want = _oracle(lat, m, n, d, primes)
        for mode, tune in (("graph", None), ("batched", dict(lanes_v=8)),
                           ("graph", dict(lanes_v=8, targets_per_wave=3, waves_per_block=2, xcd_order=2)),
                           ("batched", dict(lanes_v=8, targets_per_wave=33, waves_per_block=8, streams=2))):
            if tune is None and d < 256:
                continue
            got = api.series(lat, m, n, d, primes, mode=mode, tuning=tune).astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"{lat} m={m} d={d} {mode} {tune}")


def test_series_lanes_v8_identical_to_narrower(monkeypatch):
    # the same truncation through every chunk width, 32-bit and 64-bit row
    # addressing
    primes = W.seeded_primes(2, 15)
    ref = api.series(SQ, 9, 7, 60, primes, mode="graph", tuning=dict(lanes_v=1))
    for tune in (dict(lanes_v=2), dict(lanes_v=4), dict(lanes_v=8)):
        np.testing.assert_array_equal(api.series(SQ, 9, 7, 60, primes, mode="graph", tuning=tune), ref)
    monkeypatch.setenv("CHROMSTRIP_WIDE_ROWS", "1")
    for mode in ("graph", "batched"):
        got = api.series(SQ, 9, 7, 60, primes, mode=mode, tuning=dict(lanes_v=8))
        np.testing.assert_array_equal(got, ref, err_msg=f"wide rows {mode}")


def test_prepare_series_then_capture_free_call():
    # maps prepared ahead; the series call itself then only queues work
    api.prepare_series(TRI, 9)
    primes = W.seeded_primes(2, 5)
    got = api.series(TRI, 9, 4, 30, primes, mode="graph").astype(np.int64)
    np.testing.assert_array_equal(got, _oracle(TRI, 9, 4, 30, primes))
    with pytest.raises(api.ChromError):
        api.prepare_series(SQ, 0)


@pytest.mark.parametrize("lat,m", [(SQ, 1), (SQ, 2), (SQ, 9), (SQ, 13), (TRI, 3), (TRI, 12)])
def test_device_built_maps_equal_host_maps(lat, m):
    # with the reader order applied on the device, the maps built there are
    # word for word the host builder's (same spaces, numbering and codes)
    api.release_maps()
    for which in (4, 5):
        for i in range(m):
            rp_d, ent_d, nc_d = api.series_map_export(lat, m, which, i)
            rp_h, cols, codes, nc_h = api.map_export(lat, m, which, i)
            ent_h = (cols | (codes << 26)).astype(np.uint32)
            assert nc_d == nc_h, (which, i)
            np.testing.assert_array_equal(rp_d, rp_h, err_msg=f"row pointers {which} {i}")
            np.testing.assert_array_equal(ent_d, ent_h, err_msg=f"entries {which} {i}")


def test_series_bad_arguments():
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 64, [P31], tuning=dict(lanes_v=1))          # d_max >= 64 lanes_v
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 10, [P31], tuning=dict(fuse=2))
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 10, [P31], mode="grouped")
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 10, [4])
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 512, [P31])                                 # past 64 * 8 slots
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 300, [P31], tuning=dict(lanes_v=8, unroll=8))
    with pytest.raises(api.ChromError):
        api.series(SQ, 4, 3, 300, [P31], tuning=dict(lanes_v=16))
    with pytest.raises(api.ChromError):                                   # evaluation form: at most 4
        api.strip(SQ, 4, 3, [3, 4], [P31], mode="batched", tuning=dict(lanes_v=8))


def test_series_wide_row_addressing_identical(monkeypatch):
    # 64-bit row bases (used when one chunk's vector reaches 4 GiB, m >= 19
    # with 80+ coefficients) give the same residues as 32-bit offsets
    primes = W.seeded_primes(2, 14)
    ref = api.series(SQ, 8, 6, 90, primes, mode="graph", tuning=dict(lanes_v=2))
    monkeypatch.setenv("CHROMSTRIP_WIDE_ROWS", "1")
    for mode, tune in (("graph", dict(lanes_v=2)), ("batched", dict(lanes_v=2, unroll=8, streams=2)),
                       ("graph", dict(lanes_v=4, targets_per_wave=3, waves_per_block=2))):
        got = api.series(SQ, 8, 6, 90, primes, mode=mode, tuning=tune)
        np.testing.assert_array_equal(got, ref, err_msg=f"{mode} {tune}")
    got = api.series(TRI, 7, 5, 40, primes, mode="graph", tuning=dict(lanes_v=1))
    monkeypatch.delenv("CHROMSTRIP_WIDE_ROWS")
    np.testing.assert_array_equal(got, api.series(TRI, 7, 5, 40, primes, mode="graph", tuning=dict(lanes_v=1)))


@pytest.mark.parametrize("lat,m,d", [(SQ, 1, 10), (SQ, 7, 40), (SQ, 12, 79), (TRI, 3, 20), (TRI, 11, 60)])
def test_device_built_maps_match_host_built(monkeypatch, lat, m, d):
    # the coefficient form's maps built on the device (paper order) and on the
    # host (reader order, uploaded) give the same coefficients
    primes = W.seeded_primes(3, 21)
    api.release_maps()
    dev = api.series(lat, m, m + 2, d, primes, mode="graph")
    api.release_maps()
    monkeypatch.setenv("CHROMSTRIP_HOST_MAPS", "1")
    host_built = api.series(lat, m, m + 2, d, primes, mode="graph")
    api.release_maps()
    monkeypatch.delenv("CHROMSTRIP_HOST_MAPS")
    np.testing.assert_array_equal(dev, host_built)
    np.testing.assert_array_equal(dev[:, :, 0], 1)


@pytest.mark.parametrize("lat,m,n", [(SQ, 1, 4), (SQ, 4, 6), (TRI, 3, 5), (SQ, 6, 7), (SQ, 6, 43), (TRI, 7, 73)])
def test_exact_chromatic_polynomials(lat, m, n):
    # the whole integer polynomial from the coefficient form and CRT, no
    # interpolation, against the oracle's exact polynomials
    from paper_1005_3609_amd import polynomial as PL
    polys, used = PL.chromatic_polynomials(lat, m, n)
    want = OT.chromatic_exact(lat, m, n)
    for r in range(n):
        got = list(polys[r])
        while len(got) > 1 and got[-1] == 0:
            got.pop()
        assert got == want[r], (lat, m, r + 1)
    assert used >= 2


def test_exact_polynomials_past_256_vertices_against_three_colourings():
    # square 12 x r, r = 1..22 (|V| up to 264: 512-slot rows): P(3) of every
    # rectangle equals the number of proper 3-colourings counted by the
    # oracle's colour transfer matrix, which shares nothing with the
    # partition transfer matrix; every polynomial has the properties of check
    from oracle import colourings as OC
    from paper_1005_3609_amd import polynomial as PL
    polys, used = PL.chromatic_polynomials(SQ, 12, 22)
    assert [PL.evaluate(p, 3) for p in polys] == OC.square_three_colourings(12, 22)
    for r, p in enumerate(polys, start=1):
        assert PL.check(SQ, 12, r, p) == [], r
