"""GPU parity: every execution path of the native library against the CPU
oracle, bit for bit (the arithmetic is exact, so the tolerance is zero).

Small cases run the oracle live; full-size workloads compare against stored
oracle values written by tests/golden/make_golden.py on sampled instances,
plus invariants that hold at any size."""
import json
import os

import numpy as np
import pytest

from oracle import graphs as OG
from oracle import transfer as OT
from paper_1005_3609_amd import api, host
from paper_1005_3609_amd import workloads as W

pytestmark = pytest.mark.gpu

P31 = 2 ** 31 - 1
HERE = os.path.dirname(os.path.abspath(__file__))
MODES = ["plain", "batched", "graph", "grouped", "resident"]


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def _sampled(res, g):
    """res [n][nq][np] -> [n][len(sample)] for the golden file's instances."""
    flat = res.reshape(res.shape[0], -1)
    return flat[:, g["instance_index"]].astype(np.int64)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    yield


# ---------------------------------------------------------------------------
# The 4 x 5 square rectangle, q = 0..20, p = 2^31 - 1
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", MODES)
def test_square_4x5_all_q(mode):
    q = list(range(21))
    got = api.strip("square", 4, 5, q, [P31], mode=mode).astype(np.int64)
    np.testing.assert_array_equal(got, OT.chromatic_grid("square", 4, 5, q, [P31]))
    exact = OG.chromatic_by_colour_classes("square", 4, 5)
    V, E = OG.lattice_graph("square", 4, 5)
    assert [int(x) for x in got[-1, :, 0]] == [OG.poly_eval(exact, qq) % P31 for qq in q]
    # brute-force colour counts where they are cheap
    V3, E3 = OG.lattice_graph("square", 4, 3)
    for qq in range(4):
        assert int(got[2, qq, 0]) == OG.count_colourings(V3, E3, qq) % P31


def test_square_4x5_interpolates_to_the_exact_polynomial():
    q = list(range(21))
    got = api.strip("square", 4, 5, q, [P31], mode="batched")
    coeffs, _ = host.exact_polynomial(q, got[-1], [P31])
    assert coeffs == OT.chromatic_exact("square", 4, 5)[-1]
    assert coeffs[20] == 1 and coeffs[19] == -31 and coeffs[18] == 465 and coeffs[0] == 0


# ---------------------------------------------------------------------------
# Small widths, every path, ragged instance counts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat", ["square", "triangular"])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_small_widths_all_paths(lat, m):
    q = list(range(0, 35))                      # 35 x 2 = 70 instances: ragged chunks
    p = [P31, 1000000007]
    want = OT.chromatic_grid(lat, m, 6, q, p)
    for mode in MODES:
        got = api.strip(lat, m, 6, q, p, mode=mode).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=mode)


@pytest.mark.parametrize("tune", [
    dict(lanes_v=1, targets_per_wave=1, waves_per_block=1),
    dict(lanes_v=1, targets_per_wave=16, waves_per_block=8, xcd_order=2),
    dict(lanes_v=2, targets_per_wave=4, waves_per_block=2),
    dict(lanes_v=4, targets_per_wave=8, waves_per_block=4, xcd_order=2),
    dict(lanes_v=4, targets_per_wave=63, waves_per_block=1),
    dict(lanes_v=2, targets_per_wave=33, waves_per_block=8, xcd_order=2),
    dict(lanes_v=1, targets_per_wave=8, waves_per_block=4, unroll=8, streams=2),
    dict(lanes_v=2, targets_per_wave=5, waves_per_block=2, unroll=8, streams=4),
    dict(lanes_v=4, targets_per_wave=16, waves_per_block=4, unroll=8, streams=3, xcd_order=2),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=4, unroll=8, streams=3, fuse=2),
    dict(lanes_v=1, targets_per_wave=3, waves_per_block=8, fuse=3),
    dict(lanes_v=4, targets_per_wave=8, waves_per_block=2, unroll=8, streams=2, fuse=3),
    dict(lanes_v=1, targets_per_wave=1, waves_per_block=1, xcd_order=3, fuse=2),
    dict(lanes_v=2, targets_per_wave=2, waves_per_block=1, xcd_order=4, streams=3, fuse=2),
    dict(lanes_v=2, targets_per_wave=4, waves_per_block=4, fuse=2, stage=1),
    dict(lanes_v=1, targets_per_wave=3, waves_per_block=8, unroll=8, stage=1),
    dict(lanes_v=2, targets_per_wave=16, waves_per_block=2, streams=3, fuse=3, stage=1),
    dict(lanes_v=1, targets_per_wave=1, waves_per_block=1, fuse=2, stage=1, xcd_order=3),
    dict(lanes_v=4, targets_per_wave=8, waves_per_block=4, stage=1),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=2, stage=2),
    dict(lanes_v=1, targets_per_wave=4, waves_per_block=4, stage=2, streams=3),
    dict(lanes_v=2, targets_per_wave=16, waves_per_block=2, fuse=3, stage=2, xcd_order=2),
    dict(lanes_v=1, targets_per_wave=1, waves_per_block=1, fuse=2, stage=2, xcd_order=3),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=2, stage=3),
    dict(lanes_v=1, targets_per_wave=4, waves_per_block=4, stage=3, streams=3),
    dict(lanes_v=2, targets_per_wave=16, waves_per_block=2, fuse=3, stage=3, xcd_order=2),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=2, stage=4, streams=3),
    dict(lanes_v=1, targets_per_wave=4, waves_per_block=4, stage=4, xcd_order=2),
    dict(lanes_v=4, targets_per_wave=16, waves_per_block=2, fuse=3, stage=4),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=2, stage=5, streams=3),
    dict(lanes_v=1, targets_per_wave=4, waves_per_block=4, stage=5, xcd_order=2),
    dict(lanes_v=2, targets_per_wave=16, waves_per_block=2, fuse=2, stage=5),
    dict(lanes_v=2, targets_per_wave=1, waves_per_block=1, stage=5, xcd_order=4),
    dict(lanes_v=1, targets_per_wave=63, waves_per_block=8, fuse=2, stage=5),
    dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=2, stage=6, streams=3),
    dict(lanes_v=1, targets_per_wave=3, waves_per_block=4, stage=6, xcd_order=3),
    dict(lanes_v=4, targets_per_wave=16, waves_per_block=2, fuse=3, stage=6),
])
def test_tuning_choices_are_bit_identical(tune):
    q = list(range(1, 66))                      # 65 q x 2 p = 130 instances
    p = [P31, 998244353]
    want = OT.chromatic_grid("square", 7, 5, q, p)
    for mode in ("batched", "graph", "grouped"):
        if mode == "grouped" and tune.get("stage", 0) not in (0, 4, 6):
            # grouped launches gather directly: only the target orders apply
            with pytest.raises(api.ChromError, match="stage 0, 4 or 6"):
                api.strip("square", 7, 5, q, p, mode=mode, tuning=tune)
            continue
        got = api.strip("square", 7, 5, q, p, mode=mode, tuning=tune).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=f"{mode} {tune}")


@pytest.mark.parametrize("nq", [41, 38, 64, 144, 57])
def test_lanes_v4_instance_split(nq):
    # 41 q x 8 p = 328 instances: 256 at lanes_v 4 and 72 at lanes_v 2 on a
    # parallel branch; 38 x 8 = 304: the 48 left run at lanes_v 1; 64 x 8 =
    # 512: no split; 144 x 8 = 1152: four chunks of 256 (four chunk-group
    # chains at streams 4) and 128 left; 57 x 8 = 456: 200 left.  Same
    # residues as the oracle in every mode and shape.
    q, p = list(range(1, nq + 1)), [P31, 998244353, 1000000007, 2147483629, 2147483587, 1000000009,
                                    998244853, 2147483563]
    want = OT.chromatic_grid("square", 7, 5, q, p)
    for tune in (dict(lanes_v=4), dict(lanes_v=4, streams=2, fuse=2, stage=6, targets_per_wave=8),
                 dict(lanes_v=4, streams=3, fuse=2, stage=4), dict(lanes_v=4, streams=4, fuse=2, stage=6)):
        for mode in ("batched", "graph"):
            got = api.strip("square", 7, 5, q, p, mode=mode, tuning=tune).astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"{nq} {mode} {tune}")
    # the factor launches alone (the bench's roofline leg) run both jobs
    import torch
    tune = dict(lanes_v=4, fuse=2, stage=6)
    out, ws = api.strip_async("square", 7, 5, q, p, mode="batched", tuning=tune)
    api.factor_launches("square", 7, q, p, 2, ws, tune)
    torch.cuda.synchronize()


@pytest.mark.parametrize("lat,m,np_", [("square", 5, 8), ("triangular", 4, 3)])
def test_graph_mode_long_strips(lat, m, np_):
    # 69 rows: graphs of up to 32 rows (a multiple of two when a row has an
    # odd number of launches) replayed twice, the remaining rows run eagerly
    # after them; every chunk group is a chain with its own row counter, and
    # 41 x 8 = 328 instances split at lanes_v 4.  Every row equals the oracle,
    # on the first call (capture) and on a replay of the cached graphs.
    import torch
    q = list(range(1, 42))
    p = [P31, 998244353, 1000000007, 2147483629, 2147483587, 1000000009, 998244853, 2147483563][:np_]
    want = OT.chromatic_grid(lat, m, 70, q, p)
    for tune in (dict(lanes_v=4, streams=2, fuse=2, stage=6, targets_per_wave=8),
                 dict(lanes_v=2, streams=3, fuse=1),
                 dict(lanes_v=1, streams=2, fuse=3, stage=4)):
        out, ws = api.strip_async(lat, m, 70, q, p, mode="graph", tuning=tune)
        for call in range(2):
            if call:
                out.zero_()
                api.strip_async(lat, m, 70, q, p, mode="graph", tuning=tune, workspace=ws, out=out)
            torch.cuda.synchronize()
            got = api.to_u32(out).astype(np.int64).reshape(70, len(q), len(p))
            np.testing.assert_array_equal(got, want, err_msg=f"{lat} {m} {tune} call {call}")


def test_edge_cases():
    # m = 1 paths, n_max = 1, one instance, q >= p, q = 0
    for lat in ("square", "triangular"):
        for mode in MODES:
            got = api.strip(lat, 1, 7, [0, 3, P31 + 5], [P31], mode=mode).astype(np.int64)
            np.testing.assert_array_equal(got, OT.chromatic_grid(lat, 1, 7, [0, 3, 5], [P31]))
            got = api.strip(lat, 6, 1, [4], [101], mode=mode).astype(np.int64)
            np.testing.assert_array_equal(got, OT.chromatic_grid(lat, 6, 1, [4], [101]))
    assert api.strip("square", 5, 0, [3], [P31], mode="batched").shape == (0, 1, 1)


def test_repeat_runs_identical():
    q, p = list(range(1, 40)), [P31]
    a = api.strip("triangular", 9, 7, q, p, mode="grouped")
    for _ in range(3):
        assert np.array_equal(api.strip("triangular", 9, 7, q, p, mode="grouped"), a)
        assert np.array_equal(api.strip("triangular", 9, 7, q, p, mode="graph"), a)


# ---------------------------------------------------------------------------
# Workload: square m = 10, n = 1..11, q = 1..80 x 4 primes (plain path)
# ---------------------------------------------------------------------------
def test_square_m10_plain_and_batched():
    w = W.workload("square_m10")
    lat, m, n = w["strips"][0]
    want = OT.chromatic_grid(lat, m, n, w["q_points"], w["primes"])
    for mode in ("plain", "batched", "resident"):
        got = api.strip(lat, m, n, w["q_points"], w["primes"], mode=mode).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=mode)


# ---------------------------------------------------------------------------
# Workload: triangular m = 12, n = 1..13, 48 q x 6 primes (graph + grouped)
# ---------------------------------------------------------------------------
def test_triangular_m12_against_stored_oracle():
    w = W.workload("triangular_m12")
    g = _golden("oracle_triangular_12x13.json")
    for mode in ("graph", "grouped", "resident"):
        got = api.strip("triangular", 12, 13, w["q_points"], w["primes"], mode=mode)
        np.testing.assert_array_equal(_sampled(got, g), np.array(g["z"], dtype=np.int64), err_msg=mode)
        # invariants at every length: P(1) = 0; P(2) = 0 and P(3) = 6 for r >= 2
        flat = got.reshape(13, 48, 6).astype(np.int64)
        assert (flat[:, 0, :] == 0).all()
        assert (flat[1:, 1, :] == 0).all() and (flat[1:, 2, :] == 6).all()


# ---------------------------------------------------------------------------
# Workload: square m = 2..14, n <= m+1, 80 q x 8 primes, one graph of grouped launches
# ---------------------------------------------------------------------------
def test_square_sweep_one_launch():
    import torch
    w = W.workload("square_sweep_2_14")
    jobs = [dict(lattice=lat, m=m, n_max=n, q_points=w["q_points"], primes=w["primes"])
            for lat, m, n in w["strips"]]
    outs, ws = api.batch(jobs)
    torch.cuda.synchronize()
    res = {jb["m"]: api.to_u32(o).astype(np.int64) for jb, o in zip(jobs, outs)}
    sample = W.sample_instances(640, 24, 5)
    qs = [w["q_points"][k // 8] for k in sample]
    ps = [w["primes"][k % 8] for k in sample]
    for m in range(2, 11):
        want = OT.chromatic_residues("square", m, m + 1, qs, ps)
        got = res[m].reshape(m + 1, -1)[:, sample]
        np.testing.assert_array_equal(got, want, err_msg=f"m={m}")
    for m in range(11, 15):
        g = _golden(f"oracle_square_{m}x{m + 1}.json")
        np.testing.assert_array_equal(_sampled(res[m], g), np.array(g["z"], dtype=np.int64), err_msg=f"m={m}")
    for m in range(2, 15):
        z = res[m].reshape(m + 1, 80, 8)
        assert (z[:, 0, :] == 0).all() and (z[:, 1, :] == 2).all()   # P(1) = 0, P(2) = 2
    # transposition: P(m x (m+1)) from width m equals P((m+1) x m) from width m+1
    for m in range(2, 14):
        np.testing.assert_array_equal(res[m][m], res[m + 1][m - 1])


# ---------------------------------------------------------------------------
# Square 14 x 15, 640 instances, in the configurations the benchmark times:
# graph row replay with the tuned launch shape (its step) and batched launches
# on one stream (its roofline leg), then the roofline's bare factor launches
# ---------------------------------------------------------------------------
def test_square_14x15_benchmark_configurations():
    import torch
    from paper_1005_3609_amd import tune as tuner
    w = W.workload("square_14x15")
    q, p = w["q_points"], w["primes"]
    g = _golden("oracle_square_14x15.json")
    tune = dict(tuner.lookup_tuned("square", 14, 640, 15) or {})
    tune.pop("mode", None)
    tune.pop("ms", None)
    want = np.array(g["z"], dtype=np.int64)
    for mode, t in (("graph", tune), ("batched", dict(tune, streams=1))):
        out, ws = api.strip_async("square", 14, 15, q, p, mode=mode, tuning=t)
        torch.cuda.synchronize()
        res = api.to_u32(out).astype(np.int64)
        np.testing.assert_array_equal(_sampled(res, g), want, err_msg=f"{mode} {t}")
        z = res.reshape(15, 80, 8)
        assert (z[:, 0, :] == 0).all() and (z[:, 1, :] == 2).all()
        if mode == "batched":
            # the bare factor launches leave the strip's output untouched
            stream = torch.cuda.current_stream()
            api.factor_launches("square", 14, q, p, 2, ws, t, stream)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(api.to_u32(out).astype(np.int64), res)
        del ws


# ---------------------------------------------------------------------------
# Square 18 x 19 (the large-state run), 640 instances, in the launch shape the
# benchmark times (graph row replay, tuned): sampled instances against stored
# oracle residues on every row the file holds, and the q = 3 column of every
# row and prime against exact 3-colouring counts of the 18 x r rectangles
# ---------------------------------------------------------------------------
def _three_colourings(lat, m):
    want = {}
    with open(os.path.join(HERE, "golden", f"{lat}_three_colourings_m{m}.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                _, mm, r, qq, val = line.split()
                assert int(mm) == m and int(qq) == 3
                want[int(r)] = int(val)
    return want


def test_square_18x19_benchmark_shape_against_oracle():
    import torch
    from paper_1005_3609_amd import tune as tuner
    w = W.workload("square_18x19")
    q, p = w["q_points"], w["primes"]
    g = _golden("oracle_square_18x19.json")
    tune = dict(tuner.lookup_tuned("square", 18, len(q) * len(p), 19) or {})
    mode = tune.pop("mode", "graph")
    tune.pop("ms", None)
    out, ws = api.strip_async("square", 18, 19, q, p, mode=mode, tuning=tune)
    torch.cuda.synchronize()
    res = api.to_u32(out).astype(np.int64)
    rows = g.get("rows_present", 19)
    np.testing.assert_array_equal(_sampled(res, g)[:rows], np.array(g["z"], dtype=np.int64)[:rows])
    z = res.reshape(19, len(q), len(p))
    assert (z[:, q.index(1), :] == 0).all() and (z[:, q.index(2), :] == 2).all()
    three = _three_colourings("square", 18)
    want = np.array([[three[r] % pp for pp in p] for r in range(1, 20)], dtype=np.int64)
    np.testing.assert_array_equal(z[:, q.index(3), :], want)
    del ws


# ---------------------------------------------------------------------------
# Resident mode: the whole strip in one launch, state vectors in LDS (the
# square 4 x 5 case and the m = 5 strips once ran a work-queue design that
# stalled; this kernel has no inter-workgroup waits)
# ---------------------------------------------------------------------------
def test_resident_square_4x5():
    q = list(range(21))
    got = api.strip("square", 4, 5, q, [P31], mode="resident").astype(np.int64)
    np.testing.assert_array_equal(got, OT.chromatic_grid("square", 4, 5, q, [P31]))


@pytest.mark.parametrize("lat", ["square", "triangular"])
def test_resident_small_widths(lat):
    q, p = list(range(0, 35)), [P31, 1000000007]
    got = api.strip(lat, 5, 6, q, p, mode="resident").astype(np.int64)
    np.testing.assert_array_equal(got, OT.chromatic_grid(lat, 5, 6, q, p))


@pytest.mark.parametrize("tune", [
    dict(lanes_v=1, waves_per_block=1),
    dict(lanes_v=1, waves_per_block=16),
    dict(lanes_v=2, waves_per_block=4),
    dict(lanes_v=4, waves_per_block=8),
    dict(lanes_v=4, waves_per_block=2, fuse=2),
    dict(lanes_v=1, waves_per_block=8, fuse=2),
    dict(lanes_v=2, waves_per_block=16, fuse=3),
    dict(lanes_v=1, waves_per_block=4, fuse=3),
    # modular arithmetic throughout (stage 0 takes exact double accumulation
    # wherever its bound holds: every case above but some fused triples)
    dict(lanes_v=1, waves_per_block=16, stage=1),
    dict(lanes_v=2, waves_per_block=8, fuse=2, stage=1),
    dict(lanes_v=4, waves_per_block=4, fuse=3, stage=1),
])
@pytest.mark.parametrize("lat", ["square", "triangular"])
def test_resident_tuning_choices_are_bit_identical(lat, tune):
    q = list(range(1, 44))                      # 43 q x 3 p = 129 instances: ragged groups at lanes_v 2, 4
    p = [P31, 998244353, 1000000007]
    want = OT.chromatic_grid(lat, 7, 5, q, p)
    got = api.strip(lat, 7, 5, q, p, mode="resident", tuning=tune).astype(np.int64)
    np.testing.assert_array_equal(got, want, err_msg=f"{lat} {tune}")


@pytest.mark.parametrize("lat", ["square", "triangular"])
def test_resident_large_q_leaves_the_double_form(lat):
    # q near 2^31 and past it: |c(q)| exceeds the double form's bound, so
    # stage 0 runs these jobs in modular arithmetic; small q alongside
    q = [2, 5, 2**31 - 1, 3_000_000_000, 4_294_967_295]
    p = [P31, 998244353]
    want = OT.chromatic_grid(lat, 6, 5, q, p)
    for tune in (dict(lanes_v=2, waves_per_block=8), dict(lanes_v=2, waves_per_block=8, stage=1),
                 dict(lanes_v=1, waves_per_block=8, stage=0)):
        got = api.strip(lat, 6, 5, q, p, mode="resident", tuning=tune).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=f"{lat} {tune}")
    # the small q alone take the double form
    got = api.strip(lat, 6, 5, q[:2], p, mode="resident").astype(np.int64)
    np.testing.assert_array_equal(got, OT.chromatic_grid(lat, 6, 5, q[:2], p))


def test_resident_largest_widths():
    # the widest strips whose vectors fit: square m = 12 and triangular m = 13
    # (one instance per workgroup), against the live oracle on a few instances
    for lat, m in (("square", 12), ("triangular", 13)):
        q, p = [1, 2, 3, 7, 40], [P31, 998244353]
        want = OT.chromatic_grid(lat, m, 4, q, p)
        got = api.strip(lat, m, 4, q, p, mode="resident", tuning=dict(lanes_v=1, waves_per_block=16))
        np.testing.assert_array_equal(got.astype(np.int64), want, err_msg=f"{lat} {m}")


@pytest.mark.parametrize("stage", [1, 2, 3, 4])
def test_staged_tiles_with_rows_past_the_lds_slots(stage):
    # square m = 11 fused triples have rows reading up to 137 distinct
    # sources, more than the 96 LDS slots of a staged tile at lanes_v 2:
    # such a row's tile reads its remaining sources straight from memory
    q, p = list(range(1, 33)), [P31, 998244353]
    want = OT.chromatic_grid("square", 11, 4, q, p)
    for mode in ("batched", "graph"):
        tune = dict(lanes_v=2, targets_per_wave=8, waves_per_block=8, fuse=3, stage=stage)
        got = api.strip("square", 11, 4, q, p, mode=mode, tuning=tune).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=f"{mode} stage {stage}")


# ---------------------------------------------------------------------------
# Op-stream gathers (stage 5): unit-coefficient factors only
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lat,m,fuse", [("square", 11, 2), ("square", 9, 1), ("triangular", 9, 1)])
def test_op_stream_gathers(lat, m, fuse):
    # streams of every length (targets_per_wave 1..63 rows), rows longer than
    # a sixteen-word block (fused pairs at m = 11 read up to 46 sources)
    q, p = list(range(1, 41)), [P31, 998244353, 1000000007]
    want = OT.chromatic_grid(lat, m, 4, q, p)
    for tpw, wpb in ((1, 1), (7, 4), (16, 8), (63, 2)):
        for mode in ("batched", "graph"):
            tune = dict(lanes_v=2 if tpw != 7 else 1, targets_per_wave=tpw, waves_per_block=wpb, fuse=fuse,
                        stage=5)
            got = api.strip(lat, m, 4, q, p, mode=mode, tuning=tune).astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"{mode} {tune}")


@pytest.mark.parametrize("xcd", [5, 6])
def test_xcd_runs_of_64_and_256_tiles(xcd):
    # one wavefront per tile and workgroup: about 8000 tiles per chunk, so
    # whole rounds of 8 x 64 and 8 x 256 remapped ids and a ragged rest
    q, p = list(range(1, 70)), [P31]
    want = OT.chromatic_grid("square", 11, 3, q, p)
    for mode in ("batched", "graph", "grouped"):
        tune = dict(lanes_v=1, targets_per_wave=1, waves_per_block=1, xcd_order=xcd, fuse=2)
        got = api.strip("square", 11, 3, q, p, mode=mode, tuning=tune).astype(np.int64)
        np.testing.assert_array_equal(got, want, err_msg=f"{mode} {tune}")


def test_op_stream_gathers_refuse_other_coefficients():
    # fused triples of the square lattice and fused pairs of the triangular
    # lattice have digits beyond +-1 or a t^3 term: refused, not approximated
    for lat, fuse in (("square", 3), ("triangular", 2)):
        with pytest.raises(api.ChromError, match="unit coefficients"):
            api.strip(lat, 7, 3, [1, 2, 3], [P31], mode="batched", tuning=dict(fuse=fuse, stage=5))


# ---------------------------------------------------------------------------
# The grouped mode's cached graph reads its stage tables from the caller's
# workspace: an identical call on a workspace overwritten in between (same
# address, as a caching allocator hands it back) must upload them again
# ---------------------------------------------------------------------------
def test_grouped_graph_reuploads_its_tables_into_a_reused_workspace():
    import torch
    q, p = list(range(1, 30)), [P31, 998244353]
    want = OT.chromatic_grid("square", 6, 5, q, p)
    for mode in ("grouped", "graph"):
        out, ws = api.strip_async("square", 6, 5, q, p, mode=mode, tuning=dict(fuse=2))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(api.to_u32(out).astype(np.int64), want, err_msg=mode)
        for fill in (0xFF, 0x00):
            ws.fill_(fill)
            out.zero_()
            api.strip_async("square", 6, 5, q, p, mode=mode, tuning=dict(fuse=2), workspace=ws, out=out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(api.to_u32(out).astype(np.int64), want, err_msg=f"{mode} fill {fill}")
