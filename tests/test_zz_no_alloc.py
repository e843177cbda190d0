"""The no-allocation strip (chromatic_strip_noalloc, workspace in the
library's device array) against chromatic_strip_async in the batched mode,
bit for bit, on two calls in a row (the second with a smaller strip and fewer
instances), through the C ABI."""
import ctypes as C

import numpy as np
import pytest

from paper_1005_3609_amd import _lib, api
from paper_1005_3609_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(lat, m, n, q, p, tune=None):
    import torch
    qa = np.ascontiguousarray(q, dtype=np.uint32)
    pa = np.ascontiguousarray(p, dtype=np.uint32)
    out = torch.full((n, qa.size, pa.size), -1, dtype=torch.int32, device="cuda")
    t = _lib.tuning(tune)
    stream = torch.cuda.current_stream()
    rc = api.lib().chromatic_strip_noalloc(api.lattice_id(lat), m, n, qa.ctypes.data_as(C.c_void_p), qa.size,
                                           pa.ctypes.data_as(C.c_void_p), pa.size, C.byref(t) if t else None,
                                           C.c_void_p(stream.cuda_stream), C.c_void_p(out.data_ptr()))
    api.check(rc)
    torch.cuda.synchronize()
    return api.to_u32(out)


def _async(lat, m, n, q, p, tune=None):
    import torch
    out, ws = api.strip_async(lat, m, n, q, p, mode="batched", tuning=tune)
    torch.cuda.synchronize()
    return api.to_u32(out)


def test_noalloc_matches_strip_async_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    w = W.workload("square_sweep_2_14")
    big = ("square", 12, 13, w["q_points"], w["primes"])            # 640 instances, 56 MB of workspace
    small = ("triangular", 7, 6, list(range(0, 35)), [2 ** 31 - 1, 998244353])
    for lat, m, n, q, p in (big, small):
        api.prepare(lat, m)
        want = _async(lat, m, n, q, p)
        got = _noalloc(lat, m, n, q, p)
        np.testing.assert_array_equal(got, want, err_msg=f"{lat} {m}x{n}")


def test_noalloc_fused_family_and_launch_shape():
    # a fused family becomes usable once another entry point has built it
    q, p = list(range(1, 41)), [2 ** 31 - 1, 1000000007, 998244353]
    tune = dict(lanes_v=1, targets_per_wave=4, waves_per_block=4, fuse=2)
    api.prepare("square", 9)
    want = _async("square", 9, 8, q, p, tune)
    np.testing.assert_array_equal(_noalloc("square", 9, 8, q, p, tune), want)
    np.testing.assert_array_equal(_noalloc("square", 9, 8, q, p), want)   # single factors, same residues


def test_noalloc_refuses_what_it_cannot_do():
    w = W.workload("square_14x15")
    api.prepare("square", 14)
    with pytest.raises(api.ChromError, match="bytes of workspace"):
        _noalloc("square", 14, 15, w["q_points"], w["primes"])           # 294 MB of vectors
    with pytest.raises(api.ChromError, match="one stream"):
        _noalloc("square", 5, 3, [3], [101], dict(streams=3))
    with pytest.raises(api.ChromError, match="at most"):
        _noalloc("square", 5, 3, list(range(600)), [101])
