"""Python front end of the chromatic-strip library: argument marshalling only.

Every step of the sweep runs in the native library (``libchromstrip.so``);
PyTorch supplies device memory and streams for the asynchronous calls.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import ChromError, check, lib  # noqa: F401  (re-exported)

LATTICES = {"square": _lib.SQUARE, "triangular": _lib.TRIANGULAR, 0: 0, 1: 1}


def lattice_id(lat) -> int:
    try:
        return LATTICES[lat]
    except KeyError:
        raise ValueError(f"unknown lattice {lat!r}") from None


def _u32(a) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    if arr.size and (arr.min() < 0 or arr.max() >= 2 ** 32):
        raise ValueError("values must fit in uint32")
    return arr.astype(np.uint32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# Synchronous whole-strip calls (host buffers)
# ---------------------------------------------------------------------------
def strip(lattice, m: int, n_max: int, q_points, primes, mode: str = "plain", tuning=None) -> np.ndarray:
    """Residues P_{m x r}(q_a) mod p_b, shape [n_max, nq, np], dtype uint32."""
    q = _u32(q_points)
    p = _u32(primes)
    out = np.zeros((max(n_max, 0), q.size, p.size), dtype=np.uint32)
    L = lib()
    if mode == "plain":
        check(L.chromatic_strip(lattice_id(lattice), m, n_max, _ptr(q), q.size, _ptr(p), p.size, _ptr(out)))
    else:
        t = _lib.tuning(tuning)
        check(L.chromatic_strip_batched(lattice_id(lattice), m, n_max, _ptr(q), q.size, _ptr(p), p.size,
                                        _lib.MODES[mode], C.byref(t) if t else None, _ptr(out)))
    return out


# ---------------------------------------------------------------------------
# Coefficient form: the normalised polynomial P~ = q^-|V| P in x = 1/q
# ---------------------------------------------------------------------------
def series(lattice, m: int, n_max: int, d_max: int, primes, mode: str = "graph", tuning=None) -> np.ndarray:
    """Coefficients of x^0..x^d_max of P~ for the m x r rectangles, r =
    1..n_max, mod every prime: uint32 [n_max, np, d_max + 1]."""
    p = _u32(primes)
    out = np.zeros((max(n_max, 0), p.size, d_max + 1), dtype=np.uint32)
    t = _lib.tuning(tuning)
    check(lib().chromatic_series(lattice_id(lattice), m, n_max, d_max, _ptr(p), p.size, _lib.MODES[mode],
                                 C.byref(t) if t else None, _ptr(out)))
    return out


def series_workspace_bytes(lattice, m: int, n_max: int, np_: int, d_max: int, mode: str = "graph",
                           tuning=None) -> int:
    t = _lib.tuning(tuning)
    n = lib().chromatic_series_workspace_bytes(lattice_id(lattice), m, n_max, np_, d_max, _lib.MODES[mode],
                                               C.byref(t) if t else None)
    if n == 0:
        check(-1)
    return int(n)


def series_async(lattice, m: int, n_max: int, d_max: int, primes, mode: str = "graph", tuning=None,
                 workspace=None, out=None, stream=None, device=None):
    """Queues a coefficient-form strip on `stream`; returns (out, workspace),
    out = int32 storage of uint32 [n_max, np, d_max + 1]."""
    torch = _torch()
    p = _u32(primes)
    t = _lib.tuning(tuning)
    need = series_workspace_bytes(lattice, m, n_max, p.size, d_max, mode, tuning)
    if workspace is None:
        workspace = alloc_workspace(need, device)
    if out is None:
        out = torch.zeros((max(n_max, 1), p.size, d_max + 1), dtype=torch.int32, device=workspace.device)
    check(lib().chromatic_series_async(lattice_id(lattice), m, n_max, d_max, _ptr(p), p.size, _lib.MODES[mode],
                                       C.byref(t) if t else None, C.c_void_p(workspace.data_ptr()),
                                       workspace.numel(), _stream_handle(stream), C.c_void_p(out.data_ptr())))
    return out, workspace


def code_table(lattice, m: int, normalised: bool = False) -> np.ndarray:
    """int64 [n_codes, 4]: coefficients of z^0..z^3 of every code (z = q, or
    x = 1/q for the normalised maps)."""
    L = lib()
    n = C.c_int()
    check(L.chromatic_code_table(lattice_id(lattice), m, int(normalised), C.byref(n), None))
    out = np.zeros((n.value, 4), dtype=np.int64)
    check(L.chromatic_code_table(lattice_id(lattice), m, int(normalised), None, _ptr(out)))
    return out


def prepare(lattice, m: int) -> None:
    check(lib().chromatic_prepare(lattice_id(lattice), m))


def prepare_series(lattice, m: int) -> None:
    """Coefficient-form maps of (lattice, m) on the current device ahead of
    time (the first series call would build them itself)."""
    check(lib().chromatic_prepare_series(lattice_id(lattice), m))


def series_map_info(lattice, m: int, which: int, idx: int):
    """(rows, columns, entries) of a coefficient-form map on the current
    device, without copying it; which 4 = forward, 5 = read-out factor."""
    nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
    check(lib().chromatic_series_map_export(lattice_id(lattice), m, which, idx, C.byref(nr), C.byref(nc), C.byref(nz),
                                            None, None))
    return int(nr.value), int(nc.value), int(nz.value)


def series_map_export(lattice, m: int, which: int, idx: int):
    """The coefficient-form map the current device holds: (row_ptr int32,
    entries uint32, n_cols); which 4 = forward, 5 = read-out factor."""
    L = lib()
    nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
    check(L.chromatic_series_map_export(lattice_id(lattice), m, which, idx, C.byref(nr), C.byref(nc), C.byref(nz),
                                        None, None))
    rp = np.zeros(nr.value + 1, dtype=np.int32)
    ent = np.zeros(max(nz.value, 1), dtype=np.uint32)
    check(L.chromatic_series_map_export(lattice_id(lattice), m, which, idx, None, None, None, _ptr(rp), _ptr(ent)))
    return rp, ent[: nz.value], int(nc.value)


def prepare_host(lattice, m: int, normalised: bool = False) -> None:
    """Host maps of (lattice, m) only (no device).  Builds are serialized in
    the library; call it from the thread that makes the other library calls
    (concurrent use from a second thread is not supported)."""
    check(lib().chromatic_prepare_host(lattice_id(lattice), m, 1 if normalised else 0))


def check_expansion(lattice, m: int, normalised: bool = True) -> None:
    """Raises ChromError unless the device map builder's expansion, run on the
    host, reproduces the host builder's maps of (lattice, m) (paper order)."""
    check(lib().chromatic_check_expansion(lattice_id(lattice), m, 1 if normalised else 0))


def release_maps() -> None:
    lib().chromatic_release_maps()


def device_status(stream=None) -> None:
    check(lib().chromatic_device_status(_stream_handle(stream)))


# ---------------------------------------------------------------------------
# Asynchronous calls on torch-managed device memory
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream_handle(stream):
    if stream is None:
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def workspace_bytes(lattice, m: int, n_max: int, nq: int, np_: int, mode: str = "batched", tuning=None) -> int:
    t = _lib.tuning(tuning)
    n = lib().chromatic_workspace_bytes(lattice_id(lattice), m, n_max, nq, np_, _lib.MODES[mode],
                                        C.byref(t) if t else None)
    if n == 0:
        check(-1)
    return int(n)


def alloc_workspace(nbytes: int, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def strip_async(lattice, m: int, n_max: int, q_points, primes, mode: str = "batched", tuning=None,
                workspace=None, out=None, stream=None, device=None):
    """Queues the strip on `stream` (default: torch's current stream).
    Returns the output tensor (int32 storage of uint32 residues,
    [n_max, nq, np]) and the workspace tensor; both must stay alive until the
    stream has run the work."""
    torch = _torch()
    q = _u32(q_points)
    p = _u32(primes)
    t = _lib.tuning(tuning)
    need = workspace_bytes(lattice, m, n_max, q.size, p.size, mode, tuning)
    if workspace is None:
        workspace = alloc_workspace(need, device)
    if out is None:
        out = torch.zeros((max(n_max, 1), q.size, p.size), dtype=torch.int32, device=workspace.device)
    check(lib().chromatic_strip_async(lattice_id(lattice), m, n_max, _ptr(q), q.size, _ptr(p), p.size,
                                      _lib.MODES[mode], C.byref(t) if t else None,
                                      C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                      _stream_handle(stream), C.c_void_p(out.data_ptr())))
    return out, workspace


def factor_launches(lattice, m: int, q_points, primes, rows: int, workspace, tuning=None, stream=None) -> None:
    """Queues rows x m factor-kernel launches on a workspace that
    strip_async(mode="batched") has used with the same arguments."""
    q = _u32(q_points)
    p = _u32(primes)
    t = _lib.tuning(tuning)
    check(lib().chromatic_factor_launches(lattice_id(lattice), m, _ptr(q), q.size, _ptr(p), p.size, rows,
                                          C.byref(t) if t else None, C.c_void_p(workspace.data_ptr()),
                                          workspace.numel(), _stream_handle(stream)))


def to_u32(t) -> np.ndarray:
    """Device int32 tensor of residues -> host uint32 array."""
    return t.detach().cpu().numpy().view(np.uint32)


# ---------------------------------------------------------------------------
# Many jobs in one graph of grouped launches
# ---------------------------------------------------------------------------
def _job_structs(jobs, outs):
    arr = (_lib.Job * len(jobs))()
    keep = []
    for k, jb in enumerate(jobs):
        q = _u32(jb["q_points"])
        p = _u32(jb["primes"])
        keep += [q, p]
        arr[k].lattice = lattice_id(jb["lattice"])
        arr[k].m = int(jb["m"])
        arr[k].n_max = int(jb["n_max"])
        arr[k].q_points = q.ctypes.data_as(C.POINTER(C.c_uint32))
        arr[k].nq = q.size
        arr[k].primes = p.ctypes.data_as(C.POINTER(C.c_uint32))
        arr[k].np = p.size
        arr[k].d_out = C.c_void_p(outs[k].data_ptr()) if outs is not None else None
    return arr, keep


def batch_workspace_bytes(jobs, tuning=None) -> int:
    arr, _keep = _job_structs(jobs, None)
    t = _lib.tuning(tuning)
    n = lib().chromatic_batch_workspace_bytes(arr, len(jobs), C.byref(t) if t else None)
    if n == 0 and jobs:
        check(-1)
    return int(n)


def batch(jobs, tuning=None, workspace=None, outs=None, stream=None, device=None):
    """Runs every job (dicts with lattice, m, n_max, q_points, primes) as one
    hipGraph of grouped launches.  Returns (list of output tensors, workspace)."""
    torch = _torch()
    dev = device or "cuda"
    if outs is None:
        outs = [torch.zeros((max(int(jb["n_max"]), 1), len(jb["q_points"]), len(jb["primes"])),
                            dtype=torch.int32, device=dev) for jb in jobs]
    need = batch_workspace_bytes(jobs, tuning)
    if workspace is None:
        workspace = alloc_workspace(need, dev)
    arr, _keep = _job_structs(jobs, outs)
    t = _lib.tuning(tuning)
    check(lib().chromatic_batch(arr, len(jobs), C.byref(t) if t else None, C.c_void_p(workspace.data_ptr()),
                                workspace.numel(), _stream_handle(stream)))
    return outs, workspace


# ---------------------------------------------------------------------------
# Host-side introspection
# ---------------------------------------------------------------------------
def motzkin(k: int) -> int:
    return int(lib().chromatic_motzkin(k))


def space_size(m: int, space: int = _lib.SPACE_NCNNN, i: int = 0) -> int:
    n = int(lib().chromatic_space_size(m, space, i))
    if n < 0:
        check(n)
    return n


def rank(m: int, labels, space: int = _lib.SPACE_NCNNN, i: int = 0) -> int:
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.uint8))
    assert lab.size == m
    r = int(lib().chromatic_rank(m, space, i, _ptr(lab)))
    if r < -1:
        check(-1)
    return r


def unrank(m: int, r: int, space: int = _lib.SPACE_NCNNN, i: int = 0) -> tuple:
    lab = np.zeros(m, dtype=np.uint8)
    check(lib().chromatic_unrank(m, space, i, r, _ptr(lab)))
    return tuple(int(x) for x in lab)


def family_info(lattice, m: int, fuse: int = 1) -> dict:
    """Factor count and coefficient table of a factor family; codes are
    polynomials (c0, c1, c2, c3) in q."""
    nf, nc = C.c_int(), C.c_int()
    coef = np.zeros(64 * 4, dtype=np.int64)
    check(lib().chromatic_family_info(lattice_id(lattice), m, fuse, C.byref(nf), C.byref(nc), _ptr(coef)))
    return dict(n_factors=nf.value, codes=[tuple(int(x) for x in coef[4 * c:4 * c + 4]) for c in range(nc.value)])


def maps_info(lattice, m: int) -> dict:
    info = _lib.MapsInfo()
    check(lib().chromatic_maps_info(lattice_id(lattice), m, C.byref(info)))
    return dict(n_factors=info.n_factors, n_last=info.n_last, n_codes=info.n_codes,
                codes=family_info(lattice, m, 1)["codes"],
                total_nnz=int(info.total_nnz), max_states=int(info.max_states))


def stage_export(lattice, m: int, fuse: int, idx: int, slots: int, rows: int) -> dict:
    """Staged-tile form of forward factor idx of the fuse-sized family:
    dict(tile_row0, tile_src0, src, slots (int64[nnz]), codes (int64[nnz]),
    max_slots)."""
    L = lib()
    nt, ns, mx = C.c_int32(), C.c_int64(), C.c_int32()
    args = (lattice_id(lattice), m, fuse, idx, slots, rows)
    check(L.chromatic_stage_export(*args, C.byref(nt), C.byref(ns), C.byref(mx), None, None, None, None))
    rp, _, _, _ = map_export(lattice, m, 0 if fuse == 1 else fuse, idx)
    nnz = int(rp[-1])
    tr = np.zeros(nt.value + 1, dtype=np.int32)
    ts = np.zeros(nt.value + 1, dtype=np.int32)
    src = np.zeros(max(ns.value, 1), dtype=np.int32)
    ent = np.zeros(max(nnz, 1), dtype=np.uint32)
    check(L.chromatic_stage_export(*args, None, None, None, _ptr(tr), _ptr(ts), _ptr(src), _ptr(ent)))
    ent = ent[:nnz]
    return dict(tile_row0=tr, tile_src0=ts, src=src[: ns.value], slots=(ent & ((1 << 26) - 1)).astype(np.int64),
                codes=(ent >> 26).astype(np.int64), max_slots=int(mx.value))


def cluster_export(lattice, m: int, fuse: int, idx: int, slots: int, rows: int) -> dict:
    """Clustered staged-tile form of forward factor idx of the fuse-sized
    family: dict(tile_row0, tile_src0, src, tgt, row_ptr, slots, codes,
    max_slots)."""
    L = lib()
    nt, ns, mx = C.c_int32(), C.c_int64(), C.c_int32()
    args = (lattice_id(lattice), m, fuse, idx, slots, rows)
    check(L.chromatic_cluster_export(*args, C.byref(nt), C.byref(ns), C.byref(mx), *([None] * 6)))
    rp, _, _, _ = map_export(lattice, m, 0 if fuse == 1 else fuse, idx)
    n_rows, nnz = len(rp) - 1, int(rp[-1])
    tr = np.zeros(nt.value + 1, dtype=np.int32)
    ts = np.zeros(nt.value + 1, dtype=np.int32)
    src = np.zeros(max(ns.value, 1), dtype=np.int32)
    tgt = np.zeros(max(n_rows, 1), dtype=np.int32)
    crp = np.zeros(n_rows + 1, dtype=np.int32)
    ent = np.zeros(max(nnz, 1), dtype=np.uint32)
    check(L.chromatic_cluster_export(*args, None, None, None, _ptr(tr), _ptr(ts), _ptr(src), _ptr(tgt), _ptr(crp),
                                     _ptr(ent)))
    ent = ent[:nnz]
    return dict(tile_row0=tr, tile_src0=ts, src=src[: ns.value], tgt=tgt[:n_rows], row_ptr=crp,
                slots=(ent & ((1 << 26) - 1)).astype(np.int64), codes=(ent >> 26).astype(np.int64),
                max_slots=int(mx.value))


def op_export(lattice, m: int, fuse: int, idx: int) -> dict:
    """Op-stream form (tuning stage 5) of forward factor idx of the
    fuse-sized family: dict(shift, row_first int32[n_rows+1], words
    uint32[n_words], padding included)."""
    L = lib()
    sh, nw = C.c_int32(), C.c_int64()
    check(L.chromatic_op_export(lattice_id(lattice), m, fuse, idx, C.byref(sh), C.byref(nw), None, None))
    rp, _, _, _ = map_export(lattice, m, 0 if fuse == 1 else fuse, idx)
    rows = np.zeros(len(rp), dtype=np.int32)
    words = np.zeros(max(nw.value, 1), dtype=np.uint32)
    check(L.chromatic_op_export(lattice_id(lattice), m, fuse, idx, None, None, _ptr(rows), _ptr(words)))
    return dict(shift=int(sh.value), row_first=rows, words=words[: nw.value])


def map_export(lattice, m: int, which: int, idx: int):
    """(row_ptr int32[n_rows+1], cols int64[nnz], codes int64[nnz], n_cols);
    which: 0 forward factor, 1 read-out factor (transposed), 2/3 fused family,
    4 normalised forward factor, 5 normalised read-out factor (gather form)."""
    L = lib()
    nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
    check(L.chromatic_map_export(lattice_id(lattice), m, which, idx, C.byref(nr), C.byref(nc), C.byref(nz),
                                 None, None))
    rp = np.zeros(nr.value + 1, dtype=np.int32)
    ent = np.zeros(max(nz.value, 1), dtype=np.uint32)
    check(L.chromatic_map_export(lattice_id(lattice), m, which, idx, None, None, None, _ptr(rp), _ptr(ent)))
    ent = ent[: nz.value]
    return rp, (ent & ((1 << 26) - 1)).astype(np.int64), (ent >> 26).astype(np.int64), int(nc.value)
