"""Thin ctypes binding of libmrpt (include/mrpt.h), same names as the C ABI.

Only argument marshalling happens here: every step of the search runs in the
library's HIP kernels.  Device arrays are torch CUDA tensors (torch is used for
device memory and streams only).  There is no CPU fallback: if libmrpt.so is
missing or no GPU is present, calls raise.
"""
import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrpt.so")

MRPT_OK, MRPT_EINVAL, MRPT_ENOMEM, MRPT_EDEVICE, MRPT_ENONFINITE, MRPT_EINTERNAL = 0, -1, -2, -3, -4, -5
MRPT_FP32, MRPT_BF16_RERANK, MRPT_FP8_RERANK = 0, 1, 2
_STATUS = {0: "MRPT_OK", -1: "MRPT_EINVAL", -2: "MRPT_ENOMEM", -3: "MRPT_EDEVICE", -4: "MRPT_ENONFINITE",
           -5: "MRPT_EINTERNAL"}


class MrptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class mrpt_query_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rerank_factor", ctypes.c_int32),
                ("recheck_rel", ctypes.c_float), ("check_finite", ctypes.c_int32),
                ("s_count", ctypes.c_void_p), ("stage_events", ctypes.c_void_p)]


class mrpt_build_opts(ctypes.Structure):
    _fields_ = [("on_device", ctypes.c_int32), ("exact_nnz", ctypes.c_int32)]


class mrpt_index_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("T", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("a", ctypes.c_float), ("seed", ctypes.c_uint64), ("nnz", ctypes.c_int64),
                ("max_leaf", ctypes.c_int32), ("id_chunk", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("built_on_device", ctypes.c_int32), ("max_row_nnz", ctypes.c_int32)]


class mrpt_batch(ctypes.Structure):
    _fields_ = [("index", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("nq", ctypes.c_int64), ("k", ctypes.c_int32),
                ("v", ctypes.c_int32), ("out_idx", ctypes.c_void_p), ("out_dist", ctypes.c_void_p)]


class mrpt_plan_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rerank_factor", ctypes.c_int32), ("recheck_rel", ctypes.c_float),
                ("branches", ctypes.c_int32), ("proj_rows", ctypes.c_int32), ("vote_kernel", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("vote_waves", ctypes.c_int32)]


_lib = None

EXPORTED = [
    "mrpt_build", "mrpt_build_ex", "mrpt_default_build_opts", "mrpt_query", "mrpt_query_ex", "mrpt_query_noalloc", "mrpt_default_opts", "mrpt_free", "mrpt_last_error",
    "mrpt_index_info", "mrpt_export_projection", "mrpt_export_tree", "mrpt_export_leaf_offsets",
    "mrpt_debug_leaves", "mrpt_debug_votes", "mrpt_debug_prefilter", "mrpt_debug_lowp_rows", "mrpt_candidate_cap",
    "mrpt_default_plan_opts", "mrpt_plan_create", "mrpt_plan_launch", "mrpt_plan_device_bytes", "mrpt_plan_free",
]


def load(path: str = LIB_PATH):
    """Load libmrpt.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime (same soname) must be the one libmrpt binds to
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_1509_06957_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64
    lib.mrpt_build.argtypes = [vp, i64, i32, i32, i32, f32, u64, ctypes.POINTER(vp)]
    lib.mrpt_build_ex.argtypes = [vp, i64, i32, i32, i32, f32, u64, ctypes.POINTER(mrpt_build_opts),
                                  ctypes.POINTER(vp)]
    lib.mrpt_default_build_opts.argtypes = [ctypes.POINTER(mrpt_build_opts)]
    lib.mrpt_default_build_opts.restype = None
    lib.mrpt_query.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp]
    lib.mrpt_query_ex.argtypes = [vp, vp, i64, i32, i32, vp, vp, ctypes.POINTER(mrpt_query_opts), vp]
    lib.mrpt_query_noalloc.argtypes = [vp, vp, i64, i32, i32, vp, vp, ctypes.POINTER(mrpt_query_opts), vp]
    lib.mrpt_default_opts.argtypes = [ctypes.POINTER(mrpt_query_opts)]
    lib.mrpt_default_opts.restype = None
    lib.mrpt_free.argtypes = [vp]
    lib.mrpt_free.restype = None
    lib.mrpt_last_error.restype = ctypes.c_char_p
    lib.mrpt_index_info.argtypes = [vp, ctypes.POINTER(mrpt_index_desc)]
    lib.mrpt_export_projection.argtypes = [vp, vp, vp, vp]
    lib.mrpt_export_tree.argtypes = [vp, i32, vp, vp]
    lib.mrpt_export_leaf_offsets.argtypes = [vp, vp]
    lib.mrpt_debug_leaves.argtypes = [vp, vp, i64, vp, vp]
    lib.mrpt_debug_votes.argtypes = [vp, vp, i64, i32, vp, vp, vp, i64, vp]
    lib.mrpt_debug_prefilter.argtypes = [vp, vp, i64, i32, i32, ctypes.POINTER(mrpt_query_opts), vp, vp, vp]
    lib.mrpt_debug_lowp_rows.argtypes = [vp, i32, i64, i64, vp, vp, vp]
    lib.mrpt_candidate_cap.argtypes = [vp, i32]
    lib.mrpt_candidate_cap.restype = i64
    lib.mrpt_default_plan_opts.argtypes = [ctypes.POINTER(mrpt_plan_opts)]
    lib.mrpt_default_plan_opts.restype = None
    lib.mrpt_plan_create.argtypes = [ctypes.POINTER(mrpt_batch), i32, ctypes.POINTER(mrpt_plan_opts),
                                     ctypes.POINTER(vp)]
    lib.mrpt_plan_launch.argtypes = [vp, vp]
    lib.mrpt_plan_device_bytes.argtypes = [vp]
    lib.mrpt_plan_device_bytes.restype = i64
    lib.mrpt_plan_free.argtypes = [vp]
    lib.mrpt_plan_free.restype = None
    for name in EXPORTED:
        if name not in ("mrpt_default_opts", "mrpt_default_build_opts", "mrpt_free", "mrpt_last_error",
                        "mrpt_candidate_cap", "mrpt_default_plan_opts", "mrpt_plan_device_bytes",
                        "mrpt_plan_free"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def mrpt_last_error() -> str:
    return load().mrpt_last_error().decode()


def _check(status: int):
    if status != MRPT_OK:
        raise MrptError(status, mrpt_last_error())


def _dev(t, dtype_name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError(f"expected torch.{dtype_name}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def check_query_tensors(d: int, Q, k: int, out_idx, out_dist, s_count=None):
    """Shapes, dtypes and placement of a query call's tensors, checked before
    anything reaches the library: Q is (nq, d) float32, out_idx (nq, k) int32,
    out_dist (nq, k) float32, s_count (if given) int32 with at least nq
    entries, all contiguous and on one device.  Raises ValueError/TypeError."""
    import torch
    ts = [("Q", Q), ("out_idx", out_idx), ("out_dist", out_dist)] + ([("s_count", s_count)] if s_count is not None
                                                                      else [])
    for name, t in ts:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
    if Q.dim() != 2 or Q.shape[1] != d:
        raise ValueError(f"Q has shape {tuple(Q.shape)}, expected (nq, {d})")
    nq = Q.shape[0]
    for name, t, dt in (("Q", Q, torch.float32), ("out_idx", out_idx, torch.int32),
                        ("out_dist", out_dist, torch.float32)):
        if t.dtype != dt:
            raise TypeError(f"{name} is {t.dtype}, expected {dt}")
    for name, t in (("out_idx", out_idx), ("out_dist", out_dist)):
        if tuple(t.shape) != (nq, k):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected ({nq}, {k})")
    if s_count is not None:
        if s_count.dtype != torch.int32:
            raise TypeError(f"s_count is {s_count.dtype}, expected torch.int32")
        if s_count.numel() < nq:
            raise ValueError(f"s_count holds {s_count.numel()} entries, fewer than nq = {nq}")
    for name, t in ts:
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.device != Q.device:
            raise ValueError(f"{name} is on {t.device}, Q on {Q.device}")


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def mrpt_build(data, T: int, depth: int, a: float, seed: int) -> ctypes.c_void_p:
    """Build an index over data (n x d float32 CUDA tensor); returns the handle."""
    n, d = data.shape
    h = ctypes.c_void_p()
    _check(load().mrpt_build(_dev(data, "float32"), n, d, T, depth, a, seed & (2**64 - 1), ctypes.byref(h)))
    return h


def mrpt_default_build_opts() -> mrpt_build_opts:
    o = mrpt_build_opts()
    load().mrpt_default_build_opts(ctypes.byref(o))
    return o


def mrpt_build_ex(data, T: int, depth: int, a: float, seed: int, opts: mrpt_build_opts = None) -> ctypes.c_void_p:
    """mrpt_build with options (None: the defaults)."""
    n, d = data.shape
    h = ctypes.c_void_p()
    _check(load().mrpt_build_ex(_dev(data, "float32"), n, d, T, depth, a, seed & (2**64 - 1),
                                None if opts is None else ctypes.byref(opts), ctypes.byref(h)))
    return h


def mrpt_default_opts() -> mrpt_query_opts:
    o = mrpt_query_opts()
    load().mrpt_default_opts(ctypes.byref(o))
    return o


def mrpt_query(ix, Q, k: int, v: int, out_idx, out_dist, stream=None):
    check_query_tensors(mrpt_index_info(ix).d, Q, k, out_idx, out_dist)
    nq = Q.shape[0]
    _check(load().mrpt_query(ix, _dev(Q, "float32"), nq, k, v, _dev(out_idx, "int32"),
                             _dev(out_dist, "float32"), _stream(stream)))


def mrpt_query_ex(ix, Q, k: int, v: int, out_idx, out_dist, opts: Optional[mrpt_query_opts] = None, stream=None,
                  d: Optional[int] = None):
    """d: the index's dimension when the caller knows it (else asked from the library)."""
    check_query_tensors(mrpt_index_info(ix).d if d is None else d, Q, k, out_idx, out_dist)
    nq = Q.shape[0]
    _check(load().mrpt_query_ex(ix, _dev(Q, "float32"), nq, k, v, _dev(out_idx, "int32"),
                                _dev(out_dist, "float32"), None if opts is None else ctypes.byref(opts),
                                _stream(stream)))


def mrpt_query_noalloc(ix, Q, k: int, v: int, out_idx, out_dist, opts: Optional[mrpt_query_opts] = None,
                       stream=None, d: Optional[int] = None):
    """mrpt_query_ex without device allocation (temporaries in the library's
    fixed per-GPU scratch array)."""
    check_query_tensors(mrpt_index_info(ix).d if d is None else d, Q, k, out_idx, out_dist)
    nq = Q.shape[0]
    _check(load().mrpt_query_noalloc(ix, _dev(Q, "float32"), nq, k, v, _dev(out_idx, "int32"),
                                     _dev(out_dist, "float32"), None if opts is None else ctypes.byref(opts),
                                     _stream(stream)))


def mrpt_free(ix):
    if ix:
        load().mrpt_free(ix)


def mrpt_index_info(ix) -> mrpt_index_desc:
    out = mrpt_index_desc()
    _check(load().mrpt_index_info(ix, ctypes.byref(out)))
    return out


def mrpt_export_projection(ix):
    """(rowptr, col, val) numpy arrays of the CSR of the projection vectors."""
    info = mrpt_index_info(ix)
    rows = info.T * info.depth
    rowptr = np.zeros(rows + 1, np.int32)
    col = np.zeros(max(info.nnz, 1), np.int32)
    val = np.zeros(max(info.nnz, 1), np.float32)
    _check(load().mrpt_export_projection(ix, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data))
    return rowptr, col[:info.nnz], val[:info.nnz]


def mrpt_export_tree(ix, t: int):
    """(splits, perm) numpy arrays of tree t."""
    info = mrpt_index_info(ix)
    splits = np.zeros(max((1 << info.depth) - 1, 1), np.float32)
    perm = np.zeros(info.n, np.int32)
    _check(load().mrpt_export_tree(ix, t, splits.ctypes.data, perm.ctypes.data))
    return splits[:(1 << info.depth) - 1], perm


def mrpt_export_leaf_offsets(ix):
    info = mrpt_index_info(ix)
    off = np.zeros((1 << info.depth) + 1, np.int64)
    _check(load().mrpt_export_leaf_offsets(ix, off.ctypes.data))
    return off


def mrpt_debug_leaves(ix, Q, leaf, stream=None):
    _check(load().mrpt_debug_leaves(ix, _dev(Q, "float32"), Q.shape[0], _dev(leaf, "int32"), _stream(stream)))


def mrpt_debug_votes(ix, Q, v: int, s_count, s_ids, s_votes, cap: int, stream=None):
    _check(load().mrpt_debug_votes(ix, _dev(Q, "float32"), Q.shape[0], v, _dev(s_count, "int32"),
                                   _dev(s_ids, "int32"), None if s_votes is None else _dev(s_votes, "uint8"),
                                   cap, _stream(stream)))


def mrpt_debug_prefilter(ix, Q, k: int, v: int, opts: mrpt_query_opts, s_count, keep_ids, stream=None):
    _check(load().mrpt_debug_prefilter(ix, _dev(Q, "float32"), Q.shape[0], k, v, ctypes.byref(opts),
                                       _dev(s_count, "int32"), _dev(keep_ids, "int32"), _stream(stream)))


def mrpt_debug_lowp_rows(ix, precision: int, row0: int, rows, scale_norm=None, stream=None):
    """rows: CUDA tensor of nrows x d (int16 for MRPT_BF16_RERANK, uint8 for
    MRPT_FP8_RERANK); scale_norm: optional float32 CUDA tensor of nrows x 2."""
    want = "int16" if precision == MRPT_BF16_RERANK else "uint8"
    _check(load().mrpt_debug_lowp_rows(ix, precision, row0, rows.shape[0], _dev(rows, want),
                                       None if scale_norm is None else _dev(scale_norm, "float32"),
                                       _stream(stream)))


def mrpt_candidate_cap(ix, v: int) -> int:
    return int(load().mrpt_candidate_cap(ix, v))


def mrpt_default_plan_opts() -> mrpt_plan_opts:
    o = mrpt_plan_opts()
    load().mrpt_default_plan_opts(ctypes.byref(o))
    return o


def mrpt_plan_create(batches, opts: Optional[mrpt_plan_opts] = None) -> ctypes.c_void_p:
    """batches: sequence of (index handle, Q, k, v, out_idx, out_dist) with torch
    CUDA tensors; returns the plan handle.  The tensors must outlive the plan."""
    arr = (mrpt_batch * len(batches))()
    for i, (ix, Q, k, v, out_idx, out_dist) in enumerate(batches):
        check_query_tensors(mrpt_index_info(ix).d, Q, k, out_idx, out_dist)
        arr[i] = mrpt_batch(ix, _dev(Q, "float32"), Q.shape[0], k, v, _dev(out_idx, "int32"),
                            _dev(out_dist, "float32"))
    h = ctypes.c_void_p()
    _check(load().mrpt_plan_create(arr, len(batches), None if opts is None else ctypes.byref(opts),
                                   ctypes.byref(h)))
    return h


def mrpt_plan_launch(plan, stream=None):
    _check(load().mrpt_plan_launch(plan, _stream(stream)))


def mrpt_plan_device_bytes(plan) -> int:
    return int(load().mrpt_plan_device_bytes(plan))


def mrpt_plan_free(plan):
    if plan:
        load().mrpt_plan_free(plan)


class Plan:
    """Owning wrapper of a query plan over (Index, Q, k, v) batches; results
    land in self.out[i] = (idx, dist) at every launch()."""

    def __init__(self, batches, precision: int = MRPT_FP32, rerank_factor: int = 4, recheck_rel: float = 1e-6,
                 branches: int = 4, proj_rows: int = 0, vote_kernel: int = 0, fused: int = 1, vote_waves: int = 0):
        import torch
        self.handle = None
        self.batches = list(batches)
        self.out = [(torch.empty((Q.shape[0], k), dtype=torch.int32, device=Q.device),
                     torch.empty((Q.shape[0], k), dtype=torch.float32, device=Q.device))
                    for (_, Q, k, _) in self.batches]
        o = mrpt_default_plan_opts()
        o.precision, o.rerank_factor, o.recheck_rel, o.branches = precision, rerank_factor, recheck_rel, branches
        o.proj_rows, o.vote_kernel, o.fused, o.vote_waves = proj_rows, vote_kernel, fused, vote_waves
        self.handle = mrpt_plan_create([(ix.handle, Q, k, v, oi, od) for (ix, Q, k, v), (oi, od)
                                        in zip(self.batches, self.out)], o)

    def launch(self, stream=None):
        mrpt_plan_launch(self.handle, stream)
        return self.out

    def device_bytes(self) -> int:
        return mrpt_plan_device_bytes(self.handle)

    def close(self):
        if self.handle:
            mrpt_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Index:
    """Owning wrapper of an index handle (frees it on close / garbage collection)."""

    def __init__(self, data, T: int, depth: int, a: float, seed: int, on_device: bool = True,
                 exact_nnz: bool = False):
        opts = mrpt_default_build_opts()
        opts.on_device = 1 if on_device else 0
        opts.exact_nnz = 1 if exact_nnz else 0
        self.handle = mrpt_build_ex(data, T, depth, a, seed, opts)
        self.info = mrpt_index_info(self.handle)

    def query(self, Q, k: int, v: int, precision: int = MRPT_FP32, rerank_factor: int = 4,
              recheck_rel: float = 1e-6, s_count=None, out=None, stream=None):
        import torch
        if not isinstance(Q, torch.Tensor) or Q.dim() != 2:
            raise ValueError("Q must be a 2-D torch tensor")
        nq = Q.shape[0]
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=Q.device),
                   torch.empty((nq, k), dtype=torch.float32, device=Q.device))
        check_query_tensors(self.info.d, Q, k, out[0], out[1], s_count)
        o = mrpt_default_opts()
        o.precision = precision
        o.rerank_factor = rerank_factor
        o.recheck_rel = recheck_rel
        o.s_count = None if s_count is None else _dev(s_count, "int32").value
        mrpt_query_ex(self.handle, Q, k, v, out[0], out[1], o, stream, d=self.info.d)
        return out

    def close(self):
        if self.handle:
            mrpt_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
