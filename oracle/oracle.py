"""ctypes wrapper around the plain-C oracle (oracle.c).  Test infrastructure only.

Each wrapper names the passage of "Fast k-NN Search" (arXiv:1509.06957) that
the C function follows.  Arrays are numpy, C-contiguous, on the host.
"""
import ctypes
import os

import numpy as np

__all__ = [
    "load", "philox4x64_10", "random_matrix", "exact_nnz_count", "project", "leaf_offsets", "build_index",
    "route", "query", "bruteforce", "distance", "OracleIndex", "default_threads", "all_threads",
    "bf16_round", "bf16_value", "e4m3_round", "e4m3_value", "fp8_rows", "query_prefilter",
    "ARM_BF16", "ARM_FP8",
]

ARM_BF16, ARM_FP8 = 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def all_threads() -> int:
    """Every core this process may run on (its CPU affinity set)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, n)


def default_threads() -> int:
    """Host threads the oracle uses in tests: the cores this process may run on, at most 16."""
    return min(16, all_threads())


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.oracle_random_matrix.argtypes = [_i32, _i32, _i32, ctypes.c_float, ctypes.c_uint64, _f32p]
    lib.oracle_random_matrix_exact.argtypes = [_i32, _i32, _i32, ctypes.c_float, ctypes.c_uint64, _f32p]
    lib.oracle_exact_nnz.argtypes = [_i32, ctypes.c_float]
    lib.oracle_exact_nnz.restype = _i32
    lib.oracle_project.argtypes = [_f32p, _i64, _i32, _f32p, _i32, _f32p]
    lib.oracle_leaf_offsets.argtypes = [_i64, _i32, _i64p]
    lib.oracle_build.argtypes = [_f32p, _i64, _i32, _i32, _i32, ctypes.c_float, ctypes.c_uint64, _i32,
                                 _f32p, _f32p, _i32p, _i32]
    lib.oracle_route.argtypes = [_f32p, _i64, _i32, _f32p, _i32, _i32, _f32p, _i32p]
    lib.oracle_distance.argtypes = [_f32p, _f32p, _i32]
    lib.oracle_distance.restype = ctypes.c_double
    lib.oracle_query.argtypes = [_f32p, _i64, _i32, _i32, _i32, _f32p, _f32p, _i32p, _i64p,
                                 _f32p, _i64, _i32, _i32, _i32p, _f64p, _vp, _vp, _vp, _i64, _vp, _i32]
    lib.oracle_bruteforce.argtypes = [_f32p, _i64, _i32, _f32p, _i64, _i32, _i32p, _f64p, _i32]
    lib.oracle_bf16_value.argtypes = [ctypes.c_uint16]
    lib.oracle_bf16_value.restype = ctypes.c_double
    lib.oracle_bf16_round.argtypes = [ctypes.c_float]
    lib.oracle_bf16_round.restype = ctypes.c_uint16
    lib.oracle_to_bf16.argtypes = [_f32p, _i64, np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")]
    lib.oracle_e4m3_value.argtypes = [ctypes.c_uint8]
    lib.oracle_e4m3_value.restype = ctypes.c_double
    lib.oracle_e4m3_round.argtypes = [ctypes.c_float]
    lib.oracle_e4m3_round.restype = ctypes.c_uint8
    lib.oracle_to_fp8_rows.argtypes = [_f32p, _i64, _i32, np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS"),
                                       _f32p, _f64p]
    lib.oracle_query_prefilter.argtypes = [_f32p, _i64, _i32, _i32, _i32, _f32p, _f32p, _i32p, _i64p,
                                           _f32p, _i64, _i32, _i32, _i32, _i32, _i32p, _f64p, _i64p,
                                           _i32p, _f64p, _i32p, _i32]
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def philox4x64_10(counter, key):
    """Philox4x64-10 block (Salmon et al., SC'11): 4 x uint64 counter, 2 x uint64 key."""
    out = np.zeros(4, dtype=np.uint64)
    load().oracle_philox4x64_10(_c(counter, np.uint64), _c(key, np.uint64), out)
    return out


def random_matrix(d, T, depth, a, seed, exact_nnz=False):
    """Sparse Gaussian projection vectors, Sec. II-B / Alg. 1; dense (T*depth, d).
    exact_nnz: exactly ceil(a d) nonzeros per vector (footnote of Sec. II-D)."""
    R = np.zeros((T * depth, d), dtype=np.float32)
    if T * depth > 0:
        fn = load().oracle_random_matrix_exact if exact_nnz else load().oracle_random_matrix
        fn(d, T, depth, float(a), int(seed) & (2**64 - 1), R)
    return R


def exact_nnz_count(d, a):
    """m = ceil(a d) in double, clamped to [1, d] (the exact-count mode's nonzeros per vector)."""
    return int(load().oracle_exact_nnz(int(d), float(a)))


def project(X, R):
    """P = X R^T as the float32 fused-multiply-add chain of Sec. II-C / Alg. 3."""
    X = _c(X, np.float32)
    R = _c(R, np.float32)
    P = np.zeros((X.shape[0], R.shape[0]), dtype=np.float32)
    if X.shape[0] and R.shape[0]:
        load().oracle_project(X, X.shape[0], X.shape[1], R, R.shape[0], P)
    return P


def leaf_offsets(n, depth):
    """First slot of each leaf (2^depth + 1 entries); sizes follow Sec. II-A."""
    off = np.zeros((1 << depth) + 1, dtype=np.int64)
    load().oracle_leaf_offsets(int(n), int(depth), off)
    return off


class OracleIndex:
    """T trees grown by Alg. 1-2: R (T*depth, d), splits (T, 2^depth-1), perm (T, n)."""

    def __init__(self, X, T, depth, a, seed, R, splits, perm, off):
        self.X, self.T, self.depth, self.a, self.seed = X, T, depth, a, seed
        self.R, self.splits, self.perm, self.off = R, splits, perm, off

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    def leaf(self, t, L):
        return self.perm[t, self.off[L]:self.off[L + 1]]


def build_index(X, T, depth, a, seed, nthreads=None, exact_nnz=False):
    """grow_trees (Alg. 1) calling grow_tree (Alg. 2) for every tree
    (exact_nnz: projection vectors with exactly ceil(a d) nonzeros)."""
    X = _c(X, np.float32)
    n, d = X.shape
    nsplit = (1 << depth) - 1
    R = np.zeros((T * depth, d), dtype=np.float32)
    splits = np.zeros((T, nsplit), dtype=np.float32)
    perm = np.zeros((T, n), dtype=np.int32)
    sp = splits if nsplit > 0 else np.zeros((T, 1), dtype=np.float32)
    load().oracle_build(X, n, d, T, depth, float(a), int(seed) & (2**64 - 1), 1 if exact_nnz else 0, R, sp,
                        perm, nthreads or default_threads())
    return OracleIndex(X, T, depth, a, seed, R, splits, perm, leaf_offsets(n, depth))


def route(index, Q):
    """tree_query (Alg. 3) for every query and tree: leaf index, shape (nq, T)."""
    Q = _c(Q, np.float32)
    leaf = np.zeros((Q.shape[0], index.T), dtype=np.int32)
    sp = index.splits if index.splits.size else np.zeros((index.T, 1), dtype=np.float32)
    if Q.shape[0]:
        load().oracle_route(Q, Q.shape[0], index.d, index.R if index.R.size else np.zeros((1, index.d), np.float32),
                            index.T, index.depth, _c(sp, np.float32), leaf)
    return leaf


def query(index, Q, k, v, want_sets=False, s_cap=None, nthreads=None):
    """approximate_knn (Alg. 4): voting over T leaves, then exact k-NN in S.

    Returns dict with idx (nq,k) int32, dist (nq,k) float64, s_count (nq,),
    leaf (nq,T); with want_sets also s_ids / s_votes (ascending ids per query).
    """
    Q = _c(Q, np.float32)
    nq = Q.shape[0]
    idx = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float64)
    s_count = np.zeros(nq, dtype=np.int64)
    leaf = np.zeros((nq, index.T), dtype=np.int32)
    s_ids = s_votes = None
    if want_sets:
        cap = s_cap or min(index.n, index.T * int(np.max(np.diff(index.off))))
        s_ids = np.full((nq, cap), -1, dtype=np.int32)
        s_votes = np.zeros((nq, cap), dtype=np.int32)
    else:
        cap = 0
    sp = index.splits if index.splits.size else np.zeros((index.T, 1), dtype=np.float32)
    R = index.R if index.R.size else np.zeros((1, index.d), np.float32)
    if nq:
        load().oracle_query(index.X, index.n, index.d, index.T, index.depth, R, _c(sp, np.float32),
                            index.perm, index.off, Q, nq, k, v, idx, dist,
                            s_count.ctypes.data, None if s_ids is None else s_ids.ctypes.data,
                            None if s_votes is None else s_votes.ctypes.data, cap, leaf.ctypes.data,
                            nthreads or default_threads())
    out = {"idx": idx, "dist": dist, "s_count": s_count, "leaf": leaf}
    if want_sets:
        out["s_ids"] = [s_ids[q, :min(cap, s_count[q])].copy() for q in range(nq)]
        out["s_votes"] = [s_votes[q, :min(cap, s_count[q])].copy() for q in range(nq)]
    return out


def bruteforce(X, Q, k, nthreads=None):
    """Exact k-NN (Sec. I-A) in float64, order (distance, id)."""
    X = _c(X, np.float32)
    Q = _c(Q, np.float32)
    nq = Q.shape[0]
    idx = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float64)
    if nq:
        load().oracle_bruteforce(X, X.shape[0], X.shape[1], Q, nq, k, idx, dist, nthreads or default_threads())
    return idx, dist


def distance(q, x):
    """Euclidean distance (Sec. I-A) in float64 of two float32 vectors."""
    q = _c(q, np.float32)
    x = _c(x, np.float32)
    return load().oracle_distance(q, x, q.shape[0])


# ---------------------------------------------------------------------------
# precision arms (not in the paper): low-precision rows and the prefilter
# ---------------------------------------------------------------------------
def bf16_round(x):
    """bfloat16 bit patterns (uint16) of float32 values: round to nearest, ties to even."""
    x = _c(x, np.float32)
    out = np.zeros(x.shape, dtype=np.uint16)
    if x.size:
        load().oracle_to_bf16(x.reshape(-1), x.size, out.reshape(-1))
    return out


def bf16_value(b):
    """float64 values of bfloat16 bit patterns."""
    lib = load()
    b = np.asarray(b, dtype=np.uint16)
    return np.array([lib.oracle_bf16_value(int(v)) for v in b.reshape(-1)], dtype=np.float64).reshape(b.shape)


def e4m3_value(codes):
    """float64 values of OCP E4M3 codes (NaN for 0x7f and 0xff)."""
    lib = load()
    c = np.asarray(codes, dtype=np.uint8)
    return np.array([lib.oracle_e4m3_value(int(v)) for v in c.reshape(-1)], dtype=np.float64).reshape(c.shape)


def e4m3_round(y):
    """E4M3 codes of float32 values: round to nearest, ties to the even code."""
    lib = load()
    y = np.asarray(y, dtype=np.float32)
    return np.array([lib.oracle_e4m3_round(float(v)) for v in y.reshape(-1)], dtype=np.uint8).reshape(y.shape)


def fp8_rows(X):
    """Per-row scaled E4M3 rows: (codes n x d uint8, scale n float32 = max|x|/240,
    norm n float64 = squared norm of the decoded row)."""
    X = _c(X, np.float32)
    n, d = X.shape
    codes = np.zeros((n, d), dtype=np.uint8)
    scale = np.zeros(n, dtype=np.float32)
    norm = np.zeros(n, dtype=np.float64)
    if n:
        load().oracle_to_fp8_rows(X, n, d, codes, scale, norm)
    return codes, scale, norm


def query_prefilter(index, Q, k, v, arm, kp, nthreads=None):
    """The precision arm of a query batch (arm = ARM_BF16 or ARM_FP8): S as in
    query(), ranked by the float64 squared distance to the decoded rows, the
    first kp under (score, id) kept, then the exact k-NN of the kept.

    Returns dict with idx (nq,k), dist (nq,k) float64, s_count (nq,),
    keep_ids (nq,kp) in score order (-1 padded), keep_score (nq,kp) float64,
    keep_count (nq,) = min(|S|, kp)."""
    Q = _c(Q, np.float32)
    nq = Q.shape[0]
    idx = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float64)
    s_count = np.zeros(nq, dtype=np.int64)
    keep_ids = np.zeros((nq, kp), dtype=np.int32)
    keep_score = np.zeros((nq, kp), dtype=np.float64)
    keep_count = np.zeros(nq, dtype=np.int32)
    sp = index.splits if index.splits.size else np.zeros((index.T, 1), dtype=np.float32)
    R = index.R if index.R.size else np.zeros((1, index.d), np.float32)
    if nq:
        load().oracle_query_prefilter(index.X, index.n, index.d, index.T, index.depth, R, _c(sp, np.float32),
                                      index.perm, index.off, Q, nq, k, v, int(arm), int(kp), idx, dist, s_count,
                                      keep_ids, keep_score, keep_count, nthreads or default_threads())
    return {"idx": idx, "dist": dist, "s_count": s_count, "keep_ids": keep_ids, "keep_score": keep_score,
            "keep_count": keep_count}
