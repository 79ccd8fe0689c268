"""GPU parity of every step of the query path against the oracle, through the
C ABI: projection vectors, trees, leaves, candidate sets with vote counts,
and the k nearest neighbours (float32 arm and bfloat16+rerank arm).

Sizes: the mixture-128 (n=10k, d=128) and mnist-like (n=60k, d=784)
workloads at their full sizes, plus small shapes that hit ragged tiles, the
generic kernels and the degenerate cases of the method.
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import build, check_knn, dev, dist64, leaves, query, recall, votes  # noqa: E402
from paper_1509_06957_amd import mrpt  # noqa: E402


def _print_case(name):
    print(f"[case] {name}", flush=True)


class Case:
    def __init__(self, w: W.Workload, nq=None):
        w = w if nq is None else w.scaled(nq=nq)
        self.w = w
        self.X = W.data(w)
        self.Q = W.queries(w)
        self.orc = oracle.build_index(self.X, w.T, w.depth, w.a, w.index_seed)
        self.gpu = build(self.X, w.T, w.depth, w.a, w.index_seed)
        self.Qd = dev(self.Q)


@pytest.fixture(scope="module", params=["mixture128", "mnist_like"])
def case(request):
    _print_case(request.param)
    c = Case(W.ALL[request.param])
    yield c
    c.gpu.close()


def test_projection_bit_exact(case):
    rowptr, col, val = mrpt.mrpt_export_projection(case.gpu.handle)
    R = np.zeros_like(case.orc.R)
    for r in range(R.shape[0]):
        R[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
        assert np.all(np.diff(col[rowptr[r]:rowptr[r + 1]]) > 0)
    assert np.array_equal(R.view(np.uint32), case.orc.R.view(np.uint32))


def test_trees_bit_exact(case):
    off = mrpt.mrpt_export_leaf_offsets(case.gpu.handle)
    assert np.array_equal(off, case.orc.off)
    for t in range(case.w.T):
        splits, perm = mrpt.mrpt_export_tree(case.gpu.handle, t)
        assert np.array_equal(splits.view(np.uint32), case.orc.splits[t].view(np.uint32)), f"tree {t} splits"
        assert np.array_equal(perm, case.orc.perm[t]), f"tree {t} perm"


def test_leaves_bit_exact(case):
    assert np.array_equal(leaves(case.gpu, case.Qd), oracle.route(case.orc, case.Q))


def test_vote_recount_bit_exact(case):
    # s_votes come from vote_counts_kernel, a debug recount (binary search of
    # every listed id in the query's leaves); the candidate sets come from the
    # query path's counter.  The counter's own F is pinned by the next test.
    w = case.w
    for v in sorted({1, w.v, w.T}):
        ref = oracle.query(case.orc, case.Q, w.k, v, want_sets=True)
        ids, cnt = votes(case.gpu, case.Qd, v)
        for q in range(len(case.Q)):
            assert np.array_equal(ids[q], ref["s_ids"][q]), f"v={v} query {q} S"
            assert np.array_equal(cnt[q], ref["s_votes"][q]), f"v={v} query {q} F"


def _check_every_threshold(g, orc, Q, Qd, T, label):
    """S_v from the query path's counter for every v = 1..T equals the
    oracle's; F(x) = #{v : x in S_v} is then the counter's own vote count and
    must equal the oracle's F (Sec. III-A)."""
    ref1 = oracle.query(orc, Q, 1, 1, want_sets=True)
    F = [dict() for _ in range(len(Q))]
    for v in range(1, T + 1):
        ref = ref1 if v == 1 else oracle.query(orc, Q, 1, v, want_sets=True)
        ids, _ = votes(g, Qd, v, with_counts=False)
        for q in range(len(Q)):
            assert np.array_equal(ids[q], ref["s_ids"][q]), f"{label} v={v} query {q}"
            for x in ids[q].tolist():
                F[q][x] = F[q].get(x, 0) + 1
    for q in range(len(Q)):
        got = np.array([F[q][x] for x in ref1["s_ids"][q].tolist()], dtype=np.int32)
        assert len(F[q]) == len(ref1["s_ids"][q])
        assert np.array_equal(got, ref1["s_votes"][q]), f"{label} query {q}: F"


def test_hot_counter_every_threshold(case):
    w = case.w
    _check_every_threshold(case.gpu, case.orc, case.Q, case.Qd, w.T, w.name)


@pytest.mark.parametrize("kernel", ["0", "1"])
def test_hot_counter_every_threshold_multipass(kernel, monkeypatch):
    # the multi-pass kernels: with the leaf directory (MRPT_VOTE_KERNEL=0 at
    # build and query time) and without it (1); n above one directory grain
    _print_case(f"every threshold, multi-pass vote kernel {kernel}")
    monkeypatch.setenv("MRPT_VOTE_KERNEL", kernel)
    X, Q = _small(150000, 8, 12, 7, seed=77, nq=300)
    orc = oracle.build_index(X, 12, 7, 0.5, 3)
    g = build(X, 12, 7, 0.5, 3)
    try:
        _check_every_threshold(g, orc, Q, dev(Q), 12, f"kernel {kernel}")
    finally:
        g.close()


def test_knn_fp32(case):
    w = case.w
    ref = oracle.query(case.orc, case.Q, w.k, w.v, want_sets=True)
    gi, gd, sc = query(case.gpu, case.Qd, w.k, w.v)
    assert np.array_equal(sc, ref["s_count"])
    exact = w.kind in ("mnist_like", "sift_like")
    check_knn(case.X, case.Q, gi, gd, ref["idx"], ref["dist"], exact_ids=exact,
              S=[set(s.tolist()) for s in ref["s_ids"]])
    bi, _ = oracle.bruteforce(case.X, case.Q, w.k)
    print(f"[recall] {w.name} fp32 gpu {recall(gi, bi):.4f} oracle {recall(ref['idx'], bi):.4f}", flush=True)


def test_knn_bf16_rerank(case):
    w = case.w
    ref = oracle.query(case.orc, case.Q, w.k, w.v)
    gi, gd, _ = query(case.gpu, case.Qd, w.k, w.v, precision=mrpt.MRPT_BF16_RERANK)
    fi, fd, _ = query(case.gpu, case.Qd, w.k, w.v)
    bi, _ = oracle.bruteforce(case.X, case.Q, w.k)
    r_b, r_f = recall(gi, bi), recall(fi, bi)
    print(f"[recall] {w.name} bf16+rerank {r_b:.4f} fp32 {r_f:.4f}", flush=True)
    if w.kind == "mnist_like":
        # integers <= 255 are exact in bfloat16 and every sum stays below 2^24
        assert np.array_equal(gi, fi) and np.array_equal(gd, fd)
    # returned distances are float32/float64 recomputations: always within tolerance
    for q in range(len(case.Q)):
        real = gi[q][gi[q] >= 0]
        d64 = np.sqrt(((case.X[real].astype(np.float64) - case.Q[q].astype(np.float64)) ** 2).sum(1))
        assert np.all(np.abs(gd[q][:len(real)] - d64) <= 1e-5 * d64 + 1e-6)
        assert np.all(np.diff(gd[q][:len(real)]) >= -1e-6 * gd[q][len(real) - 1])
    assert r_b >= r_f - 0.02


def test_repeat_is_deterministic(case):
    w = case.w
    a = query(case.gpu, case.Qd, w.k, w.v)
    b = query(case.gpu, case.Qd, w.k, w.v)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


# ---------------------------------------------------------------- edge cases

def _small(n, d, T, depth, seed=0, integer=False, nq=37):
    rng = np.random.default_rng(seed)
    if integer:
        X = rng.integers(0, 4, size=(n, d)).astype(np.float32)
        Q = rng.integers(0, 4, size=(nq, d)).astype(np.float32)
    else:
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = rng.standard_normal((nq, d)).astype(np.float32)
    return X, Q


def _full_compare(X, Q, T, depth, a, seed, k, v, exact_ids=False, precision=None):
    orc = oracle.build_index(X, T, depth, a, seed)
    g = build(X, T, depth, a, seed)
    Qd = dev(Q)
    assert np.array_equal(leaves(g, Qd), oracle.route(orc, Q))
    ref = oracle.query(orc, Q, k, v, want_sets=True)
    ids, cnt = votes(g, Qd, v)
    for q in range(len(Q)):
        assert np.array_equal(ids[q], ref["s_ids"][q])
        assert np.array_equal(cnt[q], ref["s_votes"][q])
    kw = {} if precision is None else {"precision": precision}
    gi, gd, sc = query(g, Qd, k, v, **kw)
    assert np.array_equal(sc, ref["s_count"])
    check_knn(X, Q, gi, gd, ref["idx"], ref["dist"], exact_ids=exact_ids,
              S=[set(s.tolist()) for s in ref["s_ids"]])
    g.close()
    return gi, gd, ref


@pytest.mark.parametrize("nq", [1, 63, 64, 65, 130])
def test_ragged_query_tiles(nq):
    _print_case(f"ragged nq={nq}")
    X, Q = _small(3000, 32, 6, 5, seed=nq, nq=nq)
    _full_compare(X, Q, 6, 5, 0.2, 11, 10, 2)


@pytest.mark.parametrize("nq,d", [(8250, 128), (8300, 96), (8200, 129)])
def test_large_batch_projection_tiles(nq, d):
    """Batches large enough for the projection's large-batch form: 16 rows per
    wave, with two queries per lane for d <= 128 (the last tile's second half
    empty at nq = 8250, partly filled at 8300) and one above."""
    _print_case(f"large-batch projection nq={nq} d={d}")
    rng = np.random.default_rng(nq + d)
    X = rng.standard_normal((20000, d)).astype(np.float32)
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    T, depth, a, seed = 64, 8, 1 / np.sqrt(d), 31
    orc = oracle.build_index(X, T, depth, a, seed)
    g = build(X, T, depth, a, seed)
    assert np.array_equal(leaves(g, dev(Q)), oracle.route(orc, Q))
    g.close()


@pytest.mark.parametrize("nq", [5, 700])
def test_query_rows_not_16_byte_aligned(nq):
    """Q starting 4 bytes past a 16-byte boundary (d = 128, a multiple of 4):
    the projection stages the tile with 4-byte loads instead of 16-byte ones,
    and the leaves still equal the oracle's."""
    _print_case(f"misaligned Q nq={nq}")
    d = 128
    rng = np.random.default_rng(nq)
    X = rng.standard_normal((6000, d)).astype(np.float32)
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    T, depth, a, seed = 12, 7, 1 / np.sqrt(d), 19
    orc = oracle.build_index(X, T, depth, a, seed)
    g = build(X, T, depth, a, seed)
    try:
        flat = torch.empty(nq * d + 4, dtype=torch.float32, device="cuda")
        Qm = flat[1:1 + nq * d].view(nq, d)
        Qm.copy_(dev(Q))
        assert Qm.data_ptr() % 16 == 4
        assert np.array_equal(leaves(g, Qm), oracle.route(orc, Q))
        gi, gd, sc = query(g, Qm, 10, 2)
        ref = oracle.query(orc, Q, 10, 2)
        assert np.array_equal(sc, ref["s_count"])
    finally:
        g.close()


@pytest.mark.parametrize("d", [1, 3, 4, 13, 36, 64, 200, 520])
def test_dimensions_generic_and_vector_kernels(d):
    _print_case(f"dim d={d}")
    X, Q = _small(1500, d, 5, 4, seed=d)
    a = min(1.0, 1 / np.sqrt(d) * 2)
    _full_compare(X, Q, 5, 4, a, 3, 7, 1)


def test_depth_zero_is_bruteforce():
    _print_case("depth 0")
    X, Q = _small(2000, 24, 3, 0, seed=5)
    gi, gd, ref = _full_compare(X, Q, 3, 0, 0.3, 1, 10, 1)
    bi, bd = oracle.bruteforce(X, Q, 10)
    check_knn(X, Q, gi, gd, bi, bd, exact_ids=False)


def test_single_tree_and_all_votes():
    _print_case("T=1 and v=T")
    X, Q = _small(4000, 16, 1, 6, seed=6)
    _full_compare(X, Q, 1, 6, 0.5, 2, 5, 1)
    X, Q = _small(4000, 16, 9, 4, seed=7)
    _full_compare(X, Q, 9, 4, 0.5, 2, 5, 9)


def test_short_candidate_sets_padded():
    _print_case("padding")
    X, Q = _small(512, 8, 3, 6, seed=8)   # leaves of 8, v = 3 keeps few
    gi, gd, ref = _full_compare(X, Q, 3, 6, 0.5, 4, 12, 3)
    assert np.any(gi == -1)


def test_integer_ties_exact():
    _print_case("integer ties")
    X, Q = _small(5000, 12, 7, 6, seed=9, integer=True)
    _full_compare(X, Q, 7, 6, 0.4, 5, 10, 2, exact_ids=True)


@pytest.mark.parametrize("k", [1, 64, 65, 100, 300])
def test_large_k(k):
    _print_case(f"k={k}")
    X, Q = _small(6000, 20, 6, 3, seed=k)
    _full_compare(X, Q, 6, 3, 0.3, 6, k, 1)


def test_bf16_generic_shapes():
    _print_case("bf16 shapes")
    for d in (8, 96, 256, 960):
        X, Q = _small(1200, d, 4, 3, seed=d, integer=True)
        gi_b, gd_b, ref = _full_compare(X, Q, 4, 3, min(1.0, 2 / np.sqrt(d)), 1, 10, 1, exact_ids=True,
                                        precision=mrpt.MRPT_BF16_RERANK)


@pytest.mark.parametrize("k", [16, 17, 30, 100])
def test_bf16_rerank_widths_at_d128(k):
    """bf16 + rerank at d = 128 for every width of the kept list: k * 4 = 64
    (the seven-wave form), 68 and 120 (two registers per lane), 400 (eight)."""
    _print_case(f"bf16 d=128 k={k}")
    X, Q = _small(3000, 128, 6, 3, seed=k, integer=True)
    _full_compare(X, Q, 6, 3, 2 / np.sqrt(128), 5, k, 1, exact_ids=True, precision=mrpt.MRPT_BF16_RERANK)


def test_streams_and_nq_zero():
    _print_case("stream")
    X, Q = _small(2000, 32, 4, 4, seed=10)
    g = build(X, 4, 4, 0.3, 1)
    Qd = dev(Q)
    ref = query(g, Qd, 5, 1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        idx = torch.empty((len(Q), 5), dtype=torch.int32, device="cuda")
        dist = torch.empty((len(Q), 5), dtype=torch.float32, device="cuda")
        mrpt.mrpt_query(g.handle, Qd, 5, 1, idx, dist, stream=s)
    s.synchronize()
    assert np.array_equal(idx.cpu().numpy(), ref[0])
    empty = torch.empty((0, 32), dtype=torch.float32, device="cuda")
    mrpt.mrpt_query(g.handle, empty, 5, 1, idx[:0], dist[:0])
    g.close()


def test_error_paths():
    _print_case("errors")
    X, Q = _small(1000, 8, 2, 3, seed=11)
    Xd, Qd = dev(X), dev(Q)
    with pytest.raises(mrpt.MrptError) as e:
        mrpt.mrpt_build(Xd, 2, 11, 0.5, 1)          # 2^11 > n
    assert e.value.status == mrpt.MRPT_EINVAL
    for T, a in ((0, 0.5), (256, 0.5), (2, 0.0), (2, 1.5)):
        with pytest.raises(mrpt.MrptError):
            mrpt.mrpt_build(Xd, T, 3, a, 1)
    bad = X.copy()
    bad[5, 3] = np.nan
    with pytest.raises(mrpt.MrptError) as e:
        mrpt.mrpt_build(dev(bad), 2, 3, 0.5, 1)
    assert e.value.status == mrpt.MRPT_ENONFINITE
    h = ctypes_build_host_pointer(X)
    assert h == mrpt.MRPT_EINVAL
    g = build(X, 2, 3, 0.5, 1)
    idx = torch.empty((len(Q), 5), dtype=torch.int32, device="cuda")
    dist = torch.empty((len(Q), 5), dtype=torch.float32, device="cuda")
    # outputs sized (nq, k) so the binding's shape check passes and the
    # library's own argument check is what rejects k and v
    for k, v in ((0, 1), (5, 0), (5, 3), (1025, 1)):
        ik = torch.empty((len(Q), k), dtype=torch.int32, device="cuda")
        dk = torch.empty((len(Q), k), dtype=torch.float32, device="cuda")
        with pytest.raises(mrpt.MrptError) as e:
            mrpt.mrpt_query(g.handle, Qd, k, v, ik, dk)
        assert e.value.status == mrpt.MRPT_EINVAL
    Qn = Q.copy()
    Qn[2, 1] = np.inf
    o = mrpt.mrpt_default_opts()
    o.check_finite = 1
    with pytest.raises(mrpt.MrptError) as e:
        mrpt.mrpt_query_ex(g.handle, dev(Qn), 5, 1, idx, dist, o)
    assert e.value.status == mrpt.MRPT_ENONFINITE
    o.check_finite = 0
    o.precision = mrpt.MRPT_BF16_RERANK
    o.rerank_factor = 200
    with pytest.raises(mrpt.MrptError):
        mrpt.mrpt_query_ex(g.handle, Qd, 5, 1, idx, dist, o)
    # a failed call leaves the outputs untouched and a later call works
    mrpt.mrpt_query(g.handle, Qd, 5, 1, idx, dist)
    torch.cuda.synchronize()
    g.close()


@pytest.mark.parametrize("precision", [mrpt.MRPT_FP32, mrpt.MRPT_BF16_RERANK])
def test_nonfinite_query_row_unchecked(precision):
    # with the finiteness check off (the default) a NaN or Inf row gives
    # in-range results (ids in [-1, n), padding where no distance compares),
    # and every other row its usual answer
    _print_case(f"non-finite query rows, check off, precision {precision}")
    X, Q = _small(3000, 32, 6, 5, seed=12, nq=40)
    g = build(X, 6, 5, 0.4, 3)
    try:
        Qd = dev(Q)
        ref_i, ref_d, ref_s = query(g, Qd, 10, 2, precision=precision)
        Qn = Q.copy()
        Qn[3, 5] = np.nan
        Qn[17, :] = np.inf
        Qn[29, 0] = -np.inf
        gi, gd, sc = query(g, dev(Qn), 10, 2, precision=precision)
        assert np.all((gi >= -1) & (gi < len(X)))
        for r in (3, 17, 29):
            real = gi[r] >= 0
            assert np.all(np.isnan(gd[r][real]) | (gd[r][real] >= 0))
            assert np.all(np.isinf(gd[r][~real]))
        keep = np.setdiff1d(np.arange(len(Q)), [3, 17, 29])
        assert np.array_equal(gi[keep], ref_i[keep]) and np.array_equal(gd[keep], ref_d[keep])
        assert np.array_equal(sc[keep], ref_s[keep])
    finally:
        g.close()


def test_query_pointer_checks():
    # host memory or a wrong shape is refused before any launch
    _print_case("query pointer checks")
    X, Q = _small(1000, 8, 2, 3, seed=13)
    g = build(X, 2, 3, 0.5, 1)
    try:
        import ctypes
        lib = mrpt.load()
        Qh = np.ascontiguousarray(Q)
        idx = torch.empty((len(Q), 5), dtype=torch.int32, device="cuda")
        dist = torch.empty((len(Q), 5), dtype=torch.float32, device="cuda")
        st = lib.mrpt_query(g.handle, ctypes.c_void_p(Qh.ctypes.data), len(Q), 5, 1,
                            ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()), None)
        assert st == mrpt.MRPT_EINVAL and "Q" in mrpt.mrpt_last_error()
        oh = np.zeros((len(Q), 5), np.int32)
        st = lib.mrpt_query(g.handle, ctypes.c_void_p(dev(Q).data_ptr()), len(Q), 5, 1,
                            ctypes.c_void_p(oh.ctypes.data), ctypes.c_void_p(dist.data_ptr()), None)
        assert st == mrpt.MRPT_EINVAL and "out_idx" in mrpt.mrpt_last_error()
        with pytest.raises(ValueError):
            g.query(dev(Q[:, :7]), 5, 1)
        with pytest.raises(ValueError):
            mrpt.mrpt_query(g.handle, dev(Q), 5, 1, idx[:, :4].contiguous(), dist)
    finally:
        g.close()


def ctypes_build_host_pointer(X):
    import ctypes
    lib = mrpt.load()
    h = ctypes.c_void_p()
    Xc = np.ascontiguousarray(X)
    return lib.mrpt_build(ctypes.c_void_p(Xc.ctypes.data), Xc.shape[0], Xc.shape[1], 2, 3, 0.5, 1,
                          ctypes.byref(h))


@pytest.mark.parametrize("kernel", ["0", "1", "default"])
def test_vote_kernel_variants_agree(kernel, monkeypatch):
    # the multi-pass vote kernel with its leaf directory (MRPT_VOTE_KERNEL=0,
    # which also makes the build create the directory), the multi-pass kernel
    # without it (1) and the default choice (single-pass id map + repeat queue
    # where it fits) compute the same candidate
    # sets.  700 queries give every persistent workgroup several queries; the
    # depth-1 and the 140-tree cases have more windows than the single-pass
    # kernel holds in registers
    _print_case(f"vote kernel {kernel}")
    if kernel == "default":
        monkeypatch.delenv("MRPT_VOTE_KERNEL", raising=False)
    else:
        monkeypatch.setenv("MRPT_VOTE_KERNEL", kernel)
    for n, d, T, depth, v in ((6000, 24, 20, 5, 1), (7000, 16, 12, 6, 3), (3000, 8, 9, 4, 5), (2500, 8, 140, 3, 20),
                              (150000, 8, 10, 7, 2), (140000, 8, 70, 9, 1), (40000, 8, 20, 1, 2),
                              (1_100_000, 4, 30, 12, 5), (200_000, 4, 40, 10, 17), (200_000, 4, 120, 10, 4)):
        X, Q = _small(n, d, T, depth, seed=n + T, nq=700)
        orc = oracle.build_index(X, T, depth, 0.5, 3)
        g = build(X, T, depth, 0.5, 3)
        ref = oracle.query(orc, Q, 5, v, want_sets=True)
        ids, cnt = votes(g, dev(Q), v)
        for q in range(len(Q)):
            assert np.array_equal(ids[q], ref["s_ids"][q]), f"n={n} T={T} v={v} query {q}"
            assert np.array_equal(cnt[q], ref["s_votes"][q])
        g.close()


@pytest.mark.parametrize("n,d,T,depth,integer", [(5000, 16, 6, 5, False), (4099, 8, 5, 7, True),
                                                 (3000, 24, 3, 0, False), (777, 4, 9, 9, True),
                                                 (20000, 3, 2, 11, True), (65537, 12, 3, 12, False)])
def test_device_build_matches_host_and_oracle(n, d, T, depth, integer, monkeypatch):
    # the GPU build (projection kernel, then each level cut by rank: a radix
    # select of every node's middle (projection, id) key and a partition,
    # with nodes over 8192 keys cut by many workgroups and smaller ones by one
    # in LDS; or, with MRPT_BUILD_SORT=1, a segmented sort of every level)
    # and the host build give the oracle's trees bit for bit; integer data in
    # {0..3} ties projections often, depth 0 is one leaf, and the scratch
    # limit forces groups of two trees.  n = 20000 and 65537 reach the
    # many-workgroup cut (levels 0-1 and 0-3; 65537 / 8 = 8192.1 keys per
    # node at level 3)
    _print_case(f"device build n={n} d={d} T={T} depth={depth} integer={integer}")
    monkeypatch.setenv("MRPT_BUILD_LIMIT", str(2 * n * (4 * max(depth, 1) + 16)))
    X, _ = _small(n, d, T, depth, seed=n + depth, integer=integer)
    orc = oracle.build_index(X, T, depth, 0.5, 11)
    for on_device, sort in ((True, "0"), (True, "1"), (False, "0")):
        monkeypatch.setenv("MRPT_BUILD_SORT", sort)
        g = mrpt.Index(dev(X), T, depth, 0.5, 11, on_device=on_device)
        assert np.array_equal(mrpt.mrpt_export_leaf_offsets(g.handle), orc.off)
        for t in range(T):
            splits, perm = mrpt.mrpt_export_tree(g.handle, t)
            assert np.array_equal(splits.view(np.uint32), orc.splits[t].view(np.uint32)), \
                f"on_device={on_device} sort={sort} tree {t} splits"
            assert np.array_equal(perm, orc.perm[t]), f"on_device={on_device} sort={sort} tree {t} perm"
        g.close()


@pytest.mark.parametrize("n,d,a", [(3000, 100, 1.0), (2500, 300, 1.0), (2000, 600, 0.3)])
def test_device_build_long_vectors(n, d, a):
    """Projection vectors of more than 64 nonzeros (dense RP trees, a = 1;
    a = 0.3 at d = 600): the GPU build's projection and the routing take a
    vector 64 entries at a time, within one feature chunk (d = 100) or over
    chunks of 252 features with several windows per chunk (d = 300, 600).
    Trees and leaves equal the oracle's bit for bit."""
    _print_case(f"device build, long vectors n={n} d={d} a={a}")
    T, depth = 4, 6
    X, Q = _small(n, d, T, depth, seed=n + d, nq=130)
    orc = oracle.build_index(X, T, depth, a, 17)
    g = mrpt.Index(dev(X), T, depth, a, 17)
    try:
        assert g.info.built_on_device == 1 and g.info.max_row_nnz > 64
        assert np.array_equal(mrpt.mrpt_export_leaf_offsets(g.handle), orc.off)
        for t in range(T):
            splits, perm = mrpt.mrpt_export_tree(g.handle, t)
            assert np.array_equal(splits.view(np.uint32), orc.splits[t].view(np.uint32)), f"tree {t} splits"
            assert np.array_equal(perm, orc.perm[t]), f"tree {t} perm"
        for nq in (1, 130):
            assert np.array_equal(leaves(g, dev(Q[:nq])), oracle.route(orc, Q[:nq])), f"nq={nq}"
    finally:
        g.close()


@pytest.mark.parametrize("k,precision", [(10, None), (100, None), (10, "bf16")])
def test_gist_like_shape_full_parity(k, precision):
    # the gist-like data (d = 960, values in (0, 1)) at a size the oracle
    # handles in seconds: 16 trees of depth 5, v = 5, k = 10 and 100 (the
    # single-pass vote kernel serves it: 15 windows of 64 ids per leaf); the
    # search runs 64 lanes x 4 float4 per row, the bf16 arm 64 lanes x 2 x 8
    w = W.GIST_LIKE.scaled(n=30000, nq=48, T=16, depth=5)
    _print_case(f"gist-like shape n={w.n} T={w.T} depth={w.depth} k={k} {precision or 'fp32'}")
    X, Q = W.data(w), W.queries(w)
    prec = mrpt.MRPT_BF16_RERANK if precision == "bf16" else None
    _full_compare(X, Q, w.T, w.depth, w.a, w.index_seed, k, w.v, precision=prec)


@pytest.mark.parametrize("precision", [mrpt.MRPT_FP8_RERANK, mrpt.MRPT_BF16_RERANK])
def test_prefilter_arm_exact_when_rerank_covers_s(precision):
    # fp8 / bf16 prefilter + float32 rerank + float64 recheck: when
    # rerank_factor * k is at least |S| every candidate is reranked (the
    # prefilter ranking is skipped), so the arm must return the oracle's k
    # nearest of S whatever the low-precision rounding did
    _print_case(f"prefilter arm {precision}, rerank covering S")
    X, Q = _small(6000, 32, 8, 5, seed=41, nq=70)
    opts = dict(precision=precision, rerank_factor=100)
    gi, gd, ref = _full_compare(X, Q, 8, 5, 0.5, 5, 5, 4, precision=None)
    g = build(X, 8, 5, 0.5, 5)
    assert int(ref["s_count"].max()) <= 5 * 100
    fi, fd, fs = query(g, dev(Q), 5, 4, **opts)
    assert np.array_equal(fs, ref["s_count"])
    check_knn(X, Q, fi, fd, ref["idx"], ref["dist"], exact_ids=False,
              S=[set(s.tolist()) for s in ref["s_ids"]])
    g.close()


@pytest.mark.parametrize("k", [10, 100])
def test_fp8_arm_gist_like_shape(k):
    # gist-like rows (d = 960, values in (0, 1)) through the fp8 arm with the
    # default rerank factor 4: results lie in S, carry float32-exact
    # distances, are ordered by (distance, id) and padded; their overlap with
    # the fp32 arm (the fp8 rounding can push a true neighbour out of the
    # reranked set) is reported
    w = W.GIST_LIKE.scaled(n=30000, nq=48, T=16, depth=5)
    _print_case(f"fp8 arm gist-like shape k={k}")
    X, Q = W.data(w), W.queries(w)
    g = build(X, w.T, w.depth, w.a, w.index_seed)
    Qd = dev(Q)
    ids, _ = votes(g, Qd, w.v, with_counts=False)
    pi, pd, ps = query(g, Qd, k, w.v)
    fi, fd, fs = query(g, Qd, k, w.v, precision=mrpt.MRPT_FP8_RERANK)
    assert np.array_equal(fs, ps)
    overlap = []
    for q in range(len(Q)):
        nreal = min(k, len(ids[q]))
        real = fi[q][:nreal]
        assert np.all(fi[q][nreal:] == -1) and np.all(np.isinf(fd[q][nreal:]))
        assert set(real.tolist()) <= set(ids[q].tolist()) and len(set(real.tolist())) == nreal
        d64 = dist64(X, Q[q], real)
        assert np.all(np.abs(fd[q][:nreal].astype(np.float64) - d64) <= 1e-5 * d64 + 1e-6)
        # ordered by float32 distance, except inside the float64 recheck window
        # (recheck_rel 1e-6 of the k-th distance), which is ordered by float64
        assert all(fd[q][r] <= fd[q][r + 1] * (1 + 2e-6) for r in range(nreal - 1))
        overlap.append(len(set(real.tolist()) & set(pi[q][:nreal].tolist())) / max(nreal, 1))
    print(f"[fp8] gist-like shape k={k}: mean overlap with the fp32 arm {np.mean(overlap):.4f}", flush=True)
    g.close()


@pytest.mark.parametrize("on_device", [True, False])
def test_exact_nnz_mode_parity(on_device):
    """Exactly ceil(a d) nonzeros per projection vector (footnote of Sec. II-D):
    vectors, trees, leaves, votes and k-NN against the oracle's exact mode."""
    w = W.MIXTURE_128.scaled(nq=200)
    _print_case(f"exact_nnz mixture128 on_device={on_device}")
    X, Q = W.data(w), W.queries(w)
    orc = oracle.build_index(X, w.T, w.depth, w.a, w.index_seed, exact_nnz=True)
    gpu = mrpt.Index(dev(X), w.T, w.depth, w.a, w.index_seed, on_device=on_device, exact_nnz=True)
    try:
        rowptr, col, val = mrpt.mrpt_export_projection(gpu.handle)
        R = np.zeros_like(orc.R)
        for r in range(R.shape[0]):
            R[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
        assert np.array_equal(R.view(np.uint32), orc.R.view(np.uint32))
        assert np.all(np.diff(rowptr) == oracle.exact_nnz_count(w.d, w.a))
        for t in range(w.T):
            splits, perm = mrpt.mrpt_export_tree(gpu.handle, t)
            assert np.array_equal(splits.view(np.uint32), orc.splits[t].view(np.uint32)), f"tree {t}"
            assert np.array_equal(perm, orc.perm[t]), f"tree {t}"
        Qd = dev(Q)
        assert np.array_equal(leaves(gpu, Qd), oracle.route(orc, Q))
        for v in (1, 3):
            ref = oracle.query(orc, Q, w.k, v, want_sets=True)
            ids, cnt = votes(gpu, Qd, v)
            for q in range(len(Q)):
                assert np.array_equal(ids[q], ref["s_ids"][q]) and np.array_equal(cnt[q], ref["s_votes"][q])
            gi, gd, _ = query(gpu, Qd, w.k, v)
            check_knn(X, Q, gi, gd, ref["idx"], ref["dist"], exact_ids=False,
                      S=[set(s.tolist()) for s in ref["s_ids"]])
    finally:
        gpu.close()


@pytest.mark.parametrize("directory", [False, True])
def test_vote_queue_overflow_is_recounted(directory, monkeypatch):
    # a repeat queue capped at 1024 entries overflows for these queries; the
    # single-pass kernel marks them and a multi-pass kernel recounts them (the
    # one with the leaf directory when the index has one: built here by
    # forcing the multi-pass choice at build time, then lifting it)
    _print_case(f"vote queue overflow, recount with directory={directory}")
    n, d, T, depth, v = 100_000, 8, 24, 7, 2
    X, Q = _small(n, d, T, depth, seed=5, nq=300)
    orc = oracle.build_index(X, T, depth, 0.5, 3)
    if directory:
        monkeypatch.setenv("MRPT_VOTE_KERNEL", "0")
    g = build(X, T, depth, 0.5, 3)
    monkeypatch.delenv("MRPT_VOTE_KERNEL", raising=False)
    monkeypatch.setenv("MRPT_VOTE_QUEUE_CAP", "1024")
    try:
        ref = oracle.query(orc, Q, 5, v, want_sets=True)
        leafsz = np.diff(orc.off)
        repeats = np.array([leafsz[ref["leaf"][q]].sum() for q in range(len(Q))]) - \
            oracle.query(orc, Q, 5, 1)["s_count"]
        assert (repeats > 1024).mean() > 0.5          # most queries do overflow
        ids, cnt = votes(g, dev(Q), v)
        for q in range(len(Q)):
            assert np.array_equal(ids[q], ref["s_ids"][q]), f"query {q}"
            assert np.array_equal(cnt[q], ref["s_votes"][q])
        gi, gd, sc = query(g, dev(Q), 5, v)
        assert np.array_equal(sc, ref["s_count"])
    finally:
        g.close()
