"""mrpt_query_noalloc (the query entry point that allocates no device memory:
its temporaries live in the library's fixed per-GPU scratch array) against
mrpt_query_ex on the same index and queries: ids, distances and |S| must be
identical (both run the same kernels), on two calls in a row with the second
smaller, in one sub-batch and in several, on the float32 and bfloat16 arms.
"""
import numpy as np
import pytest

from paper_1509_06957_amd import mrpt
from paper_1509_06957_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import dev  # noqa: E402

SCRATCH = 128 << 20


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _run(fn, ix, Qd, k, v, precision):
    nq = Qd.shape[0]
    idx = torch.full((nq, k), -7, dtype=torch.int32, device="cuda")
    dist = torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda")
    s_count = torch.full((nq,), -7, dtype=torch.int32, device="cuda")
    o = mrpt.mrpt_default_opts()
    o.precision = precision
    o.s_count = s_count.data_ptr()
    fn(ix.handle, Qd, k, v, idx, dist, o)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), s_count.cpu().numpy()


def _compare(ix, Q, k, v, precision):
    Qd = dev(Q)
    ri, rd, rs = _run(mrpt.mrpt_query_ex, ix, Qd, k, v, precision)
    ni, nd, ns = _run(mrpt.mrpt_query_noalloc, ix, Qd, k, v, precision)
    assert np.array_equal(ns, rs)
    assert np.array_equal(ni, ri)
    assert np.array_equal(nd.view(np.uint32), rd.view(np.uint32))
    assert (ri >= 0).any()


def _per_query_bytes(T, max_leaf, v, depth, n):
    cap = min(n, T * max_leaf // v)
    return 4 * (T + cap + 1) + 4 * T * depth


@pytest.mark.parametrize("precision", [mrpt.MRPT_FP32, mrpt.MRPT_BF16_RERANK])
def test_noalloc_equals_query_ex_one_sub_batch(precision):
    w = W.MIXTURE_128.scaled(nq=500)
    _case(f"noalloc {w.name} nq 500 then 37, precision {precision}")
    X, Q = W.data(w), W.queries(w)
    ix = mrpt.Index(dev(X), w.T, w.depth, w.a, w.index_seed)
    try:
        assert w.nq * _per_query_bytes(w.T, ix.info.max_leaf, w.v, w.depth, w.n) < SCRATCH
        _compare(ix, Q, w.k, w.v, precision)
        _compare(ix, Q[100:137], w.k, w.v, precision)
    finally:
        ix.close()


@pytest.mark.parametrize("precision", [mrpt.MRPT_FP32, mrpt.MRPT_BF16_RERANK])
def test_noalloc_equals_query_ex_several_sub_batches(precision):
    # 200,000 points, 64 trees of depth 6 (leaves of 3,125), v = 1: up to
    # 200,000 candidates (800 KB) per query, so 600 queries take four
    # sub-batches of the scratch and the second call (170 queries) two
    rng = np.random.default_rng(5)
    n, d, T, depth, v, k = 200_000, 32, 64, 6, 1, 10
    means = rng.normal(0, 2, (16, d)).astype(np.float32)
    X = (means[rng.integers(0, 16, n)] + rng.normal(0, 1, (n, d))).astype(np.float32)
    Q = (means[rng.integers(0, 16, 600)] + rng.normal(0, 1, (600, d))).astype(np.float32)
    _case(f"noalloc n={n} T={T} depth={depth} v={v} nq 600 then 170, precision {precision}")
    ix = mrpt.Index(dev(X), T, depth, 1 / np.sqrt(d), 17)
    try:
        per_q = _per_query_bytes(T, ix.info.max_leaf, v, depth, n)
        assert 600 * per_q > 3 * SCRATCH and 170 * per_q > SCRATCH
        _compare(ix, Q, k, v, precision)
        _compare(ix, Q[400:570], k, v, precision)
    finally:
        ix.close()


def test_noalloc_errors_and_recovery():
    w = W.MIXTURE_128.scaled(nq=64)
    _case("noalloc error paths")
    X, Q = W.data(w), W.queries(w)
    ix = mrpt.Index(dev(X), w.T, w.depth, w.a, w.index_seed)
    try:
        Qn = Q.copy()
        Qn[3, 5] = np.nan
        idx = torch.full((len(Q), w.k), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((len(Q), w.k), -7.0, dtype=torch.float32, device="cuda")
        o = mrpt.mrpt_default_opts()
        o.check_finite = 1
        with pytest.raises(mrpt.MrptError) as e:
            mrpt.mrpt_query_noalloc(ix.handle, dev(Qn), w.k, w.v, idx, dist, o)
        assert e.value.status == mrpt.MRPT_ENONFINITE
        torch.cuda.synchronize()
        assert (idx.cpu().numpy() == -7).all()
        with pytest.raises(mrpt.MrptError) as e:
            mrpt.mrpt_query_noalloc(ix.handle, dev(Q), w.k, w.T + 1, idx, dist, o)
        assert e.value.status == mrpt.MRPT_EINVAL
        # the finiteness check passes on finite queries and the results follow
        mrpt.mrpt_query_noalloc(ix.handle, dev(Q), w.k, w.v, idx, dist, o)
        torch.cuda.synchronize()
        _compare(ix, Q, w.k, w.v, mrpt.MRPT_FP32)
    finally:
        ix.close()


def test_noalloc_rejects_a_query_beyond_the_scratch():
    # one tree of depth 0 over 34,000,000 points: S = X, and one query's
    # candidate list alone (4 * 34e6 bytes) exceeds the 128 MiB scratch
    n = 34_000_000
    _case(f"noalloc beyond the scratch: n={n} d=1 T=1 depth=0")
    X = torch.arange(n, dtype=torch.float32, device="cuda").reshape(n, 1)
    ix = mrpt.Index(X, 1, 0, 1.0, 3, on_device=False)
    try:
        assert _per_query_bytes(1, ix.info.max_leaf, 1, 0, n) > SCRATCH
        Qd = torch.zeros((2, 1), dtype=torch.float32, device="cuda")
        idx = torch.full((2, 5), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((2, 5), -7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(mrpt.MrptError) as e:
            mrpt.mrpt_query_noalloc(ix.handle, Qd, 5, 1, idx, dist)
        assert e.value.status == mrpt.MRPT_EINVAL and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert (idx.cpu().numpy() == -7).all() and (dist.cpu().numpy() == -7.0).all()
    finally:
        ix.close()
        del X
        torch.cuda.empty_cache()
