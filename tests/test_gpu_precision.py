"""GPU parity of the precision arms (bfloat16 or fp8 prefilter, float32
rerank, float64 recheck) against the oracle's model of them, through the C ABI.

What is compared:
  * the low-precision rows of the index: bfloat16 patterns and E4M3 codes and
    per-row scales bit for bit, the fp8 rows' squared norms within the float32
    summation bound;
  * the kept list of the prefilter (the best kp = rerank_factor*k of S under
    the low-precision score): equal to the oracle's, except for candidates
    whose float64 score lies within the float32 evaluation bound E of the
    kp-th score, where either side of the cut is correct;
  * the answers: the k nearest (float64, order (distance, id)) of the kept
    list, with every returned distance within 1e-5 of float64;
  * a constructed near-tie at rank k, equal in float32 and unequal in float64,
    which only the float64 recheck orders correctly.

The float32 score bound: the GPU evaluates ||q||^2 + ||x~||^2 - 2 q.x~ with
three sums of d terms (any order) and at most four further roundings, so
|score32 - score| <= gamma_{d+4} (||q|| + ||x~||)^2 with gamma_m = m u / (1 - m u),
u = 2^-24 (Cauchy-Schwarz bounds the three sums of magnitudes).
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import ARM, build, check_answers, check_kept, dev, dist64, gamma, gpu_keep, gpu_rows, query  # noqa: E402,E501
from paper_1509_06957_amd import mrpt  # noqa: E402


def _case(name):
    print(f"[case] {name}", flush=True)


# ----------------------------------------------------------------- rows

def _mixed_rows():
    rng = np.random.default_rng(17)
    X = (rng.standard_normal((5000, 64)) * rng.uniform(1e-3, 50, (5000, 1))).astype(np.float32)
    X[3] = 0.0
    X[4, :] = -0.0
    X[5, ::2] = 1e-30                                     # values that round to zero
    return X


@pytest.mark.parametrize("shape", ["gist_like", "mixed"])
def test_lowp_rows_bit_exact(shape):
    if shape == "gist_like":
        w = W.GIST_LIKE.scaled(n=30000, nq=4, T=4, depth=5)
        X = W.data(w)
    else:
        X = _mixed_rows()
    n, d = X.shape
    _case(f"low-precision rows {shape} n={n} d={d}")
    g = build(X, 2, 3, 0.5, 1)
    try:
        b, _ = gpu_rows(g, mrpt.MRPT_BF16_RERANK, n, d)
        assert np.array_equal(b, oracle.bf16_round(X))
        c, sn = gpu_rows(g, mrpt.MRPT_FP8_RERANK, n, d)
        codes, scale, norm = oracle.fp8_rows(X)
        bad = np.argwhere(c != codes)
        assert bad.size == 0, f"{len(bad)} codes differ, first {bad[:5].tolist()}: " \
                              f"{c[tuple(bad[0])] if bad.size else ''} vs {codes[tuple(bad[0])] if bad.size else ''}"
        assert np.array_equal(sn[:, 0].view(np.uint32), scale.view(np.uint32))
        assert np.all(np.abs(sn[:, 1] - norm) <= gamma(d + 2) * norm)
    finally:
        g.close()


# ----------------------------------------------------------------- kept lists and answers

def _arm_case(X, Q, T, depth, a, seed, k, v, precision, rerank_factor=4):
    kp = k * rerank_factor
    orc = oracle.build_index(X, T, depth, a, seed)
    ref = oracle.query_prefilter(orc, Q, k, v, ARM[precision], kp)
    g = build(X, T, depth, a, seed)
    try:
        Qd = dev(Q)
        g_sc, g_keep = gpu_keep(g, Qd, k, v, precision, rerank_factor)
        banded = check_kept(X, Q, ref, g_sc, g_keep, kp, ARM[precision])
        gi, gd, sc = query(g, Qd, k, v, precision=precision, rerank_factor=rerank_factor)
        assert np.array_equal(sc, ref["s_count"])
        check_answers(X, Q, ref, g_keep, gi, gd, kp)
    finally:
        g.close()
    ranked = int((ref["s_count"] > kp).sum())
    print(f"[arm] precision={precision} k={k} kp={kp}: {ranked}/{len(Q)} queries ranked, "
          f"{banded} with a candidate inside the float32 band at the cut", flush=True)
    assert ranked > len(Q) // 2
    return banded


@pytest.mark.parametrize("precision", [mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
@pytest.mark.parametrize("k", [10, 100])
def test_arm_gist_like_shape(precision, k):
    # gist-like rows (d = 960, values in (0, 1)); bfloat16 and E4M3 are lossy
    # here.  At v = 5 |S| is about 200 (above kp = 40 for k = 10); k = 100
    # (kp = 400) takes v = 3, where |S| is about 660, so that the prefilter
    # ranks every query at both k
    w = W.GIST_LIKE.scaled(n=30000, nq=48, T=16, depth=5)
    v = w.v if k == 10 else 3
    _case(f"arm {precision} gist-like shape k={k} v={v}")
    X, Q = W.data(w), W.queries(w)
    _arm_case(X, Q, w.T, w.depth, w.a, w.index_seed, k, v, precision)


@pytest.mark.parametrize("precision", [mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
def test_arm_mixture128(precision):
    # Gaussian-mixture rows with negative values, d = 128 (the d <= 128 forms)
    w = W.MIXTURE_128
    _case(f"arm {precision} mixture-128")
    X, Q = W.data(w), W.queries(w)
    _arm_case(X, Q, w.T, w.depth, w.a, w.index_seed, w.k, w.v, precision)


@pytest.mark.parametrize("precision", [mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
def test_arm_mnist_like(precision):
    # integers in [0, 255]: bfloat16 is exact (kept lists identical), E4M3 is not
    w = W.MNIST_LIKE.scaled(nq=300)
    _case(f"arm {precision} mnist-like")
    X, Q = W.data(w), W.queries(w)
    banded = _arm_case(X, Q, w.T, w.depth, w.a, w.index_seed, w.k, w.v, precision)
    if precision == mrpt.MRPT_BF16_RERANK:
        assert banded == 0


# ----------------------------------------------------------------- the float64 recheck

def _near_tie_rows(d=32):
    """q = 0; ids 0..8 at distances 10, 15, ..., 50; ids 9 and 10 both at
    float32 distance 64 exactly, but id 9 holds (64, 0.01, 0, ...), whose
    float64 distance is 64.00000078, and id 10 holds (64, 0, ...); ids 11..255
    far away.  Every float32 summation order of id 9's two nonzero squares
    gives 4096 (0.0001 is below half an ulp of 4096)."""
    X = np.zeros((256, d), np.float32)
    X[:9, 0] = 10 + 5 * np.arange(9)
    X[9, 0], X[9, 1] = 64.0, 0.01
    X[10, 0] = 64.0
    X[11:, 0] = 100 + np.arange(245)
    Q = np.zeros((3, d), np.float32)
    return X, Q


@pytest.mark.parametrize("precision", [mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
def test_recheck_orders_a_float32_tie_by_float64(precision):
    _case(f"near-tie at rank k, precision {precision}")
    X, Q = _near_tie_rows()
    k = 10
    # the oracle: id 10 is nearer than id 9 in float64
    bi, bd = oracle.bruteforce(X, Q, k)
    assert bi[0].tolist() == list(range(9)) + [10] and bd[0, 9] == 64.0 and bd[0, 9] < dist64(X, Q[0], [9])[0]
    assert np.float32(np.float32(64) * np.float32(64) + np.float32(0.01) * np.float32(0.01)) == np.float32(4096)
    g = build(X, 1, 0, 1.0, 1)                          # one leaf holding every point, v = 1: S = X
    try:
        Qd = dev(Q)
        fi, fd, _ = query(g, Qd, k, 1)
        # the float32 arm sees a tie at 64 and orders it by id: id 9 at rank k
        assert fi[0, 9] == 9 and fd[0, 9] == 64.0
        gi, gd, sc = query(g, Qd, k, 1, precision=precision)
        assert sc[0] == 256 > 4 * k                       # the prefilter ranks S
        assert gi[0].tolist() == bi[0].tolist(), f"{gi[0]} vs {bi[0]}"
        assert gd[0, 9] == 64.0
    finally:
        g.close()
