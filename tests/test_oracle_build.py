"""Pins of the oracle's index construction (Alg. 1-2, Sec. II-A/II-C).

Projection is pinned to exact float64 arithmetic; the trees are pinned by the
characterisation of a median split (checked by code written independently of
the oracle's sort-and-cut): every inner node sends ceil(m/2) points left, all
left points precede all right points in (projection, id) order, and the split
value lies between them.  Leaf sizes are pinned to floor/ceil(n / 2^depth).
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W


def _f64_projection(X, R):
    return X.astype(np.float64) @ R.astype(np.float64).T


def test_projection_exact_on_dyadic_values():
    # integer data and entries with few mantissa bits: every fused multiply-add
    # in the float32 chain is exact, so it equals the float64 product exactly
    rng = np.random.default_rng(1)
    X = rng.integers(0, 256, size=(300, 96)).astype(np.float32)
    R = (rng.integers(-64, 65, size=(20, 96)) / 8.0).astype(np.float32)
    R[rng.random(R.shape) < 0.7] = 0
    P = oracle.project(X, R)
    assert np.array_equal(P.astype(np.float64), _f64_projection(X, R))


def test_projection_within_chain_error_bound():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((500, 200)).astype(np.float32)
    R = oracle.random_matrix(200, 4, 6, 0.1, seed=4)
    P = oracle.project(X, R).astype(np.float64)
    exact = _f64_projection(X, R)
    nnz = (R != 0).sum(axis=1)
    absdot = np.abs(X.astype(np.float64)) @ np.abs(R.astype(np.float64)).T
    bound = absdot * nnz[None, :] * 2.0 ** -24 * 1.01 + 1e-30
    assert np.all(np.abs(P - exact) <= bound)


def test_projection_is_not_transposed_or_shifted():
    # a single nonzero at feature i picks X[:, i] * r exactly
    X = np.arange(12, dtype=np.float32).reshape(3, 4) + 1
    R = np.zeros((2, 4), dtype=np.float32)
    R[0, 1] = 2.0
    R[1, 3] = -0.5
    P = oracle.project(X, R)
    assert np.array_equal(P, np.stack([X[:, 1] * 2.0, X[:, 3] * -0.5], axis=1))


@pytest.mark.parametrize("n", list(range(1, 70)) + [1000, 1023, 1024, 1025, 60000, 1000000])
def test_leaf_sizes_floor_ceil(n):
    for depth in range(0, 13):
        if (1 << depth) > n:
            break
        off = oracle.leaf_offsets(n, depth)
        sizes = np.diff(off)
        assert off[0] == 0 and off[-1] == n
        assert set(np.unique(sizes)) <= {n >> depth, -(-n >> depth)}
        # every inner node sends ceil(m/2) of its m points left
        for level in range(depth):
            span = 1 << (depth - level)
            for s in range(0, 1 << depth, span):
                m = off[s + span] - off[s]
                left = off[s + span // 2] - off[s]
                assert left == (m + 1) // 2


def check_tree_characterisation(X, index, t):
    """Independent check of one tree against the median-split definition."""
    depth, n = index.depth, index.n
    Rt = index.R[t * depth:(t + 1) * depth]
    P = oracle.project(X, Rt)                     # pinned above
    P = np.where(P == 0, np.float32(0), P)        # -0 and +0 are one value
    perm = index.perm[t]
    off = index.off
    assert np.array_equal(np.sort(perm), np.arange(n))
    for L in range(1 << depth):
        leaf = perm[off[L]:off[L + 1]]
        assert np.all(np.diff(leaf) > 0)           # ascending ids inside a leaf
    for level in range(depth):
        span = 1 << (depth - level)
        for j, s in enumerate(range(0, 1 << depth, span)):
            node = (1 << level) - 1 + j
            ids_l = perm[off[s]:off[s + span // 2]]
            ids_r = perm[off[s + span // 2]:off[s + span]]
            m = len(ids_l) + len(ids_r)
            assert len(ids_l) == (m + 1) // 2
            pl, pr = P[ids_l, level], P[ids_r, level]
            kl = max(zip(pl.tolist(), ids_l.tolist()))
            kr = min(zip(pr.tolist(), ids_r.tolist()))
            assert kl < kr
            split = index.splits[t, node]
            assert pl.max() <= split <= pr.min()
            order = sorted(zip(np.concatenate([pl, pr]).tolist(),
                               np.concatenate([ids_l, ids_r]).tolist()))
            if m % 2 == 1:
                assert split == np.float32(order[(m - 1) // 2][0])
            else:
                lo, hi = np.float32(order[m // 2 - 1][0]), np.float32(order[m // 2][0])
                assert split == np.float32(np.float32(lo + hi) * np.float32(0.5))


@pytest.mark.parametrize("n,d,T,depth", [(16, 4, 3, 3), (13, 3, 2, 2), (9, 2, 4, 3), (40, 5, 2, 4)])
def test_tiny_trees_exhaustive(n, d, T, depth):
    rng = np.random.default_rng(n * 31 + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    idx = oracle.build_index(X, T, depth, 0.7, seed=n + d)
    for t in range(T):
        check_tree_characterisation(X, idx, t)


def test_ties_keep_sizes():
    # integer data with many equal projections: the (projection, id) order keeps
    # the ceil(m/2) rule and the leaf sizes
    rng = np.random.default_rng(3)
    X = rng.integers(0, 3, size=(777, 8)).astype(np.float32)
    idx = oracle.build_index(X, 4, 5, 0.3, seed=5)
    for t in range(4):
        check_tree_characterisation(X, idx, t)


def test_mixture_workload_trees():
    w = W.MIXTURE_128.scaled(n=3000)
    X = W.data(w)
    idx = oracle.build_index(X, 3, w.depth, w.a, w.index_seed)
    for t in range(3):
        check_tree_characterisation(X, idx, t)


def test_build_independent_of_thread_count():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2000, 32)).astype(np.float32)
    a = oracle.build_index(X, 6, 5, 0.2, seed=8, nthreads=1)
    b = oracle.build_index(X, 6, 5, 0.2, seed=8, nthreads=4)
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.splits, b.splits)


def test_depth_zero_single_leaf():
    X = np.random.default_rng(0).standard_normal((50, 6)).astype(np.float32)
    idx = oracle.build_index(X, 2, 0, 0.5, seed=1)
    assert idx.splits.shape == (2, 0)
    assert np.array_equal(idx.perm, np.tile(np.arange(50, dtype=np.int32), (2, 1)))


def test_exact_nnz_mode_trees():
    # the exact-count projection mode changes only the vectors: every tree
    # still satisfies the median-split characterisation
    w = W.MIXTURE_128.scaled(n=2500)
    X = W.data(w)
    idx = oracle.build_index(X, 3, w.depth, w.a, w.index_seed, exact_nnz=True)
    assert np.all((idx.R != 0).sum(axis=1) == oracle.exact_nnz_count(w.d, w.a))
    for t in range(3):
        check_tree_characterisation(X, idx, t)
