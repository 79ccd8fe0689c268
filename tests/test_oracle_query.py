"""Pins of the oracle's query path (Alg. 3-4, Sec. III, Sec. I-A).

Each test checks the oracle against something it does not compute itself:
scipy's distance routine, a brute-force recount of votes over all leaves, the
special cases that reduce voting search to exact k-NN, and invariants of the
voting definitions.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_1509_06957_amd import workloads as W


def _scipy_knn(X, Q, k):
    D = cdist(Q.astype(np.float64), X.astype(np.float64))
    idx = np.zeros((len(Q), k), np.int64)
    dist = np.zeros((len(Q), k))
    for q in range(len(Q)):
        order = np.lexsort((np.arange(X.shape[0]), D[q]))[:k]
        idx[q], dist[q] = order, D[q, order]
    return idx, dist


def _route_py(index, P_q, t):
    """Descend tree t with the projections P_q[t*depth + level]: left iff <= split."""
    node = 0
    for level in range(index.depth):
        node = 2 * node + 1 if P_q[t * index.depth + level] <= index.splits[t, node] else 2 * node + 2
    return node - ((1 << index.depth) - 1)


@pytest.fixture(scope="module")
def mixture_small():
    w = W.MIXTURE_128.scaled(n=4000, nq=60)
    X, Q = W.data(w), W.queries(w)
    idx = oracle.build_index(X, 10, 5, w.a, w.index_seed)
    return w, X, Q, idx


def test_bruteforce_matches_scipy():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((3000, 40)).astype(np.float32)
    Q = rng.standard_normal((25, 40)).astype(np.float32)
    i1, d1 = oracle.bruteforce(X, Q, 15)
    i2, d2 = _scipy_knn(X, Q, 15)
    assert np.array_equal(i1, i2)
    assert np.allclose(d1, d2, rtol=1e-13, atol=0)


def test_bruteforce_tie_order_is_by_id():
    X = np.zeros((10, 3), np.float32)
    X[:, 0] = [1, 2, 1, 2, 1, 3, 0, 1, 2, 1]
    Q = np.zeros((1, 3), np.float32)
    i, d = oracle.bruteforce(X, Q, 6)
    assert i[0].tolist() == [6, 0, 2, 4, 7, 9]


def test_depth_zero_vote_one_is_bruteforce():
    # depth 0: one leaf holding every point; v = 1 makes S the whole data set
    rng = np.random.default_rng(8)
    X = rng.standard_normal((700, 24)).astype(np.float32)
    Q = rng.standard_normal((30, 24)).astype(np.float32)
    idx = oracle.build_index(X, 3, 0, 0.3, seed=2)
    r = oracle.query(idx, Q, 12, 1)
    bi, bd = _scipy_knn(X, Q, 12)
    assert np.array_equal(r["idx"], bi)
    assert np.allclose(r["dist"], bd, rtol=1e-13)
    assert np.all(r["s_count"] == 700)


def test_routing_matches_independent_descent(mixture_small):
    w, X, Q, idx = mixture_small
    P = oracle.project(Q, idx.R)
    leaf = oracle.route(idx, Q)
    for q in range(len(Q)):
        for t in range(idx.T):
            assert leaf[q, t] == _route_py(idx, P[q], t)


def test_votes_recount_over_all_leaves(mixture_small):
    # recount F(x; q) by scanning every leaf of every tree (Sec. III-A)
    w, X, Q, idx = mixture_small
    r = oracle.query(idx, Q, w.k, 1, want_sets=True)
    n = idx.n
    for q in range(len(Q)):
        F = np.zeros(n, np.int64)
        for t in range(idx.T):
            for L in range(1 << idx.depth):
                if L == r["leaf"][q, t]:
                    F[idx.leaf(t, L)] += 1
        touched = np.nonzero(F)[0]
        assert np.array_equal(r["s_ids"][q], touched)
        assert np.array_equal(r["s_votes"][q], F[touched])
        assert F.min() >= 0 and F.max() <= idx.T
        assert F.sum() == sum(len(idx.leaf(t, r["leaf"][q, t])) for t in range(idx.T))


def test_candidate_bound_and_monotone_in_v(mixture_small):
    w, X, Q, idx = mixture_small
    bound = idx.T * int(np.max(np.diff(idx.off)))
    prev = None
    for v in range(1, idx.T + 1):
        r = oracle.query(idx, Q, w.k, v, want_sets=True)
        assert np.all(r["s_count"] <= bound)
        sets = [set(s.tolist()) for s in r["s_ids"]]
        if prev is not None:
            assert all(a <= b for a, b in zip(sets, prev))
        prev = sets


def test_vote_threshold_T_is_intersection(mixture_small):
    w, X, Q, idx = mixture_small
    r = oracle.query(idx, Q, w.k, idx.T, want_sets=True)
    for q in range(len(Q)):
        inter = set(idx.leaf(0, r["leaf"][q, 0]).tolist())
        for t in range(1, idx.T):
            inter &= set(idx.leaf(t, r["leaf"][q, t]).tolist())
        assert set(r["s_ids"][q].tolist()) == inter
        assert np.all(r["s_votes"][q] == idx.T)


def test_recall_identity(mixture_small):
    # under the total order (distance, id): A cap K == S cap K
    w, X, Q, idx = mixture_small
    bi, bd = _scipy_knn(X, Q, w.k)
    for v in (1, 2, 4):
        r = oracle.query(idx, Q, w.k, v, want_sets=True)
        for q in range(len(Q)):
            A = set(r["idx"][q].tolist()) - {-1}
            K = set(bi[q].tolist())
            S = set(r["s_ids"][q].tolist())
            assert A & K == S & K


def test_knn_in_set_is_exact(mixture_small):
    w, X, Q, idx = mixture_small
    r = oracle.query(idx, Q, w.k, 2, want_sets=True)
    for q in range(len(Q)):
        S = r["s_ids"][q]
        if len(S) == 0:
            assert np.all(r["idx"][q] == -1) and np.all(np.isinf(r["dist"][q]))
            continue
        si, sd = _scipy_knn(X[S], Q[q:q + 1], min(w.k, len(S)))
        m = min(w.k, len(S))
        assert np.array_equal(r["idx"][q, :m], S[si[0]])
        assert np.allclose(r["dist"][q, :m], sd[0], rtol=1e-13)
        assert np.all(r["idx"][q, m:] == -1) and np.all(np.isinf(r["dist"][q, m:]))


def test_single_tree_is_bruteforce_on_its_leaf():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((900, 16)).astype(np.float32)
    Q = rng.standard_normal((20, 16)).astype(np.float32)
    idx = oracle.build_index(X, 1, 3, 0.5, seed=3)
    r = oracle.query(idx, Q, 5, 1)
    for q in range(len(Q)):
        leaf = idx.leaf(0, r["leaf"][q, 0])
        si, sd = _scipy_knn(X[leaf], Q[q:q + 1], 5)
        assert np.array_equal(r["idx"][q], leaf[si[0]])


def test_self_query_gets_every_vote():
    # continuous data: a data point routes to its own leaf in every tree
    rng = np.random.default_rng(10)
    X = rng.standard_normal((2000, 20)).astype(np.float32)
    idx = oracle.build_index(X, 12, 6, 0.25, seed=4)
    qs = np.arange(2000)
    r = oracle.query(idx, X[qs], 3, idx.T, want_sets=True)
    for j, i in enumerate(qs):
        assert i in set(r["s_ids"][j].tolist())
        assert r["idx"][j, 0] == i and r["dist"][j, 0] == 0.0


def test_more_trees_superset():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((3000, 30)).astype(np.float32)
    Q = rng.standard_normal((25, 30)).astype(np.float32)
    small = oracle.build_index(X, 5, 6, 0.2, seed=9)
    big = oracle.build_index(X, 9, 6, 0.2, seed=9)
    assert np.array_equal(big.perm[:5], small.perm) and np.array_equal(big.splits[:5], small.splits)
    rs = oracle.query(small, Q, 10, 2, want_sets=True)
    rb = oracle.query(big, Q, 10, 2, want_sets=True)
    for q in range(len(Q)):
        assert set(rs["s_ids"][q].tolist()) <= set(rb["s_ids"][q].tolist())


def test_short_candidate_sets_are_padded():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((64, 8)).astype(np.float32)
    idx = oracle.build_index(X, 2, 4, 0.5, seed=1)
    r = oracle.query(idx, X[:5] + 0.01, 8, 2)
    assert np.all(r["s_count"] <= 4)
    for q in range(5):
        c = r["s_count"][q]
        assert np.all(r["idx"][q, c:] == -1)
        assert np.all(np.isinf(r["dist"][q, c:]))
