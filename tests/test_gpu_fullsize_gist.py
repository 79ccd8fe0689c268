"""Full-size checks on the gist-like workload (n = 1,000,000, d = 960, 10,000
queries, T = 200, depth = 10, v = 5, k = 10 and 100) in the launch
configuration of a whole-batch query call.

The oracle's full index takes minutes of host time at this size, so it is
pinned where the oracle can compute outputs one by one: a tree does not
depend on T, so the oracle builds trees 0 and 1 alone and those trees, their
projection vectors and every query's leaf in them must match bit for bit.
The query results are checked by properties that hold at any size: the
candidate sets equal a recount of the leaf lists, every listed id has at
least v votes, the returned ids are the k nearest members of S under
(distance, id) with float64 distances, and recall against float64 brute
force is reported on a sample.
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")

from gpu_helpers import REL_DIST, ABS_DIST, build, dev, dist64, leaves, query, recall, votes  # noqa: E402
from paper_1509_06957_amd import mrpt  # noqa: E402

SAMPLE = 40
PINNED_TREES = 2


@pytest.fixture(scope="module")
def gist():
    w = W.GIST_LIKE
    print(f"[case] full size {w.name}", flush=True)
    X, Q = W.data(w), W.queries(w)
    print("[step] data generated", flush=True)
    orc = oracle.build_index(X, PINNED_TREES, w.depth, w.a, w.index_seed)
    print("[step] oracle trees 0-1 built", flush=True)
    g = build(X, w.T, w.depth, w.a, w.index_seed)
    print("[step] gpu index built", flush=True)
    Qd = dev(Q)
    sample = np.sort(np.random.default_rng(1).choice(len(Q), size=SAMPLE, replace=False))
    yield w, X, Q, Qd, orc, g, sample
    g.close()


def test_pinned_trees_bit_exact(gist):
    w, X, Q, Qd, orc, g, sample = gist
    rowptr, col, val = mrpt.mrpt_export_projection(g.handle)
    for r in range(PINNED_TREES * w.depth):
        row = np.zeros(w.d, dtype=np.float32)
        row[col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
        assert np.array_equal(row.view(np.uint32), orc.R[r].view(np.uint32)), f"vector {r}"
    assert np.array_equal(mrpt.mrpt_export_leaf_offsets(g.handle), orc.off)
    for t in range(PINNED_TREES):
        splits, perm = mrpt.mrpt_export_tree(g.handle, t)
        assert np.array_equal(splits.view(np.uint32), orc.splits[t].view(np.uint32)), f"tree {t}"
        assert np.array_equal(perm, orc.perm[t]), f"tree {t}"


def test_pinned_leaves_bit_exact(gist):
    w, X, Q, Qd, orc, g, sample = gist
    assert np.array_equal(leaves(g, Qd)[:, :PINNED_TREES], oracle.route(orc, Q))


def test_candidate_sets_match_leaf_recount(gist):
    w, X, Q, Qd, orc, g, sample = gist
    lv = leaves(g, Qd)
    off = mrpt.mrpt_export_leaf_offsets(g.handle)
    perms = [mrpt.mrpt_export_tree(g.handle, t)[1] for t in range(w.T)]
    ids, cnt = votes(g, dev(Q[sample]), w.v)
    for j, q in enumerate(sample):
        occ = np.concatenate([perms[t][off[lv[q, t]]:off[lv[q, t] + 1]] for t in range(w.T)])
        u, c = np.unique(occ, return_counts=True)
        assert np.array_equal(ids[j], u[c >= w.v]), f"query {q}"
        assert np.array_equal(cnt[j], c[c >= w.v]), f"query {q}"


@pytest.mark.parametrize("k", [10, 100])
def test_batch_query_is_knn_of_s(gist, k):
    w, X, Q, Qd, orc, g, sample = gist
    gi, gd, sc = query(g, Qd, k, w.v)                    # whole batch, one call
    ids, _ = votes(g, dev(Q[sample]), w.v, with_counts=False)
    for j, q in enumerate(sample):
        S = ids[j]
        assert sc[q] == len(S)
        d64 = dist64(X, Q[q], S)
        order = np.lexsort((S, d64))[:k]
        nreal = min(k, len(S))
        real = gi[q][:nreal]
        assert np.all(gi[q][nreal:] == -1)
        assert np.array_equal(real, S[order][:nreal]) or \
            np.allclose(np.sort(dist64(X, Q[q], real)), d64[order][:nreal], rtol=2e-5), f"query {q}"
        dq = dist64(X, Q[q], real)
        assert np.all(np.abs(gd[q][:nreal].astype(np.float64) - dq) <= REL_DIST * dq + ABS_DIST * (dq == 0))
    if k == 10:
        bi, _ = oracle.bruteforce(X, Q[sample], k)
        r = recall(gi[sample], bi)
        print(f"[recall] {w.name} fp32 recall@{k} {r:.4f} |S| mean {sc.mean():.1f}", flush=True)
