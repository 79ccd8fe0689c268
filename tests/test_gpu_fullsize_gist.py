"""Full-size checks on the gist-like workload (n = 1,000,000, d = 960, 10,000
queries, T = 200, depth = 10, v = 5, k = 10 and 100) in the launch
configuration of a whole-batch query call.

The oracle's full index takes minutes of host time at this size, so its
values are stored: tests/golden/make_gist_like_golden.py (oracle and
workload generators only) writes the SHA-256 of every tree's splits and perm
and of the projection vectors, every query's |S|, the oracle's k = 10 answer
for all 10,000 queries and its k = 100 answer for the first 500.  The GPU
index must match every digest bit for bit, |S| must match for every query,
and the answers must be the oracle's up to float32 near-ties.  Trees 0 and 1
are also rebuilt by the oracle here, and every query's leaf in them compared.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")

from gpu_helpers import (ARM, build, check_answers, check_kept, check_knn, dev, gpu_keep, leaves, query,  # noqa: E402
                         recall, votes)
from paper_1509_06957_amd import mrpt  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SAMPLE = 40
PINNED_TREES = 2


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


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
    with open(os.path.join(GOLDEN, "gist_like_trees.json")) as f:
        trees = json.load(f)
    knn = dict(np.load(os.path.join(GOLDEN, "gist_like_knn.npz")))
    sample = np.sort(np.random.default_rng(1).choice(len(Q), size=SAMPLE, replace=False))
    yield w, X, Q, Qd, orc, g, trees, knn, sample
    g.close()


def test_index_matches_golden_digests(gist):
    w, X, Q, Qd, orc, g, trees, knn, sample = gist
    rowptr, col, val = mrpt.mrpt_export_projection(g.handle)
    R = np.zeros((w.T * w.depth, w.d), dtype=np.float32)
    for r in range(R.shape[0]):
        R[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
    assert sha(R.view(np.uint32)) == trees["projection_sha256"]
    assert mrpt.mrpt_export_leaf_offsets(g.handle).tolist() == trees["leaf_offsets"]
    for t in range(w.T):
        splits, perm = mrpt.mrpt_export_tree(g.handle, t)
        assert sha(splits.view(np.uint32)) == trees["splits_sha256"][t], f"tree {t} splits"
        assert sha(perm) == trees["perm_sha256"][t], f"tree {t} perm"


def test_pinned_trees_and_leaves_bit_exact(gist):
    w, X, Q, Qd, orc, g, trees, knn, sample = gist
    for t in range(PINNED_TREES):
        splits, perm = mrpt.mrpt_export_tree(g.handle, t)
        assert np.array_equal(splits.view(np.uint32), orc.splits[t].view(np.uint32)), f"tree {t}"
        assert np.array_equal(perm, orc.perm[t]), f"tree {t} perm"
        assert sha(perm) == trees["perm_sha256"][t]
    assert np.array_equal(leaves(g, Qd)[:, :PINNED_TREES], oracle.route(orc, Q))


@pytest.mark.parametrize("k", [10, 100])
def test_batch_query_matches_golden(gist, k):
    w, X, Q, Qd, orc, g, trees, knn, sample = gist
    gi, gd, sc = query(g, Qd, k, w.v)                    # whole batch, one call
    assert np.array_equal(sc, knn["s_count"])
    m = len(Q) if k == 10 else knn["idx100"].shape[0]
    check_knn(X, Q[:m], gi[:m], gd[:m], knn[f"idx{k}"], knn[f"dist{k}"], exact_ids=False)
    if k == 10:
        bi, _ = oracle.bruteforce(X, Q[sample], k, nthreads=oracle.all_threads())
        r = recall(gi[sample], bi)
        print(f"[recall] {w.name} fp32 recall@{k} {r:.4f} (oracle brute force, {len(sample)} queries) "
              f"|S| mean {sc.mean():.1f}", flush=True)


def test_candidate_sets_match_leaf_recount(gist):
    # the counter's candidate sets and the debug recount's F against a recount
    # of the leaf lists (leaves and trees pinned above)
    w, X, Q, Qd, orc, g, trees, knn, sample = gist
    lv = leaves(g, Qd)
    off = mrpt.mrpt_export_leaf_offsets(g.handle)
    perms = [mrpt.mrpt_export_tree(g.handle, t)[1] for t in range(w.T)]
    ids, cnt = votes(g, dev(Q[sample]), w.v)
    for j, q in enumerate(sample):
        occ = np.concatenate([perms[t][off[lv[q, t]]:off[lv[q, t] + 1]] for t in range(w.T)])
        u, c = np.unique(occ, return_counts=True)
        assert np.array_equal(ids[j], u[c >= w.v]), f"query {q}"
        assert np.array_equal(cnt[j], c[c >= w.v]), f"query {q}"


@pytest.mark.parametrize("precision", [mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
def test_precision_arm_matches_golden(gist, precision):
    # the oracle's model of the arm for the first 200 queries (stored): kept
    # lists within the float32 score bound, answers the k nearest of the kept
    w, X, Q, Qd, orc, g, trees, knn, sample = gist
    name = "bf16" if precision == mrpt.MRPT_BF16_RERANK else "fp8"
    k, kp = 10, 40
    m = knn[f"{name}_keep_ids"].shape[0]
    qs = np.arange(m)
    ref = {"s_count": knn["s_count"][:m], "keep_ids": knn[f"{name}_keep_ids"],
           "keep_score": knn[f"{name}_keep_score"], "idx": knn[f"{name}_idx"]}
    g_sc, g_keep = gpu_keep(g, Qd, k, w.v, precision)
    gi, gd, _ = query(g, Qd, k, w.v, precision=precision)
    banded = check_kept(X, Q, ref, g_sc[:m], g_keep[:m], kp, ARM[precision], queries=qs)
    check_answers(X, Q, ref, g_keep[:m], gi[:m], gd[:m], kp, queries=qs)
    print(f"[arm] gist-like {name}: {banded} of {m} queries with a candidate in the float32 band at the cut",
          flush=True)
