"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the oracle under the stated tolerances.

Tolerances (float32 distance path against the float64 oracle):
  * returned distances: |d32 - d64| <= 1e-5 * d64 (1e-6 absolute when d64 = 0);
  * ids: identical where the float32 order is exact (integer-valued data,
    where every partial sum is an integer below 2^24); elsewhere an id may
    differ from the oracle's only inside a near-tie, i.e. the sorted float64
    distances of the returned ids equal the oracle's within 2e-5 relative.
"""
import numpy as np
import torch

from paper_1509_06957_amd import mrpt

REL_DIST = 1e-5
ABS_DIST = 1e-6
REL_TIE = 2e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def build(X, T, depth, a, seed):
    return mrpt.Index(dev(X), T, depth, a, seed)


def query(index, Qd, k, v, **kw):
    s_count = torch.zeros(Qd.shape[0], dtype=torch.int32, device="cuda")
    idx, dist = index.query(Qd, k, v, s_count=s_count, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), s_count.cpu().numpy()


def leaves(index, Qd):
    leaf = torch.empty((Qd.shape[0], index.info.T), dtype=torch.int32, device="cuda")
    mrpt.mrpt_debug_leaves(index.handle, Qd, leaf)
    torch.cuda.synchronize()
    return leaf.cpu().numpy()


def votes(index, Qd, v, with_counts=True):
    cap = mrpt.mrpt_candidate_cap(index.handle, v)
    nq = Qd.shape[0]
    s_count = torch.zeros(nq, dtype=torch.int32, device="cuda")
    s_ids = torch.full((nq, cap), -1, dtype=torch.int32, device="cuda")
    s_votes = torch.zeros((nq, cap), dtype=torch.uint8, device="cuda") if with_counts else None
    mrpt.mrpt_debug_votes(index.handle, Qd, v, s_count, s_ids, s_votes, cap)
    torch.cuda.synchronize()
    cnt = s_count.cpu().numpy()
    ids = s_ids.cpu().numpy()
    sv = s_votes.cpu().numpy() if with_counts else None
    out_ids, out_votes = [], []
    for q in range(nq):
        row = ids[q, :cnt[q]]
        order = np.argsort(row, kind="stable")
        out_ids.append(row[order])
        out_votes.append(sv[q, :cnt[q]][order].astype(np.int32) if with_counts else None)
    return out_ids, out_votes


def dist64(X, q, ids):
    diff = X[ids].astype(np.float64) - q.astype(np.float64)[None, :]
    return np.sqrt((diff * diff).sum(axis=1))


def check_knn(X, Q, gi, gd, oi, od, exact_ids, queries=None, S=None):
    """Compare GPU (gi, gd) with oracle (oi, od: float64) for the listed queries."""
    qs = range(len(Q)) if queries is None else queries
    for j, q in enumerate(qs):
        g_ids, g_d = gi[j], gd[j]
        o_ids, o_d = oi[j], od[j]
        nreal = int((o_ids >= 0).sum())
        assert int((g_ids >= 0).sum()) == nreal, f"query {q}: {int((g_ids >= 0).sum())} results vs {nreal}"
        assert np.all(g_ids[nreal:] == -1) and np.all(np.isinf(g_d[nreal:])), f"query {q}: padding"
        real = g_ids[:nreal]
        assert len(set(real.tolist())) == nreal, f"query {q}: duplicate ids"
        if S is not None:
            assert set(real.tolist()) <= S[j], f"query {q}: id outside S"
        if exact_ids:
            assert np.array_equal(real, o_ids[:nreal]), f"query {q}: ids {real} vs {o_ids[:nreal]}"
        d64 = dist64(X, Q[q], real)
        tol = REL_DIST * d64 + ABS_DIST * (d64 == 0)
        assert np.all(np.abs(g_d[:nreal].astype(np.float64) - d64) <= tol), f"query {q}: distance error"
        ref = o_d[:nreal]
        assert np.all(np.abs(np.sort(d64) - ref) <= REL_TIE * ref + ABS_DIST), f"query {q}: not the k nearest of S"
        if not exact_ids:
            # where the two orders agree up to near-ties, the ids coincide
            for r in range(nreal):
                if real[r] != o_ids[r]:
                    assert abs(d64[r] - ref[r]) <= REL_TIE * ref[r] + ABS_DIST, f"query {q}: rank {r}"


def recall(ids, true_ids):
    k = true_ids.shape[1]
    return float(np.mean([len(set(a.tolist()) & set(b.tolist())) / k for a, b in zip(ids, true_ids)]))
