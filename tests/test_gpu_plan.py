"""GPU parity of query plans: many batches over several indexes of uneven
size, recorded as one HIP graph and replayed.

  * every batch's results equal mrpt_query_ex's for the same arguments,
    bit for bit (the plan runs the same kernels), at every replay, with eager
    work and synchronisation between the replays;
  * a replay reads the current contents of the query buffers;
  * one branch or several give the same results;
  * the results agree with the oracle under the query path's tolerances.

Workload: the batched workload scaled down to 3 indexes (n in [2k, 20k],
d in {128, 256, 784}, T = 64, leaves of about 32) and 600 queries in batches of
1..150 with k in {1, 10, 100} (k = 100 pads where |S| < 100), v = 3.
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_helpers import check_knn, dev  # noqa: E402
from paper_1509_06957_amd import mrpt  # noqa: E402

SMALL = W.BATCHED.scaled(n_indexes=3, n_lo=2_000, n_hi=20_000, total_queries=600, max_batch=150)


@pytest.fixture(scope="module")
def setup():
    print(f"[case] plan setup {SMALL}", flush=True)
    specs = W.batched_indexes(SMALL)
    X = [W.batched_index_data(sp) for sp in specs]
    ixs = [mrpt.Index(dev(x), SMALL.T, sp.depth, sp.a, sp.index_seed) for sp, x in zip(specs, X)]
    stream = W.batched_stream(SMALL)
    Qh = [W.batched_queries(SMALL, specs[ix], b, m) for b, ix, m, _ in stream]
    Qs = [dev(q) for q in Qh]
    yield specs, X, ixs, stream, Qh, Qs
    for ix in ixs:
        ix.close()


def eager(ixs, stream, Qs, precision):
    out = [ixs[ix].query(Q, k, SMALL.v, precision=precision) for (_, ix, _, k), Q in zip(stream, Qs)]
    torch.cuda.synchronize()
    return [(i.cpu().numpy(), d.cpu().numpy()) for i, d in out]


def same(out, ref, what):
    for j, ((oi, od), (ri, rd)) in enumerate(zip(out, ref)):
        oi, od = oi.cpu().numpy(), od.cpu().numpy()
        assert np.array_equal(oi, ri), f"{what}: batch {j} ids"
        assert np.array_equal(od.view(np.uint32), rd.view(np.uint32)), f"{what}: batch {j} distances"


@pytest.mark.parametrize("precision", [mrpt.MRPT_FP32, mrpt.MRPT_BF16_RERANK, mrpt.MRPT_FP8_RERANK])
@pytest.mark.parametrize("fused,branches", [(1, 1), (0, 1), (0, 5)])
def test_plan_equals_query_calls(setup, precision, fused, branches):
    _, _, ixs, stream, _, Qs = setup
    print(f"[case] plan precision={precision} fused={fused} branches={branches} batches={len(stream)}", flush=True)
    ref = eager(ixs, stream, Qs, precision)
    plan = mrpt.Plan([(ixs[ix], Q, k, SMALL.v) for (_, ix, _, k), Q in zip(stream, Qs)],
                     precision=precision, branches=branches, fused=fused)
    assert plan.device_bytes() > 0
    for rep in range(3):
        out = plan.launch()
        torch.cuda.synchronize()
        same(out, ref, f"replay {rep}")
        for o in out:                       # stale results must not survive a replay
            o[0].fill_(-7)
            o[1].fill_(-7.0)
        ref = eager(ixs, stream, Qs, precision)
    plan.close()


def test_plan_reads_current_queries(setup):
    _, _, ixs, stream, _, Qs = setup
    print("[case] plan replay after the query buffers change", flush=True)
    plan = mrpt.Plan([(ixs[ix], Q, k, SMALL.v) for (_, ix, _, k), Q in zip(stream, Qs)], branches=3)
    plan.launch()
    saved = [Q.clone() for Q in Qs]
    try:
        for Q in Qs:
            Q.copy_(torch.flip(Q, dims=[0]) * 0.5)
        ref = eager(ixs, stream, Qs, mrpt.MRPT_FP32)
        out = plan.launch()
        torch.cuda.synchronize()
        same(out, ref, "changed queries")
    finally:
        for Q, s in zip(Qs, saved):
            Q.copy_(s)
        torch.cuda.synchronize()
        plan.close()


def test_plan_matches_oracle(setup):
    specs, X, ixs, stream, Qh, Qs = setup
    print("[case] plan against the oracle", flush=True)
    plan = mrpt.Plan([(ixs[ix], Q, k, SMALL.v) for (_, ix, _, k), Q in zip(stream, Qs)], branches=4)
    out = plan.launch()
    torch.cuda.synchronize()
    orc = {}
    for (b, ix, m, k), Qb, (gi, gd) in zip(stream, Qh, out):
        sp = specs[ix]
        if ix not in orc:
            orc[ix] = oracle.build_index(X[ix], SMALL.T, sp.depth, sp.a, sp.index_seed)
        ref = oracle.query(orc[ix], Qb, k, SMALL.v, want_sets=True)
        S = [set(s.tolist()) for s in ref["s_ids"]]
        check_knn(X[ix], Qb, gi.cpu().numpy(), gd.cpu().numpy(), ref["idx"], ref["dist"], exact_ids=False, S=S)
    plan.close()


def test_plan_rejects_bad_batch(setup):
    _, _, ixs, stream, _, Qs = setup
    (_, ix, _, k), Q = stream[0], Qs[0]
    with pytest.raises(mrpt.MrptError, match="batch 1"):
        mrpt.Plan([(ixs[ix], Q, k, SMALL.v), (ixs[ix], Q, k, SMALL.T + 1)])
    with pytest.raises(mrpt.MrptError, match="d % 8"):
        bad = W.BATCHED.scaled(n_indexes=1, n_lo=300, n_hi=300, dims=(12,))
        sp = W.batched_indexes(bad)[0]
        tiny = mrpt.Index(dev(W.batched_index_data(sp)), 4, 2, sp.a, 1)
        try:
            q = dev(W.batched_queries(bad, sp, 0, 3))
            mrpt.Plan([(tiny, q, 1, 1)], precision=mrpt.MRPT_BF16_RERANK)
        finally:
            tiny.close()


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("proj_rows,vote_kernel,vote_waves", [(4, 0, 0), (16, 0, 0), (0, 1, 0), (0, 2, 0),
                                                              (0, 0, 16), (0, 1, 8)])
def test_plan_launch_choices_keep_results(setup, proj_rows, vote_kernel, vote_waves, fused):
    # the tunable launch choices (projection vectors per wave, single- or
    # multi-pass voting, the single-pass workgroup's waves, per-stage or
    # per-group launches) change no result
    _, _, ixs, stream, _, Qs = setup
    print(f"[case] plan proj_rows={proj_rows} vote_kernel={vote_kernel} vote_waves={vote_waves} fused={fused}",
          flush=True)
    ref = eager(ixs, stream, Qs, mrpt.MRPT_BF16_RERANK)
    plan = mrpt.Plan([(ixs[ix], Q, k, SMALL.v) for (_, ix, _, k), Q in zip(stream, Qs)],
                     precision=mrpt.MRPT_BF16_RERANK, branches=3, proj_rows=proj_rows, vote_kernel=vote_kernel,
                     fused=fused, vote_waves=vote_waves)
    out = plan.launch()
    torch.cuda.synchronize()
    same(out, ref, f"proj_rows={proj_rows} vote_kernel={vote_kernel} vote_waves={vote_waves} fused={fused}")
    plan.close()


@pytest.mark.parametrize("queue_cap", [None, 1024])
def test_fused_plan_shares_launches_across_indexes(queue_cap, monkeypatch):
    """Several indexes of one d (equal kernel forms) in one per-stage launch:
    the items of the routing, vote and search tables come from different
    indexes, with k = 10 and 100 and v = 2 and 3; trees of 13 and 14 levels
    share the routing launch of the 16-level class.  With the repeat queue
    capped at 1,024 entries (MRPT_VOTE_QUEUE_CAP, read by the plan and the
    query calls alike) the vote launch marks overflowing queries and the
    multi-pass kernel recounts them.  Results equal the query calls', and the
    candidate sets equal the oracle's."""
    if queue_cap:
        monkeypatch.setenv("MRPT_VOTE_QUEUE_CAP", str(queue_cap))
    print(f"[case] fused plan, shared launches, queue cap {queue_cap}", flush=True)
    rng = np.random.default_rng(41)
    d, T = 128, 24
    # (n, depth): leaves of 70..156 ids, and deep trees (13 and 14 levels,
    # leaves of 1..3 ids) whose split walk takes the 16-level kernel class
    shapes = [(3000, 5), (4500, 5), (6000, 6), (2500, 4), (20000, 13), (33000, 14)]
    centers = rng.normal(0, 2, (16, d)).astype(np.float32)
    X = [(centers[rng.integers(0, 16, n)] + rng.normal(0, 1, (n, d))).astype(np.float32) for n, _ in shapes]
    ixs = [mrpt.Index(dev(x), T, depth, 1 / np.sqrt(d), 50 + i) for i, (x, (_, depth)) in enumerate(zip(X, shapes))]
    try:
        jobs = []
        for j in range(12):
            i = j % len(ixs)
            m = int(rng.integers(1, 90))
            Qh = (centers[rng.integers(0, 16, m)] + rng.normal(0, 1, (m, d))).astype(np.float32)
            jobs.append((i, Qh, dev(Qh), 10 if j % 3 else 100, 2 if j % 2 else 3))
        for prec in (mrpt.MRPT_FP32, mrpt.MRPT_BF16_RERANK):
            plan = mrpt.Plan([(ixs[i], Q, k, v) for i, _, Q, k, v in jobs], precision=prec, fused=1)
            out = plan.launch()
            torch.cuda.synchronize()
            ref = [ixs[i].query(Q, k, v, precision=prec) for i, _, Q, k, v in jobs]
            torch.cuda.synchronize()
            same(out, [(a.cpu().numpy(), b.cpu().numpy()) for a, b in ref], f"precision {prec}")
            plan.close()
        orc = [oracle.build_index(x, T, depth, 1 / np.sqrt(d), 50 + i) for i, (x, (_, depth)) in enumerate(zip(X, shapes))]
        plan = mrpt.Plan([(ixs[i], Q, k, v) for i, _, Q, k, v in jobs], fused=1)
        out = plan.launch()
        torch.cuda.synchronize()
        for (i, Qh, _, k, v), (gi, gd) in zip(jobs, out):
            ref = oracle.query(orc[i], Qh, k, v, want_sets=True)
            S = [set(s.tolist()) for s in ref["s_ids"]]
            check_knn(X[i], Qh, gi.cpu().numpy(), gd.cpu().numpy(), ref["idx"], ref["dist"], exact_ids=False, S=S)
        plan.close()
    finally:
        for ix in ixs:
            ix.close()


def test_tuner_times_candidates_and_caches_the_choice(setup, tmp_path):
    from paper_1509_06957_amd import tuning
    _, _, ixs, stream, _, Qs = setup
    print("[case] plan autotuner and its cache", flush=True)
    batches = [(ixs[ix], Q, k, SMALL.v) for (_, ix, _, k), Q in zip(stream, Qs)]
    path = str(tmp_path / "tuning.json")

    def time_plan(plan):
        plan.launch()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(3):
            plan.launch()
        ev[1].record()
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / 3

    grid = {"fused": [1, 0], "branches": [1, 3], "proj_rows": [0], "vote_kernel": [0], "vote_waves": [0, 16]}
    choice, timings, cached = tuning.tune(batches, mrpt.MRPT_FP32, time_plan, grid=grid, path=path)
    assert not cached and len(timings) == 8
    assert set(choice) == {"fused", "branches", "proj_rows", "vote_kernel", "vote_waves"}
    again, t2, cached2 = tuning.tune(batches, mrpt.MRPT_FP32, time_plan, grid=grid, path=path)
    assert cached2 and again == choice and t2 == {}
    ref = eager(ixs, stream, Qs, mrpt.MRPT_FP32)
    plan = mrpt.Plan(batches, precision=mrpt.MRPT_FP32, **choice)
    out = plan.launch()
    torch.cuda.synchronize()
    same(out, ref, f"tuned plan {choice}")
    plan.close()
