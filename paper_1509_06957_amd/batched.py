"""Throughput of the batched workload: many indexes of uneven size and a
stream of mixed query batches, searched by one query plan (one HIP graph
launch per step).

For every index of the workload the index is built on the GPU, the query
batches are uploaded, and plans are recorded for a grid of launch choices:
the branch count (the graph's independent chains), the projection's vectors
per wave and the vote kernel.  A small autotuner times each candidate plan
and keeps the fastest (every choice gives the same results).  It reports:
  * plan_qps: queries/s of the tuned plan (all batches, one launch per step);
  * eager_qps: the same batches as one mrpt_query_ex call each, on one stream;
  * recall@k on a sample of queries against exact k-NN from the library's
    exact mode (one tree of depth 0, v = 1: S is every point).
One JSON line on stdout.

Usage: python -m paper_1509_06957_amd.batched [--quick] [--steps K] [--precision fp32|bf16]
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print("[batched]", *a, file=sys.stderr, flush=True)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--quick", action="store_true", help="3 small indexes, 2,000 queries")
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--precision", default="bf16", choices=("fp32", "bf16"))
    p.add_argument("--fused", default="1,0", help="plan forms to try (1: per-stage launches across indexes)")
    p.add_argument("--branches", default="1,2,4,8,16")
    p.add_argument("--proj-rows", default="0,16", help="projection vectors per wave to try (0: automatic)")
    p.add_argument("--vote-kernels", default="0,2", help="vote kernels to try (0 automatic, 1 single-pass, 2 multi-pass)")
    p.add_argument("--vote-waves", default="0,16", help="single-pass vote workgroups to try (0 automatic, 8, 16 waves)")
    p.add_argument("--recall-sample", type=int, default=2000)
    p.add_argument("--retune", action="store_true", help="time every candidate even if the cache holds a choice")
    args = p.parse_args()

    import torch
    from paper_1509_06957_amd import mrpt
    from paper_1509_06957_amd import workloads as W

    bw = W.BATCHED
    if args.quick:
        bw = bw.scaled(n_indexes=3, n_lo=5_000, n_hi=50_000, total_queries=2_000)
    prec = mrpt.MRPT_BF16_RERANK if args.precision == "bf16" else mrpt.MRPT_FP32
    specs = W.batched_indexes(bw)
    stream = W.batched_stream(bw)

    ixs, build_s = [], 0.0
    for sp in specs:
        X = torch.from_numpy(W.batched_index_data(sp)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ixs.append(mrpt.Index(X, bw.T, sp.depth, sp.a, sp.index_seed))
        build_s += time.perf_counter() - t0
        del X
    log(f"{len(specs)} indexes built on the GPU in {build_s:.2f} s")
    Qs = [torch.from_numpy(W.batched_queries(bw, specs[ix], b, m)).cuda() for b, ix, m, _ in stream]
    batches = [(ixs[ix], Q, k, bw.v) for (_, ix, _, k), Q in zip(stream, Qs)]
    nq = sum(m for _, _, m, _ in stream)
    log(f"{len(stream)} batches, {nq} queries")

    def time_launches(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    # autotuner over the recorded graph's launch choices (tuning.py): plan
    # form, streams or chains, projection rows per wave, vote kernel and its
    # workgroup size; the choice is cached as JSON under the batches' signature
    from paper_1509_06957_amd import tuning
    grid = {"fused": [int(x) for x in args.fused.split(",")],
            "branches": [int(x) for x in args.branches.split(",")],
            "proj_rows": [int(x) for x in args.proj_rows.split(",")],
            "vote_kernel": [int(x) for x in args.vote_kernels.split(",")],
            "vote_waves": [int(x) for x in args.vote_waves.split(",")]}
    choice, tuning_ms, cached = tuning.tune(batches, prec, lambda pl: time_launches(pl.launch, max(2, args.steps // 2)),
                                            grid=grid, retune=args.retune, log=log)
    b_best = ",".join(f"{k}={v}" for k, v in choice.items())
    plan = mrpt.Plan(batches, precision=prec, **choice)
    plan_ms = time_launches(plan.launch, args.steps)
    out = plan.launch()
    torch.cuda.synchronize()

    def eager():
        for (ix, Q, k, v), o in zip(batches, out_eager):
            ix.query(Q, k, v, precision=prec, out=o)

    out_eager = [(torch.empty_like(a), torch.empty_like(d)) for a, d in out]
    eager_ms = time_launches(eager, args.steps)
    identical = all(torch.equal(a, c) and torch.equal(d, e) for (a, d), (c, e) in zip(out, out_eager))

    # recall on a sample: whole batches in stream order up to the sample size
    hit = tot = taken = 0
    exact = {}
    for (b, ix, m, k), Q, (gi, _) in zip(stream, Qs, out):
        if taken >= args.recall_sample:
            break
        if ix not in exact:
            X = torch.from_numpy(W.batched_index_data(specs[ix])).cuda()
            exact[ix] = mrpt.Index(X, 1, 0, 1.0, 0)
            del X
        ti, _ = exact[ix].query(Q, k, 1)
        torch.cuda.synchronize()
        g, t = gi.cpu().numpy(), ti.cpu().numpy()
        hit += sum(len(set(a[a >= 0].tolist()) & set(c.tolist())) for a, c in zip(g, t))
        tot += g.shape[0] * k
        taken += m
    for e in exact.values():
        e.close()

    res = {
        "workload": bw.name if not args.quick else "batched (quick: 3 indexes, 2k queries)",
        "indexes": [{"n": sp.n, "d": sp.d, "depth": sp.depth} for sp in specs],
        "batches": len(stream), "queries": nq, "T": bw.T, "v": bw.v,
        "precision": "bf16+rerank" if prec == mrpt.MRPT_BF16_RERANK else "fp32",
        "plan_qps": round(nq / (plan_ms / 1e3), 1), "plan_ms_per_step": round(plan_ms, 4),
        "chosen": b_best, "tuning_ms": tuning_ms, "tuning_from_cache": cached,
        "tuning_cache": tuning.cache_path(),
        "eager_qps": round(nq / (eager_ms / 1e3), 1), "eager_ms_per_step": round(eager_ms, 4),
        "plan_equals_eager": bool(identical),
        "recall_at_k": round(hit / max(tot, 1), 4), "recall_sample_queries": taken,
        "build_s": round(build_s, 3), "plan_device_bytes": plan.device_bytes(),
    }
    print(json.dumps(res), flush=True)
    plan.close()
    for ix in ixs:
        ix.close()


if __name__ == "__main__":
    main()
