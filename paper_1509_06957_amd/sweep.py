"""Recall / throughput sweeps of the query path, in the shape of the paper's
experiments (Sec. IV: a grid over the number of trees T, the depth and the
vote threshold v; Table III: the time to reach at least recall R).

For every (T, depth, v) of a grid the index is built on the GPU, the whole
query batch is timed (float32 arm, and the bfloat16 and fp8 prefilter arms
where the dimension allows them), and recall@k is measured on a sample against exact k-NN: the
stored float64 brute-force answers of that sample (--truth, written by
tests/golden/make_recall_truth.py), else the library's exact mode (one tree
of depth 0 and v = 1, so the candidate set is every point; float32
distances), which the output then names.  One JSON line per configuration is printed, then a
summary: for each recall target the fastest configuration reaching it, for
MRPT (all v), MRPT with v = 1 (voting disabled, the paper's second column)
and dense random projection trees (a = 1, v = 1, the third column; on a
smaller grid, since dense vectors are projected on the host).  Last, an
ablation at the workload's (T, depth): Bernoulli(a) projection entries
against exactly ceil(a d) nonzeros per vector, for every v.

Usage: python -m paper_1509_06957_amd.sweep [--workload sift_like] [--quick]
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print("[sweep]", *a, file=sys.stderr, flush=True)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workload", default="sift_like")
    p.add_argument("--k", type=int, default=None)
    p.add_argument("--reps", type=int, default=3)
    p.add_argument("--recall-sample", type=int, default=500)
    p.add_argument("--quick", action="store_true", help="a small grid (smoke run)")
    p.add_argument("--truth", default=None, help="npz of the sample's exact k-NN (sample, idx)")
    args = p.parse_args()

    import torch
    from paper_1509_06957_amd import mrpt
    from paper_1509_06957_amd import workloads as W

    w = W.ALL[args.workload]
    k = args.k or w.k
    X, Q = W.data(w), W.queries(w)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    nq = len(Q)
    if args.truth:
        tf = np.load(args.truth)
        rs, truth = tf["sample"], tf["idx"]
        if truth.shape[1] != k:
            raise SystemExit(f"{args.truth} holds k = {truth.shape[1]}, the sweep uses k = {k}")
        truth_kind = "stored float64 brute force"
    else:
        rs = np.random.default_rng(0).choice(nq, size=min(args.recall_sample, nq), replace=False)
        exact = mrpt.Index(Xd, 1, 0, 1.0, 0)
        truth, _ = exact.query(Qd[torch.from_numpy(rs).cuda()], k, 1)
        truth = truth.cpu().numpy()
        exact.close()
        truth_kind = "library exact mode (float32)"
    log(f"{w.name}: exact k-NN of {len(rs)} sample queries ready ({truth_kind})")

    if args.quick:
        Ts, depths, vs = (10, 50), (w.depth - 1, w.depth), (1, 2, 3)
    else:
        Ts = (10, 25, 50, 100, 200)
        depths = tuple(dd for dd in range(w.depth - 3, w.depth + 2) if (1 << dd) <= w.n)
        vs = (1, 2, 3, 4, 5, 6, 8)
    bf16_ok = w.d % 8 == 0 and w.d <= 1024
    fp8_ok = w.d % 16 == 0 and w.d <= 1024

    def timed(ix, v, precision):
        out = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
               torch.empty((nq, k), dtype=torch.float32, device="cuda"))
        ix.query(Qd, k, v, precision=precision, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            ix.query(Qd, k, v, precision=precision, out=out)
        torch.cuda.synchronize()
        return nq * args.reps / (time.perf_counter() - t0), out[0]

    def recall_of(ids):
        got = ids.cpu().numpy()[rs]
        return float(np.mean([len(set(a.tolist()) & set(b.tolist())) / k for a, b in zip(got, truth)]))

    rows = []
    for a_mode in ("sparse", "dense"):
        a = w.a if a_mode == "sparse" else 1.0
        # dense vectors (d nonzeros) are projected by the host build and the
        # fused routing kernel: a smaller grid keeps the ablation quick
        Tg = Ts if a_mode == "sparse" else tuple(t for t in Ts if t <= 50)
        dg = depths if a_mode == "sparse" else depths[-3:-1]
        for T in Tg:
            for depth in dg:
                t0 = time.perf_counter()
                ix = mrpt.Index(Xd, T, depth, a, w.index_seed)
                build_s = time.perf_counter() - t0
                for v in vs:
                    if v > T or (a_mode == "dense" and v != 1):
                        continue
                    s_count = torch.zeros(nq, dtype=torch.int32, device="cuda")
                    ix.query(Qd, k, v, s_count=s_count)
                    qps32, ids = timed(ix, v, mrpt.MRPT_FP32)
                    qps16, ids16 = timed(ix, v, mrpt.MRPT_BF16_RERANK) if bf16_ok else (None, None)
                    qps8, ids8 = timed(ix, v, mrpt.MRPT_FP8_RERANK) if fp8_ok else (None, None)
                    row = {"a": a_mode, "T": T, "depth": depth, "v": v, "recall": round(recall_of(ids), 4),
                           "qps_fp32": round(qps32, 1), "qps_bf16": None if qps16 is None else round(qps16, 1),
                           "qps_fp8": None if qps8 is None else round(qps8, 1),
                           "recall_bf16": None if ids16 is None else round(recall_of(ids16), 4),
                           "recall_fp8": None if ids8 is None else round(recall_of(ids8), 4),
                           "s_mean": round(float(s_count.float().mean()), 1), "build_s": round(build_s, 3)}
                    rows.append(row)
                    print(json.dumps(row), flush=True)
                ix.close()

    # ablation of the projection vectors: Bernoulli(a) entries against exactly
    # ceil(a d) nonzeros per vector (footnote of Sec. II-D), at the workload's
    # own (T, depth), every v
    ablation = []
    for exact in (False, True):
        ix = mrpt.Index(Xd, w.T, w.depth, w.a, w.index_seed, exact_nnz=exact)
        for v in vs:
            if v > w.T:
                continue
            s_count = torch.zeros(nq, dtype=torch.int32, device="cuda")
            ix.query(Qd, k, v, s_count=s_count)
            qps32, ids = timed(ix, v, mrpt.MRPT_FP32)
            row = {"exact_nnz": exact, "T": w.T, "depth": w.depth, "v": v, "recall": round(recall_of(ids), 4),
                   "qps_fp32": round(qps32, 1), "s_mean": round(float(s_count.float().mean()), 1)}
            ablation.append(row)
            print(json.dumps(row), flush=True)
        ix.close()

    targets = (0.8, 0.9, 0.95, 0.99)

    def best(sel, key, rkey="recall"):
        out = {}
        for r in targets:
            ok = [x for x in rows if sel(x) and x[key] is not None and x[rkey] >= r]
            if ok:
                b = max(ok, key=lambda x: x[key])
                out[str(r)] = {"qps": b[key], "T": b["T"], "depth": b["depth"], "v": b["v"], "recall": b[rkey]}
            else:
                out[str(r)] = None
        return out

    summary = {
        "workload": w.name, "k": k, "queries": nq, "recall_sample": len(rs), "recall_truth": truth_kind,
        "mrpt_fp32": best(lambda x: x["a"] == "sparse", "qps_fp32"),
        "mrpt_bf16": best(lambda x: x["a"] == "sparse", "qps_bf16", "recall_bf16"),
        "mrpt_fp8": best(lambda x: x["a"] == "sparse", "qps_fp8", "recall_fp8"),
        "mrpt_v1_fp32": best(lambda x: x["a"] == "sparse" and x["v"] == 1, "qps_fp32"),
        "rp_trees_dense_fp32": best(lambda x: x["a"] == "dense", "qps_fp32"),
        "exact_nnz_ablation": [{"v": b["v"], "recall": b["recall"], "recall_exact": e["recall"],
                                "qps": b["qps_fp32"], "qps_exact": e["qps_fp32"]}
                               for b in ablation if not b["exact_nnz"]
                               for e in ablation if e["exact_nnz"] and e["v"] == b["v"]],
    }
    print(json.dumps({"summary": summary}), flush=True)


if __name__ == "__main__":
    main()
