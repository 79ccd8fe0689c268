"""Throughput of the MRPT voting-search query path on one MI355X.

One step = one query call over the whole batch of the sift-like workload
(n = 1,000,000 points, d = 128, 10,000 queries, T = 100 trees, depth 12,
k = 10, v = 3): routing, voting and exact search in S, all in the library's
HIP kernels, inputs resident in HBM.  Two arms on the same index: float32
exact search (the headline value) and bfloat16 prefilter + float32 rerank +
float64 recheck.  Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "queries/sec at recall@10=0.9 (1M×128, k=10); FP32 plain vs BF16+rerank"
CSRC = os.path.join(ROOT, "paper_1509_06957_amd", "csrc")
# source file of each kernel family (the traffic summaries record a hash of
# it with device_common.h; a summary of older source is not used)
KERNEL_FILE = {"project_route_kernel": "kernels_route.hip",
               "vote_map_kernel": "kernels_vote.hip", "vote_dir_kernel": "kernels_vote.hip",
               "dist_fp32_kernel": "kernels_search.hip", "dist_prefilter_kernel": "kernels_search.hip",
               "dist_prefilter_w7_kernel": "kernels_search.hip", "dist_prefilter_w6_kernel": "kernels_search.hip"}
# the kernel that dominates each stage on this workload (rocprofv3 names)
STAGE_KERNEL = {"route": "project_route_kernel", "vote": "vote_map_kernel", "search": "dist_fp32_kernel"}
COPY_BYTES = 1 << 30
STAGES = ("route", "vote", "search")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="sift_like")
    p.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    p.add_argument("--recall-sample", type=int, default=500)
    p.add_argument("--latency-reps", type=int, default=50, help="timed calls per batch size (0: none)")
    p.add_argument("--cpu-sample", type=int, default=10000)
    p.add_argument("--no-host-build", action="store_true", help="skip timing the host build of the index")
    return p.parse_args()


def hbm_copy_gbps(torch, nbytes=COPY_BYTES, reps=5):
    """Bandwidth of a plain device-to-device copy of nbytes (read + write
    bytes / time): the achievable-bandwidth reference beside the 8 TB/s peak,
    and the calibration kernel of the committed HBM traffic counts."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for name in (KERNEL_FILE[kernel.split("<")[0]], "device_common.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload_key):
    """Memory-side bytes per launch of `kernel` (a rocprofv3 name prefix) from
    the committed counter summary of this workload, if it was taken on the
    current source; else None.  Returns (read + write bytes, row of the
    summary as a dict)."""
    path = os.path.join(ROOT, "profiles", f"query_kernels_{workload_key}_traffic.txt")
    if not os.path.exists(path):
        return None, None
    cols = None
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = re.split(r"\s{2,}", line.strip())
            if parts[0] == "kernel":
                cols = parts
                continue
            if cols and parts[0].startswith(kernel) and len(parts) == len(cols):
                row = dict(zip(cols, parts))
                if row.get("src_sha256_16") != kernel_source_hash(kernel):
                    return None, None
                return (float(row["read_MB"]) + float(row["write_MB"])) * 1e6, row
    return None, None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the query path is "
              "query-parallel and would shard by splitting the batch across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1509_06957_amd import mrpt
    from paper_1509_06957_amd import workloads as W

    w = W.ALL[args.workload]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    X = W.data(w)
    Q = W.queries(w)
    log(f"workload {w.name}: generated in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    # index build (outside the timed query region): GPU build, then the host
    # build of the same index for comparison (bit-identical trees)
    build = {}
    for name, on_dev in (("device", True), ("host", False))[:1 if args.no_host_build else 2]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ix = mrpt.Index(Xd, w.T, w.depth, w.a, w.index_seed, on_device=on_dev)
        build[name] = time.perf_counter() - t0
        if not on_dev:
            ix.close()
    ix = mrpt.Index(Xd, w.T, w.depth, w.a, w.index_seed, on_device=True)
    build_s = build["device"]
    log(f"index built in {build['device']:.3f}s on the GPU" +
        (f", {build['host']:.2f}s on host threads" if "host" in build else ""))
    nq, k, v = w.nq, w.k, w.v

    # |S| per query and the leaf sizes visited (for the algorithmic bytes)
    s_count = torch.zeros(nq, dtype=torch.int32, device="cuda")
    ix.query(Qd, k, v, s_count=s_count)
    leaf = torch.empty((nq, w.T), dtype=torch.int32, device="cuda")
    mrpt.mrpt_debug_leaves(ix.handle, Qd, leaf)
    torch.cuda.synchronize()
    S = s_count.cpu().numpy().astype(np.int64)
    off = mrpt.mrpt_export_leaf_offsets(ix.handle)
    sizes = np.diff(off)
    leaf_entries = int(sizes[leaf.cpu().numpy()].sum())
    sum_s = int(S.sum())
    log(f"|S| mean {S.mean():.1f} p50 {np.percentile(S, 50):.0f} p99 {np.percentile(S, 99):.0f}")

    nnz = int(ix.info.nnz)
    nsplit = (1 << w.depth) - 1
    bytes_route = nq * w.d * 4 + nq * w.T * 4 + (w.T * w.depth + 1) * 4 + nnz * 8 + w.T * nsplit * 4
    bytes_vote = nq * w.T * 4 + nq * w.T * 8 + leaf_entries * 4 + sum_s * 4 + nq * 4
    kp = 4 * k
    rerank_rows = int(np.minimum(S, kp).sum())
    bytes_search = {
        "fp32": nq * 4 + sum_s * 4 + sum_s * w.d * 4 + nq * w.d * 4 + nq * k * 8,
        "bf16": nq * 4 + sum_s * 4 + sum_s * (w.d * 2) + rerank_rows * w.d * 4 + nq * w.d * 4 + nq * k * 8,
        "fp8": nq * 4 + sum_s * 4 + sum_s * (w.d + 8) + rerank_rows * w.d * 4 + nq * w.d * 4 + nq * k * 8,
    }

    def run_arm(precision, steps, warmup):
        """The timed steps run as the product runs them (no events between
        stages); the per-stage durations come from as many further steps
        with HIP events recorded at the stage boundaries on the query's
        stream (events serialise the stages, so they stay out of the
        timed region)."""
        out = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
               torch.empty((nq, k), dtype=torch.float32, device="cuda"))
        opts = mrpt.mrpt_default_opts()
        opts.precision = precision
        for _ in range(warmup):
            mrpt.mrpt_query_ex(ix.handle, Qd, k, v, out[0], out[1], opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            mrpt.mrpt_query_ex(ix.handle, Qd, k, v, out[0], out[1], opts)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        events = []
        arrays = []
        for _ in range(steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            for e in ev:
                e.record()                       # creates the HIP event
            arr = (ctypes_void_array(4))(*[e.cuda_event for e in ev])
            events.append(ev)
            arrays.append(arr)
        torch.cuda.synchronize()
        for i in range(steps):
            opts.stage_events = ctypes_cast_events(arrays[i])
            mrpt.mrpt_query_ex(ix.handle, Qd, k, v, out[0], out[1], opts)
        torch.cuda.synchronize()
        stage_ms = np.array([[ev[j].elapsed_time(ev[j + 1]) for j in range(3)] for ev in events])
        return elapsed, stage_ms.mean(axis=0), out

    log(f"timing {args.steps} steps after {args.warmup} warmup (fp32)")
    el32, st32, out32 = run_arm(mrpt.MRPT_FP32, args.steps, args.warmup)
    log(f"fp32: {el32 / args.steps * 1e3:.3f} ms/step, stages(ms) {np.round(st32, 4).tolist()}")
    el16, st16, out16 = run_arm(mrpt.MRPT_BF16_RERANK, args.steps, args.warmup)
    log(f"bf16+rerank: {el16 / args.steps * 1e3:.3f} ms/step, stages(ms) {np.round(st16, 4).tolist()}")
    el8, st8, out8 = run_arm(mrpt.MRPT_FP8_RERANK, args.steps, args.warmup)
    log(f"fp8+rerank: {el8 / args.steps * 1e3:.3f} ms/step, stages(ms) {np.round(st8, 4).tolist()}")
    gi8, gd8 = out8[0].cpu().numpy(), out8[1].cpu().numpy()
    gi32, gd32 = out32[0].cpu().numpy(), out32[1].cpu().numpy()
    gi16, gd16 = out16[0].cpu().numpy(), out16[1].cpu().numpy()

    # recall sample (ground truth: the oracle's float64 brute force, taken in
    # the CPU-baseline leg below; without that leg, the library's exact mode)
    rs = np.random.default_rng(0).choice(nq, size=min(args.recall_sample, nq), replace=False)

    def arm_record(elapsed, stage_ms, arm):
        qps = nq * args.steps / elapsed
        by = {"route": bytes_route, "vote": bytes_vote, "search": bytes_search[arm]}
        stages = {}
        for j, name in enumerate(STAGES):
            gbs = by[name] / (stage_ms[j] * 1e-3) / 1e9
            stages[name] = {"ms": round(float(stage_ms[j]), 5), "bytes": int(by[name]),
                            "GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        total_bytes = sum(by.values())
        return qps, stages, total_bytes

    qps32, stages32, tb32 = arm_record(el32, st32, "fp32")
    qps16, stages16, tb16 = arm_record(el16, st16, "bf16")
    qps8, stages8, tb8 = arm_record(el8, st8, "fp8")
    dom = max(STAGES, key=lambda s: stages32[s]["ms"])
    copy_gbps = hbm_copy_gbps(torch)
    log(f"plain device copy: {copy_gbps:.0f} GB/s")

    def roofline_of(stage, kernel):
        """The stage's dominant kernel against 8 TB/s: algorithmic bytes per
        launch over the launch's duration (HIP events on the query stream);
        traffic = memory-side bytes per launch from the committed counter
        summary (requests leaving L2, Infinity-Cache hits included), or None
        when that summary predates the kernel's source."""
        traffic, row = read_traffic(kernel, args.workload)
        return {
            "bound": "hbm", "kernel": kernel,
            "achieved": stage["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(stage["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_over_algorithmic": round(traffic / stage["bytes"], 4) if traffic else None,
            "bytes_per_launch": stage["bytes"], "launch_ms": stage["ms"],
            "profiled_launch_us": float(row["avg_us"]) if row else None,
            "copy_GBps": round(copy_gbps, 1),
            "basis": "frac = algorithmic bytes / launch time / 8 TB/s; traffic = bytes leaving L2 "
                     "(TCC_EA0 read/write requests by size), which include Infinity-Cache hits: no "
                     "counter on this part separates those from DRAM reads",
        }

    roofline = roofline_of(stages32[dom], STAGE_KERNEL[dom])
    bf16_kernel = "dist_prefilter_w7_kernel" if w.d <= 128 else "dist_prefilter_kernel<0"
    roofline16 = roofline_of(stages16["search"], bf16_kernel)
    roofline8 = roofline_of(stages8["search"], "dist_prefilter_w6_kernel<1" if w.d <= 128 else "dist_prefilter_kernel<1")
    roofline_vote = roofline_of(stages32["vote"], "vote_map_kernel" if w.d <= 128 else "vote_dir_kernel")

    # latency of one query call (fp32 arm, all five steps) per batch size:
    # host clock around the call and a synchronisation, inputs resident
    latency = {}
    for b in (1, 16, 256, 4096):
        if b > nq or args.latency_reps <= 0:
            continue
        ob = (torch.empty((b, k), dtype=torch.int32, device="cuda"),
              torch.empty((b, k), dtype=torch.float32, device="cuda"))
        Qb = Qd[:b].contiguous()
        ts = []
        for r in range(args.latency_reps + 5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mrpt.mrpt_query(ix.handle, Qb, k, v, ob[0], ob[1])
            torch.cuda.synchronize()
            if r >= 5:
                ts.append((time.perf_counter() - t0) * 1e3)
        latency[str(b)] = {"p50_ms": round(float(np.percentile(ts, 50)), 4),
                           "p99_ms": round(float(np.percentile(ts, 99)), 4), "reps": len(ts)}
    log(f"latency (ms, p50/p99): " + ", ".join(f"{b}: {x['p50_ms']}/{x['p99_ms']}" for b, x in latency.items()))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle   # the CPU baseline: the oracle timed on this host
        nth = oracle.all_threads()
        t0 = time.perf_counter()
        orc = oracle.build_index(X, w.T, w.depth, w.a, w.index_seed, nthreads=nth)
        log(f"oracle index built in {time.perf_counter() - t0:.1f}s on {nth} threads")
        m = min(args.cpu_sample, nq)
        reps, el = 0, 0.0
        while reps == 0 or (el < 10.0 and reps < 100):      # about 10 s of host work
            t0 = time.perf_counter()
            oracle.query(orc, Q[:m], k, v, nthreads=nth)
            el += time.perf_counter() - t0
            reps += 1
        cpu = {"value": round(m * reps / el, 1), "unit": "queries/s", "cores": nth, "kind": "oracle",
               "sample": f"first {m} of the {nq} queries x {reps} passes, oracle index of the same "
                         f"seed, {el:.2f}s wall on {nth} host threads"}
        log(f"oracle: {m * reps / el:.1f} queries/s ({reps} passes)")
        # the same oracle on one host thread, over a prefix sized to about 3 s
        m1 = max(1, min(nq, int(3.0 * m * reps / el / nth)))
        t0 = time.perf_counter()
        oracle.query(orc, Q[:m1], k, v, nthreads=1)
        el1 = time.perf_counter() - t0
        cpu["one_core"] = {"value": round(m1 / el1, 1), "unit": "queries/s", "cores": 1,
                           "sample": f"first {m1} queries, one pass, {el1:.2f}s wall on 1 host thread"}
        log(f"oracle on one thread: {m1 / el1:.1f} queries/s")
        # the oracle's float64 brute force over the recall sample: the ground
        # truth of the recall figures, and the CPU's exact-search rate
        t0 = time.perf_counter()
        bi, _ = oracle.bruteforce(X, Q[rs], k, nthreads=nth)
        elb = time.perf_counter() - t0
        truth = "oracle float64 brute force"
        cpu["bruteforce"] = {"value": round(len(rs) / elb, 2), "unit": "queries/s", "cores": nth,
                             "sample": f"{len(rs)} sampled queries against all {w.n} points, "
                                       f"{elb:.2f}s wall on {nth} host threads"}
        log(f"oracle brute force: {len(rs)} queries in {elb:.1f}s")
    else:
        # no host leg: the library's exact mode (one tree of depth 0, v = 1:
        # S = X, float32 distances ranked by (distance, id))
        exact = mrpt.Index(Xd, 1, 0, 1.0, 0)
        bi, _ = exact.query(Qd[torch.from_numpy(rs).cuda()], k, 1)
        bi = bi.cpu().numpy()
        exact.close()
        truth = "library exact mode (float32, S = X)"

    def quality(gi, gd):
        rec, err = [], 0.0
        for j, q in enumerate(rs):
            rec.append(len(set(gi[q].tolist()) & set(bi[j].tolist())) / k)
            real = gi[q][gi[q] >= 0]
            d64 = np.sqrt(((X[real].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum(1))
            nz = d64 > 0
            if nz.any():
                err = max(err, float(np.max(np.abs(gd[q][:len(real)][nz] - d64[nz]) / d64[nz])))
        return float(np.mean(rec)), err

    rec32, err32 = quality(gi32, gd32)
    rec16, err16 = quality(gi16, gd16)
    rec8, err8 = quality(gi8, gd8)
    log(f"recall@{k} ({truth}): fp32 {rec32:.4f} bf16+rerank {rec16:.4f} fp8+rerank {rec8:.4f}; "
        f"max rel err {err32:.2e} / {err16:.2e} / {err8:.2e}")

    rec = {
        "metric": METRIC,
        "value": round(qps32, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el32 / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: n={w.n} d={w.d} nq={nq} T={w.T} depth={w.depth} "
                               f"a=1/sqrt(d) k={k} v={v}",
                   "n": w.n, "d": w.d, "nq": nq, "T": w.T, "depth": w.depth, "k": k, "v": v},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "recall_at_k": round(rec32, 4),
        "max_rel_err_vs_fp64": err32,
        "s_size": {"mean": round(float(S.mean()), 1), "p50": float(np.percentile(S, 50)),
                   "p99": float(np.percentile(S, 99))},
        "stages": stages32,
        "vote_roofline": roofline_vote,
        "path_hbm_frac": round(tb32 / (el32 / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "arms": {
            "fp32": {"qps": round(qps32, 1), "ms_per_step": round(el32 / args.steps * 1e3, 4),
                     "recall_at_k": round(rec32, 4), "max_rel_err_vs_fp64": err32, "stages": stages32},
            "bf16_rerank": {"qps": round(qps16, 1), "ms_per_step": round(el16 / args.steps * 1e3, 4),
                            "recall_at_k": round(rec16, 4), "max_rel_err_vs_fp64": err16,
                            "stages": stages16, "roofline": roofline16,
                            "path_hbm_frac": round(tb16 / (el16 / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                            "identical_to_fp32": bool(np.array_equal(gi32, gi16) and np.array_equal(gd32, gd16))},
            "fp8_rerank": {"qps": round(qps8, 1), "ms_per_step": round(el8 / args.steps * 1e3, 4),
                           "recall_at_k": round(rec8, 4), "max_rel_err_vs_fp64": err8, "stages": stages8,
                           "roofline": roofline8,
                           "path_hbm_frac": round(tb8 / (el8 / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                           "ids_equal_fp32_frac": round(float(np.mean(np.all(gi8 == gi32, axis=1))), 4)},
        },
        "build_s": round(build_s, 3),
        "build": {"device_s": round(build["device"], 3),
                  "host_s": round(build["host"], 2) if "host" in build else None,
                  "built_on_device": bool(ix.info.built_on_device), "max_row_nnz": int(ix.info.max_row_nnz),
                  # projection work of the build: n * (nonzeros of all T*depth vectors) multiply-adds
                  "projection_fma": int(w.n) * nnz,
                  "note": "device: projection kernel + per-level cut by rank (radix select of each node's middle key, partition); host: threads over trees"},
        "recall_sample": len(rs),
        "recall_truth": truth,
        "latency": latency,
    }
    ix.close()
    print(json.dumps(rec), flush=True)


def ctypes_void_array(n):
    import ctypes
    return ctypes.c_void_p * n


def ctypes_cast_events(arr):
    import ctypes
    return ctypes.cast(arr, ctypes.c_void_p)


if __name__ == "__main__":
    main()
