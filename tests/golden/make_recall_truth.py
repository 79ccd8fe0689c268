"""Write the exact k-NN of a workload's recall sample, computed by the
oracle's float64 brute force (Sec. I-A: the k points of X nearest to q in
Euclidean distance, order (distance, id)).  Sweeps grade recall against it.

Only the oracle (oracle/) and the seeded generators (workloads.py) are used.
The sample is the one bench.py and sweep.py draw: numpy default_rng(0)
choosing `sample` of the workload's queries without replacement.

Output: tests/golden/<workload>_truth_k<k>.npz with `sample` (int64 query
numbers), `idx` (int32, sample x k) and `dist` (float64, sample x k).
Run from the repository root:
    python tests/golden/make_recall_truth.py sift_like [gist_like ...] [--k K] [--sample M]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1509_06957_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("workloads", nargs="+")
    p.add_argument("--k", type=int, default=None, help="default: the workload's k")
    p.add_argument("--sample", type=int, default=500)
    args = p.parse_args()
    for name in args.workloads:
        w = W.ALL[name]
        k = args.k or w.k
        t0 = time.time()
        X, Q = W.data(w), W.queries(w)
        rs = np.random.default_rng(0).choice(w.nq, size=min(args.sample, w.nq), replace=False)
        idx, dist = oracle.bruteforce(X, Q[rs], k, nthreads=oracle.all_threads())
        path = os.path.join(HERE, f"{name}_truth_k{k}.npz")
        np.savez_compressed(path, sample=rs.astype(np.int64), idx=idx, dist=dist)
        print(f"{name}: {len(rs)} queries, k = {k}, {time.time() - t0:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    main()
