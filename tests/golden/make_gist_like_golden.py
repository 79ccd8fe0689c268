"""Write the oracle's golden values of the full-size gist-like workload
(n = 1,000,000, d = 960, 10,000 queries, T = 200, depth = 10, v = 5).

Only the oracle (oracle/) and the seeded generators (workloads.py) are used:
  gist_like_trees.json : SHA-256 of every tree's splits (float32 bit patterns,
                         heap order, little-endian) and perm (int32 ids, leaf
                         after leaf, little-endian), and of the projection
                         vectors (dense float32 rows, tree*depth + level);
  gist_like_knn.npz    : for every query, |S| (int32) and the oracle's k = 10
                         nearest members of S: ids (int32) and float64
                         distances; the k = 100 answer of the first 500
                         queries; and for the first 200 queries the model of
                         each precision arm at k = 10, kp = 40 (bfloat16 and
                         fp8): kept ids, their float64 scores and the answer.

Takes several minutes of host time (the oracle projects with dense rows).
Run from the repository root:  python tests/golden/make_gist_like_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1509_06957_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
K100_QUERIES = 500
ARM_QUERIES = 200


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def main():
    w = W.GIST_LIKE
    t0 = time.time()
    X, Q = W.data(w), W.queries(w)
    print(f"data {time.time() - t0:.0f}s", flush=True)
    nth = oracle.all_threads()
    ix = oracle.build_index(X, w.T, w.depth, w.a, w.index_seed, nthreads=nth)
    print(f"oracle index {time.time() - t0:.0f}s", flush=True)
    trees = {
        "workload": f"{w.name}: n={w.n} d={w.d} T={w.T} depth={w.depth} a=float32(1/sqrt(d)) seed={w.index_seed}",
        "projection_sha256": sha(ix.R.view(np.uint32)),
        "leaf_offsets": ix.off.tolist(),
        "splits_sha256": [sha(ix.splits[t].view(np.uint32)) for t in range(w.T)],
        "perm_sha256": [sha(ix.perm[t]) for t in range(w.T)],
    }
    with open(os.path.join(HERE, "gist_like_trees.json"), "w") as f:
        json.dump(trees, f, indent=0)
    r10 = oracle.query(ix, Q, 10, w.v, nthreads=nth)
    print(f"oracle k=10 {time.time() - t0:.0f}s", flush=True)
    r100 = oracle.query(ix, Q[:K100_QUERIES], 100, w.v, nthreads=nth)
    print(f"oracle k=100 {time.time() - t0:.0f}s", flush=True)
    arms = {}
    for name, arm in (("bf16", oracle.ARM_BF16), ("fp8", oracle.ARM_FP8)):
        r = oracle.query_prefilter(ix, Q[:ARM_QUERIES], 10, w.v, arm, 40, nthreads=nth)
        arms[f"{name}_keep_ids"] = r["keep_ids"]
        arms[f"{name}_keep_score"] = r["keep_score"]
        arms[f"{name}_idx"] = r["idx"]
        arms[f"{name}_dist"] = r["dist"]
        print(f"oracle {name} arm {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "gist_like_knn.npz"),
                        s_count=r10["s_count"].astype(np.int32),
                        idx10=r10["idx"], dist10=r10["dist"],
                        idx100=r100["idx"], dist100=r100["dist"], **arms)
    print("written", flush=True)


if __name__ == "__main__":
    main()
