/*
 * mrpt.h -- C ABI of the MI355X (gfx950) query path of multiple random
 * projection trees with voting search ("Fast k-NN Search", Hyvonen et al.,
 * arXiv:1509.06957).
 *
 * The problem (paper Sec. I-A): X holds n points of R^d; for a query q the
 * answer is the k points of X closest to q in Euclidean distance.  The index
 * (Sec. II, Alg. 1-2) is T random projection trees of depth `depth`, each
 * using one sparse Gaussian vector per level (Sec. II-B, II-C) and median
 * splits.  A query (Sec. III, Alg. 3-4) is routed to one leaf per tree, every
 * point gets one vote per tree whose leaf it shares with q, the points with
 * at least v votes form the candidate set S, and the k nearest members of S
 * are returned.
 *
 * Conventions shared by every entry point:
 *   - All calls return an mrpt_status and never throw.  On error the output
 *     buffers are left untouched and mrpt_last_error() (thread-local) names
 *     the problem.
 *   - "device" pointers are HIP device memory of the current device (e.g. a
 *     torch CUDA tensor's data_ptr()); "host" pointers are ordinary memory.
 *   - Matrices are row-major float32: X is n x d, Q is nq x d.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Query calls are
 *     asynchronous on that stream: they read Q and write the outputs in stream
 *     order and return before the work completes.
 *   - An index is immutable after mrpt_build.  It owns a workspace for query
 *     temporaries; calls on one index made from several host threads are
 *     serialised by the library, and calls on different streams are ordered
 *     through an event, so they are safe but do not overlap on the GPU.
 *
 * Limits (MRPT_EINVAL beyond them): 1 <= d <= 65535, 1 <= n < 2^31,
 * 2^depth <= n, depth <= 24, 1 <= T <= 255, 0 < a <= 1, 1 <= k <= min(n, 1024),
 * 1 <= v <= T.
 */
#ifndef MRPT_H
#define MRPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrpt_index mrpt_index;

typedef enum {
    MRPT_OK = 0,
    MRPT_EINVAL = -1,      /* bad argument (sizes, limits, null pointer) */
    MRPT_ENOMEM = -2,      /* device or host allocation failed */
    MRPT_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed */
    MRPT_ENONFINITE = -4,  /* NaN or Inf in the data (build) or, when asked, in Q */
    MRPT_EINTERNAL = -5    /* an internal consistency check failed */
} mrpt_status;

typedef enum {
    MRPT_FP32 = 0,         /* exact search in S with float32 distances */
    MRPT_BF16_RERANK = 1,  /* bfloat16 prefilter over S, float32 rerank of the best
                              rerank_factor*k, float64 recheck at the k-th boundary
                              (d % 8 == 0, d <= 1024) */
    MRPT_FP8_RERANK = 2    /* as MRPT_BF16_RERANK with an fp8 (e4m3) prefilter: rows
                              quantized at build time with a per-row scale max|x|/240
                              (d % 16 == 0, d <= 1024); lossy for general data, so S's
                              true k nearest can fall outside the reranked set */
} mrpt_precision;

typedef struct {
    int32_t precision;     /* mrpt_precision; default MRPT_FP32 */
    int32_t rerank_factor; /* prefilter arms: keep the best rerank_factor*k of the prefilter
                              (default 4; rerank_factor*k <= 512) */
    float recheck_rel;     /* prefilter arms: candidates whose float32 distance is within
                              recheck_rel (relative) of the k-th are re-ranked in
                              float64 (default 1e-6) */
    int32_t check_finite;  /* 1: scan Q for NaN/Inf first and return MRPT_ENONFINITE
                              (this synchronises the stream); 0: no check, and a
                              non-finite query row yields unspecified but in-range
                              results */
    int32_t* s_count;      /* optional device int32[nq]: receives |S| per query */
    void* const* stage_events; /* optional host array of 4 hipEvent_t, recorded on `stream`
                              before the routing kernel, after it, after the vote kernel
                              and after the exact-search kernel (of the first sub-batch
                              when a large batch is processed in several) */
} mrpt_query_opts;

typedef struct {
    int64_t n;
    int32_t d, T, depth;
    float a;
    uint64_t seed;
    int64_t nnz;           /* nonzeros of the T*depth projection vectors */
    int32_t max_leaf;      /* ceil(n / 2^depth) */
    int32_t id_chunk;      /* ids per vote-counting pass of the query kernels */
    int64_t device_bytes;  /* device memory held by the index (without workspace) */
    int32_t built_on_device; /* 1: the trees were grown on the GPU; 0: on host threads
                              (mrpt_build_opts.on_device = 0) */
    int32_t max_row_nnz;   /* nonzeros of the longest projection vector */
} mrpt_index_desc;

/* Build the index (paper Alg. 1 grow_trees, Alg. 2 grow_tree; Sec. II-B sparse
 * vectors with density a; Sec. II-C one vector per level).
 *   data  : device, n x d float32, finite.  Copied; the caller keeps ownership.
 *   seed  : the projection vectors are a pure function of (seed, tree, level,
 *           feature), so tree t is the same for every T > t.
 *   out   : receives the new index (release with mrpt_free).
 * Synchronous: the device is synchronised before returning.  Errors:
 * MRPT_EINVAL, MRPT_ENONFINITE, MRPT_ENOMEM, MRPT_EDEVICE. */
mrpt_status mrpt_build(const float* data, int64_t n, int32_t d, int32_t T, int32_t depth,
                       float a, uint64_t seed, mrpt_index** out);

/* Index build options. */
typedef struct {
    int32_t on_device;     /* 1 (default): grow the trees on the GPU (data projected by the
                              query path's projection kernel, every node of a level cut by
                              rank: a radix select of its middle (projection, id) key and a
                              partition; MRPT_BUILD_SORT=1 sorts each level instead); 0: on
                              host threads.  All give
                              bit-identical trees.  The GPU build takes scratch device memory
                              of about n*(4*depth + 16) bytes per tree of a group (groups
                              sized to MRPT_BUILD_LIMIT bytes, default 8 GiB). */
    int32_t exact_nnz;     /* 0 (default): each entry of a projection vector is nonzero with
                              probability a (Sec. II-B).  1: every vector has exactly
                              m = ceil(a*d) nonzeros (the variant of the Sec. II-D footnote):
                              the m features whose selection uniform is smallest, ties by
                              feature; values as in the default mode.  With a = 1 both
                              modes give the same vectors. */
} mrpt_build_opts;

/* Default build options (on_device = 1, exact_nnz = 0). */
void mrpt_default_build_opts(mrpt_build_opts* opts);

/* mrpt_build with options (opts = NULL: the defaults). */
mrpt_status mrpt_build_ex(const float* data, int64_t n, int32_t d, int32_t T, int32_t depth, float a,
                          uint64_t seed, const mrpt_build_opts* opts, mrpt_index** out);

/* Approximate k-NN of nq queries (paper Alg. 4 approximate_knn with Alg. 3
 * tree_query), float32 exact search in S.
 *   Q        : device, nq x d float32.
 *   out_idx  : device int32[nq*k]; row q holds the ids of the k nearest members
 *              of S_q ordered by (distance, id); -1 pads rows with |S_q| < k.
 *   out_dist : device float32[nq*k]; Euclidean distances (not squared); +inf pads.
 * nq = 0 is a no-op.  Asynchronous on `stream`. */
mrpt_status mrpt_query(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                       int32_t* out_idx, float* out_dist, void* stream);

/* mrpt_query with options (precision arm, rerank factor, finite check, |S|
 * export).  opts = NULL means the defaults, i.e. mrpt_query. */
mrpt_status mrpt_query_ex(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                          int32_t* out_idx, float* out_dist, const mrpt_query_opts* opts,
                          void* stream);

/* Bytes of the device array that holds mrpt_query_noalloc's temporaries (one
 * array per GPU, held from the library's load until the process ends). */
#define MRPT_NOALLOC_SCRATCH_BYTES (128u << 20)

/* mrpt_query_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as mrpt_query_ex, but no call allocates
 * (no hipMalloc, hipFree or allocating library routine): the query
 * temporaries (per query about 4*(T + T*ceil(n/2^depth)/v + 1) bytes plus
 * 4*T*depth for the projections) live in a fixed device array of
 * MRPT_NOALLOC_SCRATCH_BYTES, and a batch whose temporaries do not fit runs
 * as several sub-batches in stream order.
 *   Errors: as mrpt_query_ex, and MRPT_EINVAL when a single query's
 *   temporaries exceed MRPT_NOALLOC_SCRATCH_BYTES.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on
 * the GPU (several host threads, or several streams without an order between
 * them) race and give undefined results; calls in one stream are ordered.
 * The array keeps the last call's contents; nothing in it is assumed zero.
 * opts->check_finite = 1 synchronises the stream (not capturable). */
mrpt_status mrpt_query_noalloc(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                               int32_t* out_idx, float* out_dist, const mrpt_query_opts* opts,
                               void* stream);

/* Default options (MRPT_FP32, rerank_factor 4, recheck_rel 1e-6, no check, no
 * |S| export, no stage events). */
void mrpt_default_opts(mrpt_query_opts* opts);

/* Release an index and all device memory it owns (NULL is ignored).  The
 * device is synchronised first. */
void mrpt_free(mrpt_index* ix);

/* Message of the last failed call on this host thread ("" if none). */
const char* mrpt_last_error(void);

/* Sizes and parameters of a built index. */
mrpt_status mrpt_index_info(const mrpt_index* ix, mrpt_index_desc* out);

/* ---------------------------------------------------------------------------
 * Query plans: many query batches, over any number of indexes, recorded once
 * as one HIP graph and replayed with a single launch.  Each batch is the
 * search of Sec. III (Alg. 3-4) exactly as mrpt_query_ex runs it, with the same
 * kernels, so a batch's results equal mrpt_query_ex's for the same arguments.
 *
 * Batches with the same (index, k, v) are searched as one query call: their
 * queries are gathered into a staging array and the results scattered back
 * (every step works per query, so the results are the per-batch ones).  A
 * plan owns the workspace and staging memory of every such group.  By
 * default (fused) each stage of the search (routing, voting, exact search)
 * is one launch per kernel form over all groups of that form, whatever
 * their index: the kernels read each group's index arrays, queries,
 * workspace and outputs from a device table.  Otherwise the groups are dealt
 * over `branches` independent chains of the graph (balanced by estimated
 * work), and the GPU may run the chains concurrently.  The plan keeps the pointers it was given: each launch
 * reads the current contents of every batch's Q and overwrites its outputs,
 * in the launch stream's order.
 * The indexes must outlive the plan.  Launches of one plan must not overlap
 * (they share the workspaces): order them on one stream or synchronise.
 */
typedef struct mrpt_batch {
    const mrpt_index* index;  /* the index searched */
    const float* Q;           /* device float[nq*d] (d of that index) */
    int64_t nq;               /* queries of the batch, >= 1 */
    int32_t k;                /* neighbours per query, as for mrpt_query */
    int32_t v;                /* vote threshold, as for mrpt_query */
    int32_t* out_idx;         /* device int32[nq*k] */
    float* out_dist;          /* device float[nq*k] */
} mrpt_batch;

typedef struct mrpt_plan_opts {
    int32_t precision;      /* mrpt_precision of every batch (default MRPT_FP32) */
    int32_t rerank_factor;  /* as in mrpt_query_opts (default 4) */
    float recheck_rel;      /* as in mrpt_query_opts (default 1e-6) */
    int32_t branches;       /* 1..64 (default 4): streams a stage's launches are spread over
                               (fused), or independent chains of groups (not fused) */
    int32_t proj_rows;      /* projection vectors per wave: 0 (default) the launcher's choice
                               (4 for launches under 512 workgroups, else 16), or 4, or 16 */
    int32_t vote_kernel;    /* 0 (default) automatic; 1 the single-pass vote kernel wherever it
                               fits; 2 the multi-pass one. */
    int32_t fused;          /* 1 (default): one launch per stage for all groups of a kernel form
                               (calls of the same kernel shape, whatever their index), driven by
                               device tables of (index arrays, query range, k, v, workspace); the
                               launches of one stage run side by side on `branches` streams and
                               a stage starts when the previous one has ended; 0: every group its
                               own chain of launches, dealt over `branches`.  None of these knobs
                               changes a result; they are there for tuning the launches. */
    int32_t vote_waves;     /* waves per workgroup of the single-pass vote kernel: 0 (default)
                               automatic (8, two workgroups per CU, where half of LDS holds the
                               index's map and a queue for every repeat of a query or 4,096 of
                               them, else 16); 16; or 8 wherever the map fits half of LDS (a
                               smaller repeat queue: overflowing queries are recounted). */
} mrpt_plan_opts;

typedef struct mrpt_plan mrpt_plan;

/* Fills *opts with the defaults above. */
void mrpt_default_plan_opts(mrpt_plan_opts* opts);

/* Checks every batch as mrpt_query_ex would (MRPT_EINVAL names the first bad
 * batch), allocates the workspaces (MRPT_ENOMEM) and records the graph.
 * Synchronous; nothing is computed.  nbatch >= 1.  *out receives the plan. */
mrpt_status mrpt_plan_create(const mrpt_batch* batches, int32_t nbatch, const mrpt_plan_opts* opts,
                             mrpt_plan** out);

/* Runs every batch of the plan: one graph launch on `stream` (hipStream_t,
 * NULL = the null stream).  Asynchronous. */
mrpt_status mrpt_plan_launch(mrpt_plan* plan, void* stream);

/* Bytes of device memory the plan holds (workspaces, staging arrays, copy tables). */
int64_t mrpt_plan_device_bytes(const mrpt_plan* plan);

/* Releases the plan (after its last launch has completed).  NULL is a no-op. */
void mrpt_plan_free(mrpt_plan* plan);

/* Debug export of the projection vectors (Sec. II-B), one CSR row per (tree,
 * level) in order tree*depth + level, features ascending.
 *   rowptr : host int32[T*depth + 1];  col : host int32[nnz];  val : host float[nnz]. */
mrpt_status mrpt_export_projection(const mrpt_index* ix, int32_t* rowptr, int32_t* col, float* val);

/* Debug export of tree t (Alg. 2): splits host float[2^depth - 1] in heap
 * order (children of node i are 2i+1 and 2i+2), perm host int32[n] = the
 * point ids leaf after leaf (left to right), ascending inside each leaf.
 * Either pointer may be NULL. */
mrpt_status mrpt_export_tree(const mrpt_index* ix, int32_t t, float* splits, int32_t* perm);

/* Debug export of the leaf offsets: host int64[2^depth + 1]; leaf L of every
 * tree is perm[off[L] .. off[L+1]). */
mrpt_status mrpt_export_leaf_offsets(const mrpt_index* ix, int64_t* off);

/* Debug: the leaf of every query in every tree (Alg. 3), computed by the same
 * kernel the query path runs.  leaf: device int32[nq*T].  Asynchronous. */
mrpt_status mrpt_debug_leaves(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf,
                              void* stream);

/* Debug: the candidate sets S_q = {x : F(x; q) >= v} (Sec. III-A) computed by
 * the query path's vote kernel.
 *   s_count : device int32[nq]       |S_q|
 *   s_ids   : device int32[nq*cap]   members of S_q, in no particular order
 *   s_votes : device uint8[nq*cap]   F(x; q) of each listed member (may be NULL)
 *   cap     : row stride of s_ids/s_votes; must be >= min(n, floor(T*max_leaf/v))
 * Asynchronous. */
mrpt_status mrpt_debug_votes(const mrpt_index* ix, const float* Q, int64_t nq, int32_t v,
                             int32_t* s_count, int32_t* s_ids, uint8_t* s_votes, int64_t cap,
                             void* stream);

/* Debug: the kept list of a prefilter arm (opts->precision MRPT_BF16_RERANK or
 * MRPT_FP8_RERANK), computed by the query path's own kernels up to the end of
 * the prefilter ranking: S_q is formed as in mrpt_query_ex, ranked by the
 * low-precision squared distance ||q||^2 + ||x~||^2 - 2 q.x~ (x~ the bfloat16
 * row, or the fp8 row times its scale), and the best kp = rerank_factor*k under
 * (score, id) are kept.
 *   s_count  : device int32[nq]        |S_q|
 *   keep_ids : device int32[nq*kp]     row q: the kept ids, best first; -1
 *              past min(|S_q|, kp).  When |S_q| <= kp nothing is ranked and
 *              the row holds S_q in no particular order.
 * Arguments and errors as mrpt_query_ex (MRPT_EINVAL for the float32 arm).
 * Asynchronous on `stream`. */
mrpt_status mrpt_debug_prefilter(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                                 const mrpt_query_opts* opts, int32_t* s_count, int32_t* keep_ids,
                                 void* stream);

/* Debug: the index's low-precision copy of rows [row0, row0 + nrows) of X.
 *   precision  : MRPT_BF16_RERANK: rows receives uint16 bfloat16 patterns
 *                (round to nearest even of the float32 value), nrows*d of them;
 *                MRPT_FP8_RERANK: rows receives uint8 E4M3 codes, nrows*d, and
 *                scale_norm (may be NULL) float[2*nrows] pairs (scale =
 *                max|x|/240, squared norm of scale*decode(codes)).
 *   rows, scale_norm : device memory.  Asynchronous on `stream`.
 * MRPT_EINVAL for a row range outside [0, n) or an index without fp8 rows. */
mrpt_status mrpt_debug_lowp_rows(const mrpt_index* ix, int32_t precision, int64_t row0, int64_t nrows,
                                 void* rows, float* scale_norm, void* stream);

/* Upper bound used for the per-query candidate buffer: min(n, floor(T*max_leaf/v)). */
int64_t mrpt_candidate_cap(const mrpt_index* ix, int32_t v);

#ifdef __cplusplus
}
#endif

#endif /* MRPT_H */
