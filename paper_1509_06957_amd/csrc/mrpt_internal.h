// Internal declarations of libmrpt (the GPU library).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrpt.h"

namespace mrpt {

// ---------------------------------------------------------------- errors
mrpt_status fail(mrpt_status st, const char* fmt, ...);
void clear_error();

#define MRPT_HIP_TRY(expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::mrpt::fail(MRPT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define MRPT_TRY(expr)                        \
    do {                                      \
        mrpt_status s_ = (expr);              \
        if (s_ != MRPT_OK) return s_;         \
    } while (0)

// ---------------------------------------------------------------- limits
constexpr int kMaxT = 255;          // 8-bit vote counters
constexpr int kMaxDepth = 24;
constexpr int kMaxK = 1024;
constexpr int kMaxRerank = 512;     // rerank_factor * k
// Each tree's row of perm is padded with kPermPad entries holding n, n + 1,
// ...: a vote kernel reads an empty lane of a window from there instead of
// branching around the load, so every slot issues exactly one load.
constexpr int kPermPad = 2048;
// leaf directory grain: the multi-pass vote kernel's passes start on
// multiples of it, and the directory holds each leaf's position of them
constexpr int kDirGrain = 32768;

// ---------------------------------------------------------------- index
struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Workspace {
    int32_t* leaf = nullptr;     // nb x T
    int32_t* s_ids = nullptr;    // nb x cap
    int32_t* s_count = nullptr;  // nb
    int32_t* flag = nullptr;     // 1 int
    void* base = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;   // recorded after the last kernel that used it
};

}  // namespace mrpt

struct mrpt_index {
    int64_t n = 0;
    int32_t d = 0, T = 0, depth = 0;
    float a = 0.f;
    uint64_t seed = 0;
    int32_t nleaf = 1;           // 2^depth
    int32_t max_leaf = 0;        // ceil(n / 2^depth)
    int32_t id_chunk = 0;        // ids per vote pass at v = 1 (reported by mrpt_index_info)
    int32_t max_row_nnz = 0;     // largest number of nonzeros of one projection vector
    int32_t built_on_device = 0; // trees grown by the GPU build
    int device = 0;

    // host copy of the projection CSR (for export)
    std::vector<int32_t> h_rowptr;
    std::vector<int32_t> h_col;
    std::vector<float> h_val;
    std::vector<int64_t> h_off;

    // device arrays
    float* X = nullptr;          // n x d
    uint16_t* Xb = nullptr;      // n x d bfloat16 bits (round to nearest even)
    uint8_t* X8 = nullptr;       // n x d fp8 (e4m3) codes (d % 16 == 0 and d <= 1024, else unset)
    float2* sn8 = nullptr;       // n: (per-row scale of the fp8 codes, squared norm of the decoded row)
    int32_t* rowptr = nullptr;   // T*depth + 1
    int32_t* col = nullptr;      // nnz
    float* val = nullptr;        // nnz
    float* splits = nullptr;     // T x (2^depth - 1)
    int32_t* vdir = nullptr;     // leaf directory (T x 2^depth x vdir_nb), or null
    int32_t vdir_nb = 0;         // boundaries per leaf: ceil(n / kDirGrain) + 1
    int32_t* perm = nullptr;     // T rows of perm_ld: the tree's ids, then kPermPad entries n + j
    int64_t perm_ld = 0;         // n + kPermPad
    int32_t* off = nullptr;      // 2^depth + 1
    int64_t device_bytes = 0;

    std::mutex mu;               // guards ws
    mrpt::Workspace ws;
};

namespace mrpt {

// host-side index construction (host_build.cpp)
struct HostTrees {
    std::vector<float> splits;   // T x (2^depth - 1)
    std::vector<int32_t> perm;   // T x n
    std::vector<int64_t> off;    // 2^depth + 1
};
// projection vectors as CSR rows (tree * depth + level), features ascending;
// exact: ceil(a d) nonzeros per vector instead of Bernoulli(a) entries
void generate_projection(int32_t d, int32_t T, int32_t depth, float a, uint64_t seed, bool exact,
                         std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                         std::vector<float>& val);
int32_t exact_nnz_count(int32_t d, float a);
void leaf_offsets(int64_t n, int32_t depth, std::vector<int64_t>& off);
void grow_trees_host(const float* X, int64_t n, int32_t d, int32_t T, int32_t depth,
                     const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                     const std::vector<float>& val, HostTrees& out);

// device index build (kernels_build.hip): trees [t0, t0 + g) into ix->splits
// and ix->perm.  level_off[lv]: node offsets of level lv (lv = 0..depth).
// Scratch: P (g * depth * n floats), keys_a/keys_b (g * n each), seg_off
// (g * 2^depth + 1), node_off (2^depth + 1); temp grows as the sort needs.
size_t device_build_bytes_per_tree(int64_t n, int32_t depth);
hipError_t grow_trees_device(mrpt_index* ix, int32_t t0, int32_t g,
                             const std::vector<std::vector<int64_t>>& level_off, float* P, uint64_t* keys_a,
                             uint64_t* keys_b, void*& temp, size_t& temp_bytes, int32_t* seg_off,
                             int64_t* node_off, hipStream_t s);

// kernel launchers (kernels_route/vote/search/misc.hip); all asynchronous
// kernel variants a caller may pin (0 = the launcher's own choice); none of
// them changes a result
struct LaunchCfg {
    int32_t proj_rows = 0;     // projection vectors per wave: 4 or 16
    int32_t vote_kernel = 0;   // 1: single-pass where it fits, 2: multi-pass
    int32_t vote_waves = 0;    // single-pass workgroup: 0 automatic, 8 or 16 waves
};

// projections of the m rows of A onto vectors row0 .. row0 + nrows - 1:
// P[r * m + i] (the float32 fused multiply-add chain of Sec. II-C)
hipError_t launch_project(const mrpt_index* ix, const float* A, int64_t m, int32_t row0, int32_t nrows, float* P,
                          hipStream_t s, int32_t rows_per_wave = 0);
// leaf numbers leaf[q * T + t] of the nq queries of Q (Alg. 3)
hipError_t launch_route(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf, hipStream_t s,
                        const LaunchCfg& cfg = LaunchCfg());
hipError_t launch_vote(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v,
                       int32_t* s_ids, int64_t cap, int32_t* s_count, hipStream_t s,
                       const LaunchCfg& cfg = LaunchCfg());
// the leaf directory of the multi-pass vote kernel, when the index needs one
// (after perm and the leaf offsets are on the device); adds its bytes to *tally
hipError_t build_vote_directory(mrpt_index* ix, int64_t* tally);
hipError_t launch_vote_counts(const mrpt_index* ix, const int32_t* leaf, int64_t nq,
                              const int32_t* s_ids, int64_t cap, const int32_t* s_count,
                              uint8_t* s_votes, hipStream_t s);
hipError_t launch_dist_fp32(const mrpt_index* ix, const float* Q, int64_t nq,
                            const int32_t* s_ids, int64_t cap, const int32_t* s_count, int32_t k,
                            int32_t* out_idx, float* out_dist, hipStream_t s);
// bf16 (fp8 = 0) or fp8 (fp8 = 1) prefilter, float32 rerank, float64 recheck;
// keep_out (device int32[nq * k * rerank]) non-null: phase 1 only, the kept
// list of every query instead of the k-NN
hipError_t launch_dist_prefilter(const mrpt_index* ix, int fp8, const float* Q, int64_t nq, const int32_t* s_ids,
                                 int64_t cap, const int32_t* s_count, int32_t k, int32_t rerank, float recheck_rel,
                                 int32_t* out_idx, float* out_dist, hipStream_t s, int32_t* keep_out = nullptr);
hipError_t launch_copy_counts(const int32_t* src, int64_t nq, int32_t* dst, hipStream_t s);

// ---------------------------------------------------------------- multi-index launches
// One launch of a stage over the queries of several query calls (a query
// plan's groups) whose kernel form is the same: the calls are the items of a
// device table, in ascending order of their first workgroup (row0).

// exact search: one workgroup per query
struct SearchItem {
    const float* X;              // the index's float32 rows
    const uint8_t* Xq;           // its bfloat16 (or fp8) rows, prefilter arms
    const float2* sn8;           // its fp8 scales and norms, fp8 arm
    const float* Q;              // the call's queries
    const int32_t* s_ids;        // its candidate lists (cap per query)
    const int32_t* s_count;      // its |S| per query
    int32_t* out_idx;
    float* out_dist;
    int64_t cap;
    int64_t row0;                // first workgroup of the call
    int32_t k, kp;               // kp = rerank_factor * k (prefilter arms)
};
// voting, single-pass map kernel: one item per call (also the single-call
// kernel's argument)
struct VoteItem {
    const int32_t* leaf;         // the call's leaf numbers (nq x T)
    const int32_t* perm;         // its index's leaf lists
    const int32_t* off;          // its leaf offsets
    int32_t* s_ids;              // candidate lists (cap per query)
    int32_t* s_count;            // |S| per query (-1: repeat queue overflowed)
    int64_t cap, ld;             // candidate cap; perm row length
    int64_t row0;                // first row of the call in a multi-index launch
    int32_t n, v;
    int32_t map_words;           // map words its ids use (n + 2048 padding ids)
    int32_t pad_;
};

// the single-pass vote form of a call (equal forms share a launch: slot
// class, queueing, waves per workgroup, T, windows per leaf), -1 when the
// call needs the multi-pass kernel; map words of an index; the most repeats
// one query can queue; the queue capacity of a multi-index launch of that
// form whose map holds map_words (-1 when too small); the launch itself
// (rows whose queue overflows get count -1, counted again by
// launch_vote_recount)
int64_t vote_form(const mrpt_index* ix, int32_t v, const LaunchCfg& cfg);
int32_t vote_map_words(const mrpt_index* ix);
int64_t vote_most_queued(const mrpt_index* ix);
int64_t vote_multi_qcap(int64_t form, int32_t map_words, int64_t most_occurrences);
hipError_t launch_vote_multi(int64_t form, int32_t map_words, int64_t qcap, const VoteItem* items,
                             const int32_t* row_item, int64_t nrows, hipStream_t s);
hipError_t launch_vote_recount(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                               int64_t cap, int32_t* s_count, hipStream_t s);

// routing (projection and split walk in one kernel): one item per call, the
// workgroups of its grid (query tiles x tree groups) flattened (x fastest)
struct RouteItem {
    const float* Q;              // the call's queries
    const int32_t* rowptr;       // its index's projection vectors (CSR)
    const int32_t* col;
    const float* val;
    const float* splits;         // its split tables
    int32_t* leaf;               // leaf numbers (nq x T)
    int64_t nq;
    int64_t blk0;                // first workgroup of the call in the launch
    int64_t nbx;                 // workgroups along the queries
    int32_t d, T, depth;
    int32_t nby;                 // workgroups along the trees (tree groups)
};
// the routing form of a call's index (equal forms can share the launch),
// -1 without a multi-index form (vectors over 64 nonzeros)
int32_t route_form(const mrpt_index* ix);
// the routing kernel of `form` serves this index (its depth within the
// form's depth class): checked for every item before a launch is recorded
bool route_form_holds(int32_t form, const mrpt_index* ix);
// grid of a call in the routing launch: query tiles x tree groups
struct RouteGrid {
    int32_t rpw, qpl;            // projection rows per wave, queries per lane
    int64_t nbx, nby;
};
RouteGrid route_grid(const mrpt_index* ix, int64_t nq, int32_t rpw, int32_t qpl);
// the launch-wide projection shape of a form for a set of calls: rows per
// wave and queries per lane (total_tiles: their workgroups at 16 rows per wave)
void route_shape(int32_t form, int64_t total_tiles, int32_t rows_per_wave, int32_t* rpw, int32_t* qpl);
hipError_t launch_route_multi(int32_t form, int32_t rpw, int32_t qpl, int32_t max_d, const RouteItem* items,
                              int32_t nitems, int64_t blocks, hipStream_t s);

// the search kernel form of a call (calls of equal form can share a launch),
// or -1 when the call's form has no multi-index kernel (its own launch then);
// precision as mrpt_precision
int32_t search_form(const mrpt_index* ix, int32_t precision, int32_t k, const float* Q);
hipError_t launch_search_multi(int32_t form, int32_t d, const SearchItem* items, int32_t nitems, int64_t rows,
                               float recheck_rel, hipStream_t s);
hipError_t launch_check_finite(const float* A, int64_t count, int32_t* flag, hipStream_t s);
hipError_t launch_quantize_bf16(const float* X, int64_t n, int32_t d, uint16_t* Xb, hipStream_t s);
// device-to-device copies of 4-byte words, one job per row of the grid
// (jobs: device array; max_words: the largest job, sizes the grid)
struct CopyJob {
    const int32_t* src;
    int32_t* dst;
    int64_t words;
};
hipError_t launch_copy_jobs(const CopyJob* jobs, int32_t njobs, int64_t max_words, hipStream_t s);
hipError_t launch_quantize_fp8(const float* X, int64_t n, int32_t d, uint8_t* X8, float2* sn8, hipStream_t s);

}  // namespace mrpt
