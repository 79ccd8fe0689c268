// Routing kernel: the sparse projection of a query tile onto the depth
// vectors of each tree (Sec. II-C: one vector per tree level, so a query's
// T*depth projections form one sparse product) fused with the descent of
// Alg. 3: at level j the query goes left when its projection is <= the node's
// split (Sec. III), right otherwise.  Every projection is a float32 fused
// multiply-add chain in ascending feature order from +0.
//
// project_route_kernel: a workgroup projects a 64- or 128-query tile on the
// rows of a group of trees, keeps the projections in LDS and walks those
// trees.  project_kernel is its projection half alone, writing the rows to
// memory (the index build projects the data with it).
#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

using namespace dev;

constexpr int kQStride = 65;
constexpr int kStageUnroll = 8;     // global loads in flight per thread while staging

// features [c0, c0 + cw) of the 64-query tile starting at q0 into LDS as
// qt[(feature - c0) * 65 + query]; rows past nq read as zero
__device__ __forceinline__ void stage_query_chunk(const float* __restrict__ Q, int64_t q0, int64_t nq, int d, int c0,
                                                  int cw, float* qt, int fstride = kQStride) {
    const int tid = (int)threadIdx.x, nthreads = (int)blockDim.x;
    const int total = kWave * cw;
    const int step_q = nthreads / cw, step_f = nthreads - step_q * cw;
    int qq = tid / cw, f = tid - qq * cw;
    const float* src = Q + q0 * d + c0;
    const int64_t rows_left = nq - q0;
    for (int e0 = tid; e0 < total; e0 += kStageUnroll * nthreads) {
        float r[kStageUnroll];
        int rq[kStageUnroll], rf[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int e = e0 + u * nthreads;
            rq[u] = qq;
            rf[u] = f;
            r[u] = (e < total && qq < rows_left) ? src[(int64_t)qq * d + f] : 0.0f;
            qq += step_q;
            f += step_f;
            if (f >= cw) { f -= cw; ++qq; }
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u)
            if (e0 + u * nthreads < total) qt[rf[u] * fstride + rq[u]] = r[u];
    }
}

// ---------------------------------------------------------------------------
// The projection Pq[r][q] = q . R_r (the sparse product of Sec. II-C): a
// workgroup takes a tile of 64 * QPL queries (staged in LDS as
// [feature][query]) and 8 waves x RPW rows; a wave keeps its RPW rows in
// registers (lane e holds entry e; vectors of more than 64 nonzeros are
// taken 64 entries at a time) and advances them together, one nonzero per
// row per step, so RPW * QPL fused multiply-add chains overlap while each
// runs in ascending feature order.  The steps that every row has run
// without a branch.  project_kernel writes the rows to memory (index build);
// project_route_kernel keeps them in LDS and walks the trees (Alg. 3's
// descent) in the same workgroup.
// ---------------------------------------------------------------------------
constexpr int kProjWaves = 8;

// Workgroup order of the (query tile, row or tree group) grids, launched as
// one dimension.  Consecutive workgroups go to the eight XCDs in turn, each
// with its own L2, so workgroup r runs on XCD r mod 8.  The grid's nbx * nby
// workgroups in tile-major order (the groups of one tile consecutive) are cut
// into eight contiguous runs, one per XCD, taken in order: every group of a
// query tile runs on one XCD (two at a run's edge), one after another, and
// stages the tile from that XCD's L2 after the first.  With the tile's groups
// spread over all XCDs, each read it from memory again.  The map is a
// bijection of [0, nbx * nby) for any XCD count; eight is the one it is
// tuned for.  An offset to r that is the same for the whole grid (a
// multi-index launch's item) keeps the property.
constexpr int kXcds = 8;
// most workgroups of a one-dimensional launch: the dispatch counts the grid
// in work-items, fewer than 2^32 per dimension
constexpr int64_t kMaxGrid = ((int64_t(1) << 32) - 1) / (kProjWaves * kWave);
__device__ __forceinline__ void xcd_tile_group(int64_t r, int64_t nbx, int32_t nby, int64_t& tile, int32_t& grp) {
    const int64_t n = nbx * nby;
    const int64_t per = n / kXcds, extra = n - per * kXcds;
    const int64_t x = r % kXcds, k = r / kXcds;
    const int64_t m = x * per + (x < extra ? x : extra) + k;
    tile = m / nby;
    grp = (int32_t)(m - tile * nby);
}

// The workgroup's 64-query tile is staged in LDS as [feature][query], in
// chunks of at most kProjChunk features when d is wider.  A vector's
// nonzeros are in ascending feature order, so those of one chunk are a
// contiguous run of its list (found by a ballot): every fused multiply-add
// chain still runs over the features in ascending order, chunk after chunk.
constexpr int kProjChunk = (64 * 1024) / (kQStride * 4);   // 252 features: 64 KB of LDS

// The tile of 64 * QPL queries from q0 (d features, d % 4 == 0, rows 16-byte
// aligned) into LDS as qt[f * QPL * 65 + (r / 64) * 65 + r % 64] for tile
// row r; rows past nq read as zero.  Each thread issues all its 16-byte
// loads before it stores any: one memory round trip for the tile when it
// holds at most kStageUnroll loads per thread (d = 128, two 64-query halves).
template <int QPL>
__device__ __forceinline__ void stage_tile_v4(const float* __restrict__ Q, int64_t q0, int64_t nq, int d,
                                              float* qt) {
    constexpr int FS = QPL * kQStride;
    const int tid = (int)threadIdx.x, nthreads = (int)blockDim.x;
    const int d4 = d >> 2;
    const int total = kWave * QPL * d4;
    const int64_t rows_left = nq - q0;
    for (int e0 = tid; e0 < total; e0 += kStageUnroll * nthreads) {
        float4 r[kStageUnroll];
        int rq[kStageUnroll], rf[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int e = e0 + u * nthreads;
            const int qq = e / d4;
            rq[u] = qq;
            rf[u] = e - qq * d4;
            r[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (e < total && qq < rows_left)
                r[u] = reinterpret_cast<const float4*>(Q + (q0 + qq) * d)[rf[u]];
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            if (e0 + u * nthreads < total) {
                float* dst = qt + 4 * rf[u] * FS + (rq[u] >> 6) * kQStride + (rq[u] & (kWave - 1));
                dst[0] = r[u].x;
                dst[FS] = r[u].y;
                dst[2 * FS] = r[u].z;
                dst[3 * FS] = r[u].w;
            }
        }
    }
}

// acc[h][i] = projection of query q0 + 64 h + lane on row r0 + i (rows at
// or past rend give 0) for this wave's RPW rows; the workgroup stages the
// query tile in proj_smem (every wave calls this; it ends with the tile
// still being read, so a caller that reuses proj_smem waits first)
template <int RPW, bool CHUNKED, int QPL>
__device__ __forceinline__ void project_accumulate(const float* __restrict__ Q, int64_t nq, int32_t d,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col, const float* __restrict__ val,
                                                   int32_t r0, int32_t rend, int64_t q0, float* proj_smem,
                                                   float (&acc)[QPL][RPW]) {
    static_assert(QPL == 1 || !CHUNKED, "two queries per lane only with the whole tile in LDS");
    const int lane = lane_id();
    const int nrows = rend;
    int len[RPW];
    int colr[RPW];
    float valr[RPW];
    int kb[RPW];                         // first entry of the current chunk, per row
    int maxlen = 0, minlen = kWave;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        len[i] = 0;
        colr[i] = 0;
        valr[i] = 0.0f;
        kb[i] = 0;
        if (r0 + i < nrows) {
            const int b = uniform(rowptr[r0 + i]);
            len[i] = uniform(rowptr[r0 + i + 1]) - b;
            if (lane < len[i]) {
                colr[i] = col[b + lane];
                valr[i] = val[b + lane];
            }
            maxlen = len[i] > maxlen ? len[i] : maxlen;
        }
        minlen = len[i] < minlen ? len[i] : minlen;
    }
#pragma unroll
    for (int h = 0; h < QPL; ++h)
#pragma unroll
        for (int i = 0; i < RPW; ++i) acc[h][i] = 0.0f;
    if constexpr (!CHUNKED) {
        // the whole tile fits: one staging, entries in order; lane l holds
        // queries q0 + l and q0 + 64 + l (QPL = 2), which share every
        // nonzero taken from the row registers
        constexpr int FS = QPL * kQStride;
        if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0) {
            stage_tile_v4<QPL>(Q, q0, nq, d, proj_smem);
        } else {
#pragma unroll
            for (int h = 0; h < QPL; ++h)
                stage_query_chunk(Q, q0 + h * kWave, nq, d, 0, d, proj_smem + h * kQStride, FS);
        }
        __syncthreads();
        // entries every row has: no branch, so the LDS reads of all rows
        // issue together; then the rows' remaining entries
        int k = 0;
        for (; k < minlen; ++k) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int c = read_lane_i(colr[i], k);
                const float v = read_lane_f(valr[i], k);
#pragma unroll
                for (int h = 0; h < QPL; ++h)
                    acc[h][i] = __builtin_fmaf(proj_smem[c * FS + h * kQStride + lane], v, acc[h][i]);
            }
        }
        for (; k < maxlen; ++k) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                if (k < len[i]) {
                    const int c = read_lane_i(colr[i], k);
                    const float v = read_lane_f(valr[i], k);
#pragma unroll
                    for (int h = 0; h < QPL; ++h)
                        acc[h][i] = __builtin_fmaf(proj_smem[c * FS + h * kQStride + lane], v, acc[h][i]);
                }
            }
        }
    } else
    for (int c0 = 0; c0 < d; c0 += kProjChunk) {
        const int cw = d - c0 < kProjChunk ? d - c0 : kProjChunk;
        if (c0 > 0) __syncthreads();     // every wave is done with the previous chunk
        stage_query_chunk(Q, q0, nq, d, c0, cw, proj_smem);
        __syncthreads();
        // entries of row i in this chunk: [kb[i], ke[i]), a prefix count of
        // the entries below the chunk's end
        int ke[RPW];
        int span = 0, common = kWave;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            ke[i] = (int)__popcll(__builtin_amdgcn_ballot_w64(lane < len[i] && colr[i] < c0 + cw));
            span = ke[i] - kb[i] > span ? ke[i] - kb[i] : span;
            common = ke[i] - kb[i] < common ? ke[i] - kb[i] : common;
        }
        int k = 0;
        for (; k < common; ++k) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int c = read_lane_i(colr[i], kb[i] + k);
                const float v = read_lane_f(valr[i], kb[i] + k);
                acc[0][i] = __builtin_fmaf(proj_smem[(c - c0) * kQStride + lane], v, acc[0][i]);
            }
        }
        for (; k < span; ++k) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                if (kb[i] + k < ke[i]) {
                    const int c = read_lane_i(colr[i], kb[i] + k);
                    const float v = read_lane_f(valr[i], kb[i] + k);
                    acc[0][i] = __builtin_fmaf(proj_smem[(c - c0) * kQStride + lane], v, acc[0][i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) kb[i] = ke[i];
    }
}

// As project_accumulate for vectors of any length: a row's entries are
// taken 64 at a time into the registers (lane e holds entry kb + e), in
// ascending feature order, so every chain is the same as with the whole row
// in registers.  A window of a feature chunk holds the row's next entries
// below the chunk's end (a ballot counts them); a row with 64 such entries
// may have more, so the windows of a chunk repeat until no row fills one.
template <int RPW, bool CHUNKED, int QPL>
__device__ __forceinline__ void project_accumulate_long(const float* __restrict__ Q, int64_t nq, int32_t d,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const float* __restrict__ val, int32_t r0, int32_t rend,
                                                        int64_t q0, float* proj_smem, float (&acc)[QPL][RPW]) {
    static_assert(QPL == 1 || !CHUNKED, "two queries per lane only with the whole tile in LDS");
    constexpr int FS = CHUNKED ? kQStride : QPL * kQStride;
    const int lane = lane_id();
    int rb[RPW], rlen[RPW], kb[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        rb[i] = 0;
        rlen[i] = 0;
        kb[i] = 0;
        if (r0 + i < rend) {
            rb[i] = uniform(rowptr[r0 + i]);
            rlen[i] = uniform(rowptr[r0 + i + 1]) - rb[i];
        }
#pragma unroll
        for (int h = 0; h < QPL; ++h) acc[h][i] = 0.0f;
    }
    const int cstep = CHUNKED ? kProjChunk : d;
    for (int c0 = 0; c0 < d; c0 += cstep) {
        const int cw = d - c0 < cstep ? d - c0 : cstep;
        if (c0 > 0) __syncthreads();     // every wave is done with the previous chunk
        if constexpr (CHUNKED) {
            stage_query_chunk(Q, q0, nq, d, c0, cw, proj_smem);
        } else if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0) {
            stage_tile_v4<QPL>(Q, q0, nq, d, proj_smem);
        } else {
#pragma unroll
            for (int h = 0; h < QPL; ++h)
                stage_query_chunk(Q, q0 + h * kWave, nq, d, 0, d, proj_smem + h * kQStride, FS);
        }
        __syncthreads();
        for (;;) {
            int colr[RPW], cnt[RPW];
            float valr[RPW];
            int span = 0, common = kWave;
            bool full = false;
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int e = kb[i] + lane;
                const bool in = e < rlen[i];
                colr[i] = in ? col[rb[i] + e] : 0;
                valr[i] = in ? val[rb[i] + e] : 0.0f;
                cnt[i] = (int)__popcll(__builtin_amdgcn_ballot_w64(in && colr[i] < c0 + cw));
                span = cnt[i] > span ? cnt[i] : span;
                common = cnt[i] < common ? cnt[i] : common;
                full = full || cnt[i] == kWave;
            }
            int k = 0;
            for (; k < common; ++k) {
#pragma unroll
                for (int i = 0; i < RPW; ++i) {
                    const int c = read_lane_i(colr[i], k);
                    const float v = read_lane_f(valr[i], k);
#pragma unroll
                    for (int h = 0; h < QPL; ++h)
                        acc[h][i] = __builtin_fmaf(proj_smem[(c - c0) * FS + h * kQStride + lane], v, acc[h][i]);
                }
            }
            for (; k < span; ++k) {
#pragma unroll
                for (int i = 0; i < RPW; ++i) {
                    if (k < cnt[i]) {
                        const int c = read_lane_i(colr[i], k);
                        const float v = read_lane_f(valr[i], k);
#pragma unroll
                        for (int h = 0; h < QPL; ++h)
                            acc[h][i] = __builtin_fmaf(proj_smem[(c - c0) * FS + h * kQStride + lane], v,
                                                       acc[h][i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < RPW; ++i) kb[i] += cnt[i];
            if (!full) break;
        }
    }
}

template <int RPW, bool CHUNKED, int QPL, bool LONG>
__device__ __forceinline__ void project_body(const float* __restrict__ Q, int64_t nq, int32_t d,
                                             const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                             const float* __restrict__ val, int32_t nrows, float* __restrict__ Pq,
                                             float* proj_smem, const int64_t bx, const int32_t by) {
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t q0 = bx * (kWave * QPL);
    const int r0 = uniform(by * (kProjWaves * RPW) + w * RPW);
    float acc[QPL][RPW];
    if constexpr (LONG) project_accumulate_long<RPW, CHUNKED, QPL>(Q, nq, d, rowptr, col, val, r0, nrows, q0, proj_smem, acc);
    else project_accumulate<RPW, CHUNKED, QPL>(Q, nq, d, rowptr, col, val, r0, nrows, q0, proj_smem, acc);
#pragma unroll
    for (int h = 0; h < QPL; ++h) {
        const int64_t q = q0 + h * kWave + lane;
        if (q < nq) {
#pragma unroll
            for (int i = 0; i < RPW; ++i)
                if (r0 + i < nrows) Pq[(int64_t)(r0 + i) * nq + q] = acc[h][i];
        }
    }
}

// Projection and descent in one kernel (Sec. II-C, Alg. 3): workgroup
// (x, y) takes the query tile x (64 * QPL queries) and the trees
// y * G .. y * G + G - 1, G = floor(8 * RPW / depth), i.e. their G * depth
// projection rows, one RPW-row group per wave.  The projections go to LDS
// (over the query tile, once every wave is done with it) instead of to
// memory, and each thread then walks (tree, query) pairs of the group, three
// descents interleaved, reading the split tables from memory.  Same
// arithmetic as the two-kernel form: every projection is the same chain in
// ascending feature order and the walk the same comparisons.
// trees per workgroup of the fused form: as many whole trees as the eight
// waves' RPW-row groups hold (all trees when there is no level)
__host__ __device__ constexpr int route_group_trees(int rpw, int depth, int T) {
    return depth > 0 ? kProjWaves * rpw / depth : T;
}

template <int RPW, bool CHUNKED, int QPL, int MAXL, bool LONG>
__device__ __forceinline__ void project_route_body(const float* __restrict__ Q, int64_t nq, int32_t d,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col, const float* __restrict__ val,
                                                   const float* __restrict__ splits, int32_t T, int32_t depth,
                                                   int32_t* __restrict__ leaf, float* proj_smem, int64_t bx,
                                                   int32_t by) {
    constexpr int TQ = kWave * QPL;
    const int G = route_group_trees(RPW, depth, T);
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t q0 = bx * TQ;
    const int t0 = by * G;
    const int ng = T - t0 < G ? T - t0 : G;
    const int row_begin = t0 * depth, row_end = (t0 + ng) * depth;
    const int r0 = uniform(row_begin + w * RPW);
    float acc[QPL][RPW];
    if constexpr (LONG) project_accumulate_long<RPW, CHUNKED, QPL>(Q, nq, d, rowptr, col, val, r0, row_end, q0, proj_smem, acc);
    else project_accumulate<RPW, CHUNKED, QPL>(Q, nq, d, rowptr, col, val, r0, row_end, q0, proj_smem, acc);
    __syncthreads();                          // every wave is done with the query tile
#pragma unroll
    for (int h = 0; h < QPL; ++h)
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            if (r0 + i < row_end) proj_smem[(r0 + i - row_begin) * TQ + h * kWave + lane] = acc[h][i];
    __syncthreads();
    const int nsplit = (1 << depth) - 1;
    const int pairs = ng * TQ;
    constexpr int kChains = 3;
    for (int base = (int)threadIdx.x; base < pairs; base += kChains * kProjWaves * kWave) {
        int node[kChains], g[kChains], qi[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int i = base + c * kProjWaves * kWave;
            g[c] = i < pairs ? i / TQ : 0;
            qi[c] = i < pairs ? i - g[c] * TQ : 0;
            node[c] = 0;
        }
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < depth) {
#pragma unroll
                for (int c = 0; c < kChains; ++c) {
                    const float sp = splits[(int64_t)(t0 + g[c]) * nsplit + node[c]];
                    const float p = proj_smem[(g[c] * depth + j) * TQ + qi[c]];
                    node[c] = (p <= sp) ? 2 * node[c] + 1 : 2 * node[c] + 2;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int i = base + c * kProjWaves * kWave;
            const int64_t q = q0 + qi[c];
            if (i < pairs && q < nq) leaf[q * T + t0 + g[c]] = node[c] - nsplit;
        }
    }
}

template <int RPW, bool CHUNKED, int QPL, int MAXL, bool LONG>
__global__ __launch_bounds__(kProjWaves * kWave) void project_route_kernel(
    const float* __restrict__ Q, int64_t nq, int32_t d, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const float* __restrict__ val, const float* __restrict__ splits, int32_t T,
    int32_t depth, int32_t* __restrict__ leaf, int64_t nbx, int32_t nby) {
    extern __shared__ float proj_smem[];   // query tile, then [G * depth][64 * QPL] projections
    int64_t tile;
    int32_t grp;
    xcd_tile_group(blockIdx.x, nbx, nby, tile, grp);
    project_route_body<RPW, CHUNKED, QPL, MAXL, LONG>(Q, nq, d, rowptr, col, val, splits, T, depth, leaf, proj_smem,
                                                      tile, grp);
}

template <int RPW, bool CHUNKED, int QPL, bool LONG>
__global__ __launch_bounds__(kProjWaves * kWave) void project_kernel(const float* __restrict__ Q, int64_t nq,
                                                                     int32_t d, const int32_t* __restrict__ rowptr,
                                                                     const int32_t* __restrict__ col,
                                                                     const float* __restrict__ val, int32_t nrows,
                                                                     float* __restrict__ Pq, int64_t nbx, int32_t nby) {
    extern __shared__ float proj_smem[];   // [min(d, kProjChunk)][QPL][65]
    int64_t tile;
    int32_t grp;
    xcd_tile_group(blockIdx.x, nbx, nby, tile, grp);
    project_body<RPW, CHUNKED, QPL, LONG>(Q, nq, d, rowptr, col, val, nrows, Pq, proj_smem, tile, grp);
}

// the item of a multi-index launch that holds workgroup b (items ascending
// by their first workgroup)
__device__ __forceinline__ int32_t find_route_item(const RouteItem* __restrict__ items, int32_t nitems, int64_t b) {
    int32_t lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// projection and descent of several query calls in one launch: workgroup b
// is workgroup b - blk0 of its item's own grid, in the XCD order above
template <int RPW, bool CHUNKED, int QPL, int MAXL>
__global__ __launch_bounds__(kProjWaves * kWave) void project_route_multi_kernel(const RouteItem* __restrict__ items,
                                                                                 int32_t nitems) {
    extern __shared__ float proj_smem[];
    const int32_t i = find_route_item(items, nitems, blockIdx.x);
    const RouteItem& it = items[i];
    int64_t tile;
    int32_t grp;
    xcd_tile_group((int64_t)blockIdx.x - it.blk0, it.nbx, it.nby, tile, grp);
    project_route_body<RPW, CHUNKED, QPL, MAXL, false>(it.Q, it.nq, it.d, it.rowptr, it.col, it.val, it.splits, it.T,
                                                it.depth, it.leaf, proj_smem, tile, grp);
}

}  // namespace

int lds_per_block_limit() {
    static int limit = -1;
    if (limit < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        limit = v;
    }
    return limit;
}

namespace {

constexpr int kProjRows = 16;     // rows per wave in project_kernel
// at most this d, a lane of a large batch takes two queries: the tile
// (128 queries, 66.5 KB at d = 128) still leaves room for two workgroups
// per CU, and each nonzero read out of the row registers serves both
constexpr int kProjPairMaxD = 128;

}  // namespace

hipError_t launch_project(const mrpt_index* ix, const float* A, int64_t m, int32_t row0, int32_t nrows, float* P,
                          hipStream_t s, int32_t rows_per_wave) {
    if (m == 0 || nrows == 0) return hipSuccess;
    const int d = ix->d;
    const int64_t tiles = (m + kWave - 1) / kWave;
    // a small batch gets 4 rows per wave: four times the waves, each with a
    // shorter serial chain (the per-row arithmetic is the same)
    const bool small = rows_per_wave == 4 ||
                       (rows_per_wave != kProjRows &&
                        tiles * ((nrows + kProjWaves * kProjRows - 1) / (kProjWaves * kProjRows)) < 512);
#define MRPT_PROJ_K(RPW, CH, QPL, LG)                                                                          \
    do {                                                                                                      \
        const size_t lds = (size_t)std::min(d, kProjChunk) * kQStride * 4 * (QPL);                           \
        const int64_t nbx = (m + kWave * (QPL) - 1) / (kWave * (QPL));                                        \
        if (nbx > kMaxGrid) return hipErrorInvalidConfiguration;                                              \
        /* row groups per launch: the one-dimensional grid within the dispatch limit */                       \
        const int32_t step = (int32_t)std::min<int64_t>(kMaxGrid / nbx, INT32_MAX / (kProjWaves * (RPW))) *   \
                             (kProjWaves * (RPW));                                                            \
        (void)hipFuncSetAttribute((const void*)project_kernel<RPW, CH, QPL, LG>,                              \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                      \
        for (int32_t c0 = 0; c0 < nrows; c0 += step) {                                                        \
            const int32_t rows_c = std::min(step, nrows - c0);                                                \
            const int32_t nby = (rows_c + kProjWaves * (RPW) - 1) / (kProjWaves * (RPW));                     \
            hipLaunchKernelGGL((project_kernel<RPW, CH, QPL, LG>), dim3((unsigned)(nbx * nby)),                \
                               dim3(kProjWaves * kWave), lds, s, A, m, d, ix->rowptr + row0 + c0, ix->col,     \
                               ix->val, rows_c, P + (int64_t)c0 * m, nbx, nby);                               \
        }                                                                                                     \
    } while (0)
#define MRPT_PROJ(RPW, CH, QPL)                     \
    do {                                            \
        if (long_rows) MRPT_PROJ_K(RPW, CH, 1, true); \
        else MRPT_PROJ_K(RPW, CH, QPL, false);      \
    } while (0)
    const bool chunked = d > kProjChunk;
    const bool long_rows = ix->max_row_nnz > kWave;
    if (small) {
        if (chunked) MRPT_PROJ(4, true, 1);
        else MRPT_PROJ(4, false, 1);
    } else {
        if (chunked) MRPT_PROJ(kProjRows, true, 1);
        else if (d <= kProjPairMaxD) MRPT_PROJ(kProjRows, false, 2);
        else MRPT_PROJ(kProjRows, false, 1);
    }
#undef MRPT_PROJ
#undef MRPT_PROJ_K
    return hipGetLastError();
}

namespace {

// projection and descent in one launch of project_route_kernel (vectors of
// more than 64 nonzeros: the windowed form, one query per lane)
hipError_t launch_route_fused(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf, hipStream_t s,
                              const LaunchCfg& cfg) {
    const int depth = ix->depth;
    static_assert(kMaxDepth <= kProjWaves * 4, "a workgroup of 4-row waves holds one tree's rows");
    // small batches take 4 rows per wave (more, shorter workgroups), large
    // ones 16, with two queries per lane when d <= 128
    const int d = ix->d;
    const int64_t tiles64 = (nq + kWave - 1) / kWave;
    const int g16 = route_group_trees(kProjRows, depth, ix->T);
    const bool small = cfg.proj_rows == 4 ||
                       (cfg.proj_rows != kProjRows && tiles64 * ((ix->T + g16 - 1) / g16) < 512);
    const bool chunked = d > kProjChunk;
    const bool long_rows = ix->max_row_nnz > kWave;
#define MRPT_PR_K(RPW, CH, QPL, ML, LG)                                                                          \
    do {                                                                                                        \
        const int G = route_group_trees(RPW, depth, ix->T);                                                     \
        const size_t tile_b = (size_t)std::min(d, kProjChunk) * kQStride * 4 * (QPL);                           \
        const size_t proj_b = (size_t)G * depth * kWave * (QPL) * 4;                                            \
        const size_t lds = std::max(tile_b, proj_b);                                                            \
        const int32_t nby = (ix->T + G - 1) / G;                                                                \
        /* queries per launch: the one-dimensional grid within the dispatch limit */                            \
        const int64_t step = (kMaxGrid / nby) * kWave * (QPL);                                                  \
        (void)hipFuncSetAttribute((const void*)project_route_kernel<RPW, CH, QPL, ML, LG>,                      \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                        \
        for (int64_t q0 = 0; q0 < nq; q0 += step) {                                                             \
            const int64_t nq_c = std::min(step, nq - q0);                                                       \
            const int64_t nbx = (nq_c + kWave * (QPL) - 1) / (kWave * (QPL));                                   \
            hipLaunchKernelGGL((project_route_kernel<RPW, CH, QPL, ML, LG>), dim3((unsigned)(nbx * nby)),        \
                               dim3(kProjWaves * kWave), lds, s, Q + q0 * d, nq_c, d, ix->rowptr, ix->col,       \
                               ix->val, ix->splits, ix->T, depth, leaf + q0 * ix->T, nbx, nby);                 \
        }                                                                                                       \
    } while (0)
#define MRPT_PR_D(RPW, CH, QPL, LG)                         \
    do {                                                    \
        if (depth <= 8) MRPT_PR_K(RPW, CH, QPL, 8, LG);     \
        else if (depth <= 12) MRPT_PR_K(RPW, CH, QPL, 12, LG); \
        else if (depth <= 16) MRPT_PR_K(RPW, CH, QPL, 16, LG); \
        else MRPT_PR_K(RPW, CH, QPL, 24, LG);               \
    } while (0)
#define MRPT_PR(RPW, CH, QPL)                           \
    do {                                                \
        if (long_rows) MRPT_PR_D(RPW, CH, 1, true);     \
        else MRPT_PR_D(RPW, CH, QPL, false);            \
    } while (0)
    if (small) {
        if (chunked) MRPT_PR(4, true, 1);
        else MRPT_PR(4, false, 1);
    } else {
        if (chunked) MRPT_PR(kProjRows, true, 1);
        else if (d <= kProjPairMaxD) MRPT_PR(kProjRows, false, 2);
        else MRPT_PR(kProjRows, false, 1);
    }
#undef MRPT_PR
#undef MRPT_PR_D
#undef MRPT_PR_K
    return hipGetLastError();
}

}  // namespace

hipError_t launch_route(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf, hipStream_t s,
                        const LaunchCfg& cfg) {
    if (nq == 0) return hipSuccess;
    return launch_route_fused(ix, Q, nq, leaf, s, cfg);
}

// Routing forms: 100 * projection class + depth class.  Projection class
// 0: d <= 128 (two queries per lane in large launches), 1: the whole tile in
// LDS, 2: chunked tiles.  Depth class 0..3: walks of up to 8, 12, 16, 24
// levels.
constexpr int32_t encode_route_form(int pc, int dc) { return 100 * pc + dc; }
constexpr bool route_forms_decode() {
    for (int pc = 0; pc < 3; ++pc)
        for (int dc = 0; dc < 4; ++dc) {
            const int32_t f = encode_route_form(pc, dc);
            if (f / 100 != pc || f % 100 != dc) return false;
        }
    return true;
}
static_assert(route_forms_decode(), "every routing form decodes to its classes");

int32_t route_form(const mrpt_index* ix) {
    if (ix->max_row_nnz > kWave) return -1;
    const int d = ix->d, depth = ix->depth;
    const int pc = d <= kProjPairMaxD ? 0 : d <= kProjChunk ? 1 : 2;
    const int dc = depth <= 8 ? 0 : depth <= 12 ? 1 : depth <= 16 ? 2 : 3;
    return encode_route_form(pc, dc);
}

// the most levels of a routing form's depth class
static int form_max_depth(int32_t form) {
    const int dc = form % 100;
    return dc == 0 ? 8 : dc == 1 ? 12 : dc == 2 ? 16 : 24;
}

void route_shape(int32_t form, int64_t total_tiles, int32_t rows_per_wave, int32_t* rpw, int32_t* qpl) {
    const int pc = form / 100;
    const bool small = rows_per_wave == 4 || (rows_per_wave != kProjRows && total_tiles < 512);
    *rpw = small ? 4 : kProjRows;
    *qpl = (!small && pc == 0) ? 2 : 1;
}

bool route_form_holds(int32_t form, const mrpt_index* ix) {
    return route_form(ix) == form && ix->depth <= form_max_depth(form);
}

RouteGrid route_grid(const mrpt_index* ix, int64_t nq, int32_t rpw, int32_t qpl) {
    RouteGrid g;
    g.rpw = rpw;
    g.qpl = qpl;
    const int G = route_group_trees(rpw, ix->depth, ix->T);
    g.nbx = (nq + kWave * qpl - 1) / (kWave * qpl);
    g.nby = (ix->T + G - 1) / G;
    return g;
}

hipError_t launch_route_multi(int32_t form, int32_t rpw, int32_t qpl, int32_t max_d, const RouteItem* items,
                              int32_t nitems, int64_t blocks, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (blocks > kMaxGrid) return hipErrorInvalidConfiguration;
    const int pc = form / 100, dc = form % 100;
    if (pc > 2 || dc > 3) return hipErrorInvalidValue;
    const bool chunked = pc == 2;
    // LDS: the largest query tile of the class, or the most projections a
    // workgroup keeps (8 * RPW rows of 64 * QPL queries)
#define MRPT_PRM_K(RPW, CH, QPL, ML)                                                                            \
    do {                                                                                                       \
        const size_t lds = std::max((size_t)std::min(max_d, kProjChunk) * kQStride * 4 * (QPL),                \
                                    (size_t)kProjWaves * (RPW) * kWave * (QPL) * 4);                           \
        (void)hipFuncSetAttribute((const void*)project_route_multi_kernel<RPW, CH, QPL, ML>,                   \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                       \
        hipLaunchKernelGGL((project_route_multi_kernel<RPW, CH, QPL, ML>), dim3((unsigned)blocks),             \
                           dim3(kProjWaves * kWave), lds, s, items, nitems);                                   \
    } while (0)
#define MRPT_PRM(RPW, CH, QPL)                             \
    do {                                                   \
        if (dc == 0) MRPT_PRM_K(RPW, CH, QPL, 8);          \
        else if (dc == 1) MRPT_PRM_K(RPW, CH, QPL, 12);    \
        else if (dc == 2) MRPT_PRM_K(RPW, CH, QPL, 16);    \
        else MRPT_PRM_K(RPW, CH, QPL, 24);                 \
    } while (0)
    if (rpw == 4) {
        if (chunked) MRPT_PRM(4, true, 1);
        else MRPT_PRM(4, false, 1);
    } else {
        if (chunked) MRPT_PRM(kProjRows, true, 1);
        else if (qpl == 2) MRPT_PRM(kProjRows, false, 2);
        else MRPT_PRM(kProjRows, false, 1);
    }
#undef MRPT_PRM
#undef MRPT_PRM_K
    return hipGetLastError();
}

}  // namespace mrpt
