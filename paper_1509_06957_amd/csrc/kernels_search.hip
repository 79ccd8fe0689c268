// Exact-search kernels: knn(q, k, S) of Alg. 4 over the candidate set of
// each query.
//
//   dist_fp32 : gather of the candidate rows, float32 squared Euclidean
//               distance (Sec. I-A) by direct differences, wave-level top-k
//               under the order (distance, id), merge of the wave lists.
//   dist_bf16 : bfloat16 prefilter over S, float32 rerank of the best r*k,
//               float64 recheck of the candidates at the k-th boundary.
#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// dist_fp32: one workgroup (4 waves) per query.  A group of G lanes holds a
// candidate row as NV float4 per lane; G = 32 for d = 128 (two rows per wave
// per load).  Each step a wave gathers U rows per group (16 float4 per
// lane, 16 KB per wave in flight at four waves per SIMD; 8 at seven waves
// was 2 % slower) while the candidate ids of the next step are already
// loading; every load is issued unconditionally (clamped addresses,
// masked afterwards), so the compiler can count them in flight.  Each group's
// squared distance (direct differences, per-lane fused accumulation,
// butterfly reduction) is offered to the wave's sorted top-k list; the 4
// lists are merged by rank.
// ---------------------------------------------------------------------------
constexpr int kDistWaves = 4;

// Selection of the best candidates of a query: up to kPfChunk candidates are
// scored at a time into LDS, and a block-wide radix select over them and the
// list kept so far keeps the best ones under (score, id).
constexpr int kPfChunk = 1024;                  // candidates scored per selection round
constexpr int kPfBuf = kPfChunk + kMaxRerank;   // prefilter: one round's scores, then the list kept so far

// monotone map of a float32 score to an unsigned key: -0 as +0, NaN after
// every number (a NaN score comes from a non-finite query and ranks last)
__device__ __forceinline__ uint32_t score_key(float s) {
    uint32_t u = __builtin_bit_cast(uint32_t, s);
    if ((u << 1) == 0u) u = 0u;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0u) return 0xFFFFFFFFu;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// wave 0 of a select pass: the bucket of hist[0..255] that holds the rem-th
// smallest of the counted pairs; sel = {bucket, rank within it, its count}
__device__ __forceinline__ void pick_bucket(const uint32_t* hist, int rem, int* sel) {
    const int lane = lane_id();
    const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const int own = (int)(h0 + h1 + h2 + h3);
    int incl = own;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int excl = incl - own;
    if (excl < rem && rem <= incl) {
        const uint32_t h[4] = {h0, h1, h2, h3};
        int c = excl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (c < rem && rem <= c + (int)h[j]) {
                sel[0] = 4 * lane + j;
                sel[1] = rem - c;
                sel[2] = (int)h[j];
            }
            c += (int)h[j];
        }
    }
}

// The pair (T, idT) of rank need (1-based) among the tot pairs (key[e],
// id[e]) under (key, id), ids distinct, 1 <= need <= tot: a radix select over
// the key's bytes from the top finds T and how many pairs at T rank up to
// need; when that is not all of them, a second radix select over the ids of
// the pairs at T finds idT (else idT = 0xFFFFFFFF: every pair at T is within
// the rank).  The pairs of rank <= need are those with key < T, or key == T
// and id <= idT.  All 256 threads of the workgroup take part.
__device__ void block_threshold(const uint32_t* key, const int32_t* id, int tot, int need, uint32_t* hist, int* sel,
                                uint32_t& T, uint32_t& idT) {
    const int tid = (int)threadIdx.x;
    const int w = tid >> 6;
    uint32_t prefix = 0u, pmask = 0u;
    int rem = need, eq = tot;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0u;
        __syncthreads();
        for (int e = tid; e < tot; e += 256) {
            const uint32_t kk = key[e];
            if ((kk & pmask) == prefix) atomicAdd(&hist[(kk >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (w == 0) pick_bucket(hist, rem, sel);
        __syncthreads();
        prefix |= (uint32_t)sel[0] << shift;
        pmask |= 0xFFu << shift;
        rem = sel[1];
        eq = sel[2];
    }
    T = prefix;
    idT = 0xFFFFFFFFu;
    if (rem < eq) {
        uint32_t ip = 0u, im = 0u;
        for (int shift = 24; shift >= 0; shift -= 8) {
            hist[tid] = 0u;
            __syncthreads();
            for (int e = tid; e < tot; e += 256) {
                const uint32_t ii = (uint32_t)id[e];
                if (key[e] == T && (ii & im) == ip) atomicAdd(&hist[(ii >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (w == 0) pick_bucket(hist, rem, sel);
            __syncthreads();
            ip |= (uint32_t)sel[0] << shift;
            im |= 0xFFu << shift;
            rem = sel[1];
        }
        idT = ip;
    }
}

// The need smallest of the tot pairs (key[e], id[e]) under (key, id), ids
// distinct, need < tot, written to (okey, oid)[0, need) in no particular
// order (block_threshold, then one compaction).
__device__ void block_select(const uint32_t* key, const int32_t* id, int tot, int need, uint32_t* okey,
                             int32_t* oid, uint32_t* hist, int* sel) {
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    uint32_t T, idT;
    block_threshold(key, id, tot, need, hist, sel, T, idT);
    if (tid == 0) sel[3] = 0;
    __syncthreads();
    for (int e0 = 0; e0 < tot; e0 += 256) {      // uniform trip count
        const int e = e0 + tid;
        bool take = false;
        uint32_t kk = 0u;
        int32_t ii = 0;
        if (e < tot) {
            kk = key[e];
            ii = id[e];
            take = kk < T || (kk == T && (uint32_t)ii <= idT);
        }
        const uint64_t m = __ballot(take);
        int base = 0;
        if (lane == 0 && m) base = atomicAdd(&sel[3], __popcll(m));
        base = __shfl(base, 0);
        if (take) {
            const int p = base + __popcll(m & __lanemask_lt());
            okey[p] = kk;
            oid[p] = ii;
        }
    }
    __syncthreads();
}

// append this thread's index e to the LDS list (out, *count) when take
__device__ __forceinline__ void block_append(bool take, int e, int32_t* out, int* count) {
    const uint64_t m = __ballot(take);
    int base = 0;
    if (lane_id() == 0 && m) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, 0);
    if (take) out[base + __popcll(m & __lanemask_lt())] = e;
}

template <int G, int NV, int R>
__device__ __forceinline__ void dist_fp32_body(const float* __restrict__ X, int32_t d, const float* __restrict__ Q,
                                               const int32_t* __restrict__ s_ids, int64_t cap,
                                               const int32_t* __restrict__ s_count, int32_t k,
                                               int32_t* __restrict__ out_idx, float* __restrict__ out_dist,
                                               const int64_t q) {
    constexpr int GPW = kWave / G;
    constexpr int U = 16 / NV > 0 ? 16 / NV : 1;
    __shared__ float md[kDistWaves][kWave * R];
    __shared__ int32_t mi[kDistWaves][kWave * R];
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int g = lane / G, gl = lane - g * G;
    const int ns = uniform(s_count[q]);
    const int32_t* S = s_ids + q * cap;
    const int nvec = d >> 2;

    float4 qv[NV];
    const float4* qrow = reinterpret_cast<const float4*>(Q + q * d);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int vi = gl + i * G;
        qv[i] = vi < nvec ? qrow[vi] : make_float4(0.f, 0.f, 0.f, 0.f);
    }

    WaveTopK<R> top;
    top.init(kPadId + w * kWave * R);
    float tau_d;
    int32_t tau_i;
    top.get(k - 1, tau_d, tau_i);

    constexpr int kStep = kDistWaves * GPW * U;
    // candidate slot of (step base b, row u) for this group; ids past ns read
    // slot 0 (any in-range slot) and are marked -1 after the load
    auto slot = [&](int b, int u) { return b + (u * kDistWaves + w) * GPW + g; };
    int32_t craw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int ci = slot(0, u);
        craw[u] = S[ci < ns ? ci : 0];
    }
    for (int b0 = 0; b0 < ns; b0 += kStep) {
        int32_t cid[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cid[u] = slot(b0, u) < ns ? craw[u] : -1;
        float4 xv[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float4* xr = reinterpret_cast<const float4*>(X + (int64_t)(cid[u] < 0 ? 0 : cid[u]) * d);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int vi = gl + i * G;
                xv[u][i] = xr[vi < nvec ? vi : 0];
            }
        }
        // ids of the next step, in flight while this step's rows arrive
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ci = slot(b0 + kStep, u);
            craw[u] = S[ci < ns ? ci : 0];
        }
        float s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float a = 0.0f;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const bool in = gl + i * G < nvec;
                const float4 x = xv[u][i];
                const float dx = in ? qv[i].x - x.x : 0.f, dy = in ? qv[i].y - x.y : 0.f;
                const float dz = in ? qv[i].z - x.z : 0.f, dw = in ? qv[i].w - x.w : 0.f;
                a = __builtin_fmaf(dx, dx, a);
                a = __builtin_fmaf(dy, dy, a);
                a = __builtin_fmaf(dz, dz, a);
                a = __builtin_fmaf(dw, dw, a);
            }
            s[u] = group_sum<G>(a);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int gg = 0; gg < GPW; ++gg) {
                const int32_t ci = read_lane_i(cid[u], gg * G);
                const float cd = read_lane_f(s[u], gg * G);
                if (ci >= 0 && key_less(cd, ci, tau_d, tau_i)) {
                    top.insert(cd, ci);
                    top.get(k - 1, tau_d, tau_i);
                }
            }
        }
    }

    top.store(md[w], mi[w], k);
    __syncthreads();
    for (int e = (int)threadIdx.x; e < kDistWaves * k; e += (int)blockDim.x) {
        const int ww = e / k, pos = e - ww * k;
        const float kd = md[ww][pos];
        const int32_t ki = mi[ww][pos];
        int rank = pos;
#pragma unroll
        for (int o = 0; o < kDistWaves; ++o)
            if (o != ww) rank += count_less(md[o], mi[o], k, kd, ki);
        if (rank < k) {
            const bool real = kd < INFINITY;
            out_idx[q * k + rank] = real ? ki : -1;
            out_dist[q * k + rank] = real ? sqrtf(kd) : INFINITY;
        }
    }
}

template <int G, int NV, int R>
__global__ __launch_bounds__(256) void dist_fp32_kernel(const float* __restrict__ X, int32_t d,
                                                        const float* __restrict__ Q,
                                                        const int32_t* __restrict__ s_ids, int64_t cap,
                                                        const int32_t* __restrict__ s_count, int32_t k,
                                                        int32_t* __restrict__ out_idx,
                                                        float* __restrict__ out_dist) {
    dist_fp32_body<G, NV, R>(X, d, Q, s_ids, cap, s_count, k, out_idx, out_dist, blockIdx.x);
}

// the item of a multi-index launch that holds workgroup b: items are in
// ascending order of their first workgroup (binary search, scalar loads)
__device__ __forceinline__ int32_t find_item(const SearchItem* __restrict__ items, int32_t nitems, int64_t b) {
    int32_t lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].row0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// one launch over the queries of several query calls of the same kernel form
// (indexes of one d, k in one register class): workgroup b serves query
// b - row0 of the item that holds it
template <int G, int NV, int R>
__global__ __launch_bounds__(256) void dist_fp32_multi_kernel(const SearchItem* __restrict__ items, int32_t nitems,
                                                              int32_t d) {
    const int32_t i = find_item(items, nitems, blockIdx.x);
    const SearchItem& it = items[i];
    dist_fp32_body<G, NV, R>(it.X, d, it.Q, it.s_ids, it.cap, it.s_count, it.k, it.out_idx, it.out_dist,
                             (int64_t)blockIdx.x - it.row0);
}

// generic fallback (any d): scalar loads, one wave per candidate row
template <int R>
__global__ __launch_bounds__(256) void dist_fp32_generic_kernel(const float* __restrict__ X, int32_t d,
                                                                const float* __restrict__ Q,
                                                                const int32_t* __restrict__ s_ids,
                                                                int64_t cap,
                                                                const int32_t* __restrict__ s_count,
                                                                int32_t k, int32_t* __restrict__ out_idx,
                                                                float* __restrict__ out_dist) {
    __shared__ float md[kDistWaves][kWave * R];
    __shared__ int32_t mi[kDistWaves][kWave * R];
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t q = blockIdx.x;
    const int ns = uniform(s_count[q]);
    const int32_t* S = s_ids + q * cap;
    const float* gq = Q + q * d;
    WaveTopK<R> top;
    top.init(kPadId + w * kWave * R);
    float tau_d;
    int32_t tau_i;
    top.get(k - 1, tau_d, tau_i);
    for (int c = w; c < ns; c += kDistWaves) {
        const int32_t id = uniform(S[c]);
        const float* xr = X + (int64_t)id * d;
        float a = 0.0f;
        for (int i = lane; i < d; i += kWave) {
            const float df = gq[i] - xr[i];
            a = __builtin_fmaf(df, df, a);
        }
        const float cd = read_lane_f(group_sum<kWave>(a), 0);
        if (key_less(cd, id, tau_d, tau_i)) {
            top.insert(cd, id);
            top.get(k - 1, tau_d, tau_i);
        }
    }
    top.store(md[w], mi[w], k);
    __syncthreads();
    for (int e = (int)threadIdx.x; e < kDistWaves * k; e += (int)blockDim.x) {
        const int ww = e / k, pos = e - ww * k;
        const float kd = md[ww][pos];
        const int32_t ki = mi[ww][pos];
        int rank = pos;
        for (int o = 0; o < kDistWaves; ++o)
            if (o != ww) rank += count_less(md[o], mi[o], k, kd, ki);
        if (rank < k) {
            const bool real = kd < INFINITY;
            out_idx[q * k + rank] = real ? ki : -1;
            out_dist[q * k + rank] = real ? sqrtf(kd) : INFINITY;
        }
    }
}

// ---------------------------------------------------------------------------
// dist_prefilter (bf16 and fp8 arms): phase 1 ranks S by
// ||q||^2 - 2 q.x~ + ||x~||^2 with x~ the low-precision row (bfloat16: 8
// values per 16-byte load; fp8 e4m3: 16 values per load and a per-row scale,
// x~ = scale * decode(code)), float32 accumulation, and keeps the best
// kp = r*k under (score, id): the scores of up to kPfChunk candidates at a
// time go to LDS, and a block-wide radix select over them and the list kept
// so far takes the kp smallest; phase 2 recomputes those kp with float32
// direct differences from the float32 rows and orders them by (distance,
// id); phase 3 recomputes in float64 every candidate whose float32 distance
// is within recheck_rel of the k-th and orders that window by (float64
// distance, id).  One workgroup (4 waves) per query.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

constexpr int kFmtBf16 = 0;
constexpr int kFmtFp8 = 1;

// KEEP: stop after phase 1 and write the kept list (ids in prefilter rank
// order, -1 past min(|S|, kp); S in slot order when |S| <= kp) to
// keep_out[q * kp ...] instead of the k-NN (the parity hook of the arm)
template <int FMT, int GB, int NVB, int G2, int NV2, bool KEEP = false>
__device__ __forceinline__ void dist_prefilter_body(const float* __restrict__ X, const uint8_t* __restrict__ Xq,
                                                    const float2* __restrict__ sn8, int32_t d,
                                                    const float* __restrict__ Q,
                                                    const int32_t* __restrict__ s_ids, int64_t cap,
                                                    const int32_t* __restrict__ s_count, int32_t k, int32_t kp,
                                                    float recheck_rel, int32_t* __restrict__ out_idx,
                                                    float* __restrict__ out_dist, const int64_t q,
                                                    int32_t* __restrict__ keep_out = nullptr) {
    constexpr int GPW = kWave / GB;
    // rows per group in flight: 8 / NVB, but 4 for the fp8 rows of d <= 128
    // (eight lanes per row), whose kernel then runs at six waves per SIMD
    // (8 rows at five waves: 3 % slower)
    constexpr int U = (FMT == kFmtFp8 && GB == 8 && NVB == 1) ? 4 : 8 / NVB;
    constexpr int EPU = FMT == kFmtBf16 ? 8 : 16;      // row values per 16-byte load
    constexpr int ROWB = FMT == kFmtBf16 ? 2 : 1;       // bytes per row value
    // phase 2 reads float32 rows as the fp32 kernel does: G2 lanes x NV2 float4
    constexpr int GPW2 = kWave / G2;
    constexpr int U2 = 8 / NV2;
    static_assert(kPfChunk % (kDistWaves * (kWave / GB) * U) == 0, "a round covers whole steps");
    // phase 1 (round scores and the kept list) and phases 2-3 (distances,
    // order, final slots) use the same LDS
    __shared__ __align__(16) unsigned char pf_smem[kPfBuf * 8];
    uint32_t* pkey = reinterpret_cast<uint32_t*>(pf_smem);             // kPfBuf keys
    int32_t* pid = reinterpret_cast<int32_t*>(pf_smem + kPfBuf * 4);   // kPfBuf ids
    double* d64 = reinterpret_cast<double*>(pf_smem);                  // float64 squared distances (window only)
    float* d32 = reinterpret_cast<float*>(pf_smem + kMaxRerank * 8);   // float32 squared distances of the kept
    int32_t* order = reinterpret_cast<int32_t*>(pf_smem + kMaxRerank * 12);       // rank by (d32, id) -> slot
    int32_t* final_slot = reinterpret_cast<int32_t*>(pf_smem + kMaxRerank * 16);  // k <= kp <= kMaxRerank
    static_assert(kMaxRerank * 20 <= kPfBuf * 8, "phases 2-3 fit the phase-1 buffer");
    __shared__ int32_t cand[kMaxRerank];      // the kept list (prefilter survivors)
    __shared__ uint32_t ckey[kMaxRerank];     // their score keys
    __shared__ uint32_t hist[256];
    __shared__ int sel[4];
    __shared__ int win_lo, win_hi;
    __shared__ __align__(16) float qs[1024 + 64];   // query (float32) for phases 2-3, d <= 1024

    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int g = lane / GB, gl = lane - g * GB;
    const int ns = uniform(s_count[q]);
    const int32_t* S = s_ids + q * cap;
    const int nv8 = d / EPU;                       // 16-byte loads per row
    const float* qrow = Q + q * d;

    for (int i = (int)threadIdx.x; i < d; i += (int)blockDim.x) qs[i] = qrow[i];

    // query slice (EPU floats per 16-byte load) and ||q||^2
    float qf[NVB][EPU];
    float qn_part = 0.0f;
#pragma unroll
    for (int i = 0; i < NVB; ++i) {
        const int vi = gl + i * GB;
#pragma unroll
        for (int j = 0; j < EPU; ++j) {
            qf[i][j] = vi < nv8 ? qrow[vi * EPU + j] : 0.0f;
            qn_part = __builtin_fmaf(qf[i][j], qf[i][j], qn_part);
        }
    }
    const float qn = read_lane_f(group_sum<GB>(qn_part), 0);

    if (ns > kp) {
        // as in dist_fp32: the next step's candidate ids are loaded while this
        // step's rows arrive, and every load is unconditional (clamped, masked)
        constexpr int kStep = kDistWaves * GPW * U;
        auto slot = [&](int b, int u) { return b + (u * kDistWaves + w) * GPW + g; };
        int32_t craw[U];
    #pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ci = slot(0, u);
            craw[u] = S[ci < ns ? ci : 0];
        }
        int nk = 0;                            // entries of the kept list (cand, ckey)
        for (int c0 = 0; c0 < ns; c0 += kPfChunk) {
            const int cend = ns - c0 < kPfChunk ? ns : c0 + kPfChunk;
            for (int b0 = c0; b0 < cend; b0 += kStep) {
                int32_t cid[U];
    #pragma unroll
                for (int u = 0; u < U; ++u) cid[u] = slot(b0, u) < cend ? craw[u] : -1;
                uint4 xv[U][NVB];
                float xs[U], xn[U];
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t row = cid[u] < 0 ? 0 : cid[u];
                    const uint4* xr = reinterpret_cast<const uint4*>(Xq + row * d * ROWB);
    #pragma unroll
                    for (int i = 0; i < NVB; ++i) {
                        const int vi = gl + i * GB;
                        xv[u][i] = xr[vi < nv8 ? vi : 0];
                    }
                    const float2 sn = FMT == kFmtFp8 ? sn8[row] : make_float2(1.0f, 0.0f);
                    xs[u] = sn.x;
                    xn[u] = sn.y;
                }
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int ci = slot(b0 + kStep, u);
                    craw[u] = S[ci < ns ? ci : 0];
                }
                // the dot product q.x~; the bfloat16 row's squared norm is
                // accumulated beside it from the row in registers (no norm
                // load), the fp8 row's (scale^2 * sum decode^2, stored at
                // build) comes with the scale in one 8-byte load
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    float a = 0.0f, r2 = 0.0f;
    #pragma unroll
                    for (int i = 0; i < NVB; ++i) {
                        const bool in = gl + i * GB < nv8;
                        const uint32_t wv[4] = {in ? xv[u][i].x : 0u, in ? xv[u][i].y : 0u, in ? xv[u][i].z : 0u,
                                                in ? xv[u][i].w : 0u};
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            if constexpr (FMT == kFmtBf16) {
                                const float x0 = bf16_lo(wv[j]), x1 = bf16_hi(wv[j]);
                                a = __builtin_fmaf(qf[i][2 * j], x0, a);
                                a = __builtin_fmaf(qf[i][2 * j + 1], x1, a);
                                r2 = __builtin_fmaf(x0, x0, r2);
                                r2 = __builtin_fmaf(x1, x1, r2);
                            } else {
                                const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)wv[j], false);
                                const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)wv[j], true);
                                a = __builtin_fmaf(qf[i][4 * j], lo[0], a);
                                a = __builtin_fmaf(qf[i][4 * j + 1], lo[1], a);
                                a = __builtin_fmaf(qf[i][4 * j + 2], hi[0], a);
                                a = __builtin_fmaf(qf[i][4 * j + 3], hi[1], a);
                            }
                        }
                    }
                    const float dot = group_sum<GB>(a);
                    float sc;
                    if constexpr (FMT == kFmtBf16) sc = (qn + group_sum<GB>(r2)) - 2.0f * dot;
                    else sc = (qn + xn[u]) - 2.0f * (xs[u] * dot);
                    // the group's first lane files the score under the slot
                    if (gl == 0 && cid[u] >= 0) {
                        const int e = slot(b0, u) - c0;
                        pkey[e] = score_key(sc);
                        pid[e] = cid[u];
                    }
                }
            }
            // the round's scores, then the list kept so far; keep the best kp
            const int m = cend - c0;
            __syncthreads();
            for (int j = (int)threadIdx.x; j < nk; j += (int)blockDim.x) {
                pkey[m + j] = ckey[j];
                pid[m + j] = cand[j];
            }
            __syncthreads();
            const int tot = m + nk;
            if (tot <= kp) {
                for (int j = (int)threadIdx.x; j < tot; j += (int)blockDim.x) {
                    ckey[j] = pkey[j];
                    cand[j] = pid[j];
                }
                nk = tot;
                __syncthreads();
            } else {
                block_select(pkey, pid, tot, kp, ckey, cand, hist, sel);
                nk = kp;
            }
        }
        if constexpr (KEEP) {
            // the kept list in prefilter rank order, (score, id)
            for (int c = (int)threadIdx.x; c < kp; c += (int)blockDim.x) {
                int rank = 0;
                for (int o = 0; o < kp; ++o)
                    rank += (ckey[o] < ckey[c] || (ckey[o] == ckey[c] && cand[o] < cand[c])) ? 1 : 0;
                keep_out[q * kp + rank] = cand[c];
            }
            return;
        }
    } else {
        // every candidate survives the prefilter: phase 2 takes S as it is
        // (it orders by float32 distance and id, whatever the slot order)
        for (int c = (int)threadIdx.x; c < kp; c += (int)blockDim.x) cand[c] = c < ns ? S[c] : -1;
        __syncthreads();
    }
    if constexpr (KEEP) {
        for (int c = (int)threadIdx.x; c < kp; c += (int)blockDim.x) keep_out[q * kp + c] = cand[c];
        return;
    }

    // phase 2: float32 direct distances of the survivors, gathered as in
    // dist_fp32 (same lanes per row, same summation order, U2 rows per group
    // in flight).  Slots past the kq = min(|S|, kp) survivors are empty (id
    // -1, distance +inf).
    const int kq = ns < kp ? ns : kp;
    {
        const int g2 = lane / G2, gl2 = lane - g2 * G2;
        const int nvec = d >> 2;
        float4 q2[NV2];
#pragma unroll
        for (int i = 0; i < NV2; ++i) {
            const int vi = gl2 + i * G2;
            q2[i] = vi < nvec ? reinterpret_cast<const float4*>(qs)[vi] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        constexpr int kStep2 = kDistWaves * GPW2 * U2;
        for (int c0 = 0; c0 < kq; c0 += kStep2) {
            int32_t id[U2];
#pragma unroll
            for (int u = 0; u < U2; ++u) {
                const int c = c0 + (u * kDistWaves + w) * GPW2 + g2;
                id[u] = c < kq ? cand[c] : -1;
            }
            float4 xv2[U2][NV2];
#pragma unroll
            for (int u = 0; u < U2; ++u) {
                const float4* xr = reinterpret_cast<const float4*>(X + (int64_t)(id[u] < 0 ? 0 : id[u]) * d);
#pragma unroll
                for (int i = 0; i < NV2; ++i) {
                    const int vi = gl2 + i * G2;
                    xv2[u][i] = xr[vi < nvec ? vi : 0];
                }
            }
#pragma unroll
            for (int u = 0; u < U2; ++u) {
                float a = 0.0f;
#pragma unroll
                for (int i = 0; i < NV2; ++i) {
                    const bool in = gl2 + i * G2 < nvec;
                    const float4 x = xv2[u][i];
                    const float dx = in ? q2[i].x - x.x : 0.f, dy = in ? q2[i].y - x.y : 0.f;
                    const float dz = in ? q2[i].z - x.z : 0.f, dw = in ? q2[i].w - x.w : 0.f;
                    a = __builtin_fmaf(dx, dx, a);
                    a = __builtin_fmaf(dy, dy, a);
                    a = __builtin_fmaf(dz, dz, a);
                    a = __builtin_fmaf(dw, dw, a);
                }
                const float r = group_sum<G2>(a);
                const int c = c0 + (u * kDistWaves + w) * GPW2 + g2;
                // a NaN distance (non-finite query) ranks as +inf, i.e. as an
                // empty slot: the ordering below needs keys that compare
                if (gl2 == 0 && c < kq) d32[c] = (id[u] >= 0 && !__builtin_isnan(r)) ? r : INFINITY;
            }
        }
        for (int c = kq + (int)threadIdx.x; c < kp; c += (int)blockDim.x) d32[c] = INFINITY;
    }
    __syncthreads();
    // phase 3.  The kk = min(k, kp)-th kept candidate under (d32, id) (kk = k
    // since kp >= k): when there are fewer, no recheck.  Its float32 distance
    // dk fixes the recheck window, the candidates whose float32 distance is
    // within recheck_rel * dk of dk (contiguous in the (d32, id) order); the
    // candidates below it take ranks 0.. by (d32, id), the window's then
    // follow by (d64, id) after a float64 recompute, and only ranks < k are
    // written (so only about k candidates are ranked, not all kp).
    const int kk = k < kp ? k : kp;
    float dk2 = INFINITY;
    if (kq >= kk) {
        for (int c = (int)threadIdx.x; c < kq; c += (int)blockDim.x) ckey[c] = score_key(d32[c]);
        __syncthreads();
        uint32_t T, idT;
        block_threshold(ckey, cand, kq, kk, hist, sel, T, idT);
        dk2 = T >= 0xFF800000u ? INFINITY : __builtin_bit_cast(float, T ^ 0x80000000u);
    }
    int32_t* below = order;                                             // candidates below the window
    int32_t* winl = reinterpret_cast<int32_t*>(pf_smem + kMaxRerank * 20);   // the window
    static_assert(kMaxRerank * 24 <= kPfBuf * 8, "the window list fits the phase-1 buffer");
    if (threadIdx.x == 0) { win_lo = 0; win_hi = 0; }
    __syncthreads();
    {
        const bool finite = dk2 < INFINITY;
        const float dk = finite ? sqrtf(dk2) : INFINITY;
        const float tol = finite ? recheck_rel * dk : 0.0f;
        for (int c0 = 0; c0 < kq; c0 += (int)blockDim.x) {   // uniform trip count
            const int c = c0 + (int)threadIdx.x;
            bool in_win = false, is_below = false;
            if (c < kq) {
                const float x = d32[c];
                if (finite) {
                    const float sx = sqrtf(x);
                    in_win = fabsf(sx - dk) <= tol;
                    is_below = !in_win && sx < dk;
                } else {
                    is_below = x < INFINITY;
                }
            }
            block_append(is_below, c, below, &win_lo);
            block_append(in_win, c, winl, &win_hi);
        }
    }
    __syncthreads();
    const int nb = win_lo, nw = win_hi;
    for (int i = (int)threadIdx.x; i < nb; i += (int)blockDim.x) {
        const int c = below[i];
        const float kd = d32[c];
        const int32_t ki = cand[c];
        int rank = 0;
        for (int j = 0; j < nb; ++j) rank += key_less(d32[below[j]], cand[below[j]], kd, ki) ? 1 : 0;
        if (rank < k) final_slot[rank] = c;
    }
    for (int j = w; j < nw; j += kDistWaves) {
        const int c = uniform(winl[j]);
        const int32_t id = uniform(cand[c]);
        const float* xr = X + (int64_t)id * d;
        double a = 0.0;
        for (int i = lane; i < d; i += kWave) {
            const double df = (double)qs[i] - (double)xr[i];
            a = __builtin_fma(df, df, a);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) d64[c] = a;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < nw; i += (int)blockDim.x) {
        const int c = winl[i];
        const double kd = d64[c];
        const int32_t ki = cand[c];
        int rank = nb;
        for (int j = 0; j < nw; ++j) {
            const int oc = winl[j];
            rank += (d64[oc] < kd || (d64[oc] == kd && cand[oc] < ki)) ? 1 : 0;
        }
        if (rank < k) final_slot[rank] = -2 - c;  // marks a rechecked slot
    }
    for (int r = nb + nw + (int)threadIdx.x; r < k; r += (int)blockDim.x) final_slot[r] = -1;
    __syncthreads();
    for (int r = (int)threadIdx.x; r < k; r += (int)blockDim.x) {
        const int fs = final_slot[r];
        int32_t id = -1;
        float dist = INFINITY;
        if (fs <= -2) {
            const int c = -2 - fs;
            id = cand[c];
            dist = (float)sqrt(d64[c]);
        } else if (fs >= 0 && cand[fs] >= 0 && d32[fs] < INFINITY) {
            id = cand[fs];
            dist = sqrtf(d32[fs]);
        }
        out_idx[q * k + r] = id;
        out_dist[q * k + r] = dist;
    }
}

#define MRPT_PF_PARAMS                                                                                          \
    const float *__restrict__ X, const uint8_t *__restrict__ Xq, const float2 *__restrict__ sn8, int32_t d,    \
        const float *__restrict__ Q, const int32_t *__restrict__ s_ids, int64_t cap,                           \
        const int32_t *__restrict__ s_count, int32_t k, int32_t kp, float recheck_rel,                         \
        int32_t *__restrict__ out_idx, float *__restrict__ out_dist
#define MRPT_PF_ARGS X, Xq, sn8, d, Q, s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist, blockIdx.x

template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) void dist_prefilter_kernel(MRPT_PF_PARAMS) {
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(MRPT_PF_ARGS);
}

// The same kernel held to 72 registers, for seven waves per SIMD instead of
// six.  Used where that costs no spill: bf16 rows of d <= 128 (the fp8 forms
// spill heavily under the cap).
template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void dist_prefilter_w7_kernel(
    MRPT_PF_PARAMS) {
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(MRPT_PF_ARGS);
}

// The fp8 forms of d <= 128 (four rows in flight per group) held to 80
// registers, six waves per SIMD instead of four, with no spill.
template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void dist_prefilter_w6_kernel(
    MRPT_PF_PARAMS) {
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(MRPT_PF_ARGS);
}

// phase 1 only: the kept list of every query (parity hook)
template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) void dist_prefilter_keep_kernel(MRPT_PF_PARAMS, int32_t* __restrict__ keep_out) {
    dist_prefilter_body<FMT, GB, NVB, G2, NV2, true>(MRPT_PF_ARGS, keep_out);
}

// one launch over the queries of several query calls of the same kernel form
// (indexes of one d and arm): workgroup b serves query b - row0 of its item
template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) void dist_prefilter_multi_kernel(const SearchItem* __restrict__ items,
                                                                   int32_t nitems, int32_t d, float recheck_rel) {
    const int32_t i = find_item(items, nitems, blockIdx.x);
    const SearchItem& it = items[i];
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(it.X, it.Xq, it.sn8, d, it.Q, it.s_ids, it.cap, it.s_count, it.k,
                                               it.kp, recheck_rel, it.out_idx, it.out_dist,
                                               (int64_t)blockIdx.x - it.row0);
}

template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void dist_prefilter_multi_w7_kernel(
    const SearchItem* __restrict__ items, int32_t nitems, int32_t d, float recheck_rel) {
    const int32_t i = find_item(items, nitems, blockIdx.x);
    const SearchItem& it = items[i];
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(it.X, it.Xq, it.sn8, d, it.Q, it.s_ids, it.cap, it.s_count, it.k,
                                               it.kp, recheck_rel, it.out_idx, it.out_dist,
                                               (int64_t)blockIdx.x - it.row0);
}

template <int FMT, int GB, int NVB, int G2, int NV2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void dist_prefilter_multi_w6_kernel(
    const SearchItem* __restrict__ items, int32_t nitems, int32_t d, float recheck_rel) {
    const int32_t i = find_item(items, nitems, blockIdx.x);
    const SearchItem& it = items[i];
    dist_prefilter_body<FMT, GB, NVB, G2, NV2>(it.X, it.Xq, it.sn8, d, it.Q, it.s_ids, it.cap, it.s_count, it.k,
                                               it.kp, recheck_rel, it.out_idx, it.out_dist,
                                               (int64_t)blockIdx.x - it.row0);
}

#undef MRPT_PF_ARGS
#undef MRPT_PF_PARAMS

template <int F, int GB, int NVB, int G2, int NV2>
void launch_prefilter_form(dim3 grid, hipStream_t s, const float* X, const uint8_t* Xq, const float2* sn8, int32_t d,
                           const float* Q, const int32_t* s_ids, int64_t cap, const int32_t* s_count, int32_t k,
                           int32_t kp, float recheck_rel, int32_t* out_idx, float* out_dist, int32_t* keep_out) {
    if (keep_out)
        hipLaunchKernelGGL((dist_prefilter_keep_kernel<F, GB, NVB, G2, NV2>), grid, dim3(256), 0, s, X, Xq, sn8,
                           d, Q, s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist, keep_out);
    else if constexpr (F == kFmtBf16 && GB == 16 && NVB == 1)
        hipLaunchKernelGGL((dist_prefilter_w7_kernel<F, GB, NVB, G2, NV2>), grid, dim3(256), 0, s, X, Xq, sn8, d,
                           Q, s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist);
    else if constexpr (F == kFmtFp8 && GB == 8 && NVB == 1)
        hipLaunchKernelGGL((dist_prefilter_w6_kernel<F, GB, NVB, G2, NV2>), grid, dim3(256), 0, s, X, Xq, sn8, d,
                           Q, s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist);
    else
        hipLaunchKernelGGL((dist_prefilter_kernel<F, GB, NVB, G2, NV2>), grid, dim3(256), 0, s, X, Xq, sn8, d, Q,
                           s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist);
}

}  // namespace

hipError_t launch_dist_fp32(const mrpt_index* ix, const float* Q, int64_t nq, const int32_t* s_ids, int64_t cap,
                            const int32_t* s_count, int32_t k, int32_t* out_idx, float* out_dist,
                            hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const int d = ix->d;
    const int R = k <= 64 ? 1 : k <= 128 ? 2 : k <= 256 ? 4 : k <= 512 ? 8 : 16;
    dim3 grid((unsigned)nq), block(256);
    const bool vec = (d % 4) == 0 && d <= 1024 &&
                     ((uintptr_t)Q % 16) == 0 && ((uintptr_t)ix->X % 16) == 0;
#define MRPT_DIST(G, NV, RR)                                                                      \
    hipLaunchKernelGGL((dist_fp32_kernel<G, NV, RR>), grid, block, 0, s, ix->X, d, Q, s_ids, cap, \
                       s_count, k, out_idx, out_dist)
#define MRPT_DIST_R(G, NV)                     \
    switch (R) {                               \
        case 1: MRPT_DIST(G, NV, 1); break;    \
        case 2: MRPT_DIST(G, NV, 2); break;    \
        case 4: MRPT_DIST(G, NV, 4); break;    \
        case 8: MRPT_DIST(G, NV, 8); break;    \
        default: MRPT_DIST(G, NV, 16); break;  \
    }
    if (vec) {
        const int nvec = d / 4;
        if (nvec <= 16) { MRPT_DIST_R(16, 1); }
        else if (nvec <= 32) { MRPT_DIST_R(32, 1); }
        else if (nvec <= 64) { MRPT_DIST_R(64, 1); }
        else if (nvec <= 128) { MRPT_DIST_R(64, 2); }
        else { MRPT_DIST_R(64, 4); }
    } else {
#define MRPT_DISTG(RR)                                                                                 \
    hipLaunchKernelGGL((dist_fp32_generic_kernel<RR>), grid, block, 0, s, ix->X, d, Q, s_ids, cap, s_count, \
                       k, out_idx, out_dist)
        switch (R) {
            case 1: MRPT_DISTG(1); break;
            case 2: MRPT_DISTG(2); break;
            case 4: MRPT_DISTG(4); break;
            case 8: MRPT_DISTG(8); break;
            default: MRPT_DISTG(16); break;
        }
#undef MRPT_DISTG
    }
#undef MRPT_DIST_R
#undef MRPT_DIST
    return hipGetLastError();
}

hipError_t launch_dist_prefilter(const mrpt_index* ix, int fp8, const float* Q, int64_t nq, const int32_t* s_ids,
                                 int64_t cap, const int32_t* s_count, int32_t k, int32_t rerank, float recheck_rel,
                                 int32_t* out_idx, float* out_dist, hipStream_t s, int32_t* keep_out) {
    if (nq == 0) return hipSuccess;
    const int d = ix->d;
    const int kp = k * rerank;
    dim3 grid((unsigned)nq);
    const uint8_t* Xq = fp8 ? ix->X8 : reinterpret_cast<const uint8_t*>(ix->Xb);
#define MRPT_PF(F, GB, NVB, G2, NV2)                                                                            \
    launch_prefilter_form<F, GB, NVB, G2, NV2>(grid, s, ix->X, Xq, ix->sn8, d, Q, s_ids, cap, s_count, k, kp, \
                                                   recheck_rel, out_idx, out_dist, keep_out)
#define MRPT_PF_R(F, GB, NVB, G2, NV2) MRPT_PF(F, GB, NVB, G2, NV2)
    if (!fp8) {
        // bf16 loads per row d/8; the float32 rerank layout follows from it
        const int nv8 = d / 8;
        if (nv8 <= 16) { MRPT_PF_R(kFmtBf16, 16, 1, 32, 1); }
        else if (nv8 <= 32) { MRPT_PF_R(kFmtBf16, 32, 1, 64, 1); }
        else if (nv8 <= 64) { MRPT_PF_R(kFmtBf16, 64, 1, 64, 2); }
        else { MRPT_PF_R(kFmtBf16, 64, 2, 64, 4); }
    } else {
        // fp8 loads per row d/16 (d % 16 == 0, d <= 1024); rerank as dist_fp32
        const int nv16 = d / 16, nvec = d / 4;
        if (nvec <= 16) { MRPT_PF_R(kFmtFp8, 8, 1, 16, 1); }
        else if (nvec <= 32) { MRPT_PF_R(kFmtFp8, 8, 1, 32, 1); }
        else if (nvec <= 64) { MRPT_PF_R(kFmtFp8, 16, 1, 64, 1); }
        else if (nvec <= 128) { MRPT_PF_R(kFmtFp8, 32, 1, 64, 2); }
        else { MRPT_PF_R(kFmtFp8, 64, 1, 64, 4); }
        (void)nv16;
    }
#undef MRPT_PF_R
#undef MRPT_PF
    return hipGetLastError();
}

// Search forms: fp32 vector kernels 100 + 10 * layout + register class,
// prefilter kernels 200 (bf16) / 300 (fp8) + layout; the layouts follow the
// single-call launchers above.
namespace {
int32_t fp32_layout(int d) {
    const int nvec = d / 4;
    return nvec <= 16 ? 0 : nvec <= 32 ? 1 : nvec <= 64 ? 2 : nvec <= 128 ? 3 : 4;
}
int32_t r_class(int k) { return k <= 64 ? 0 : k <= 128 ? 1 : k <= 256 ? 2 : k <= 512 ? 3 : 4; }
int32_t pf_layout(int fp8, int d) {
    if (!fp8) {
        const int nv8 = d / 8;
        return nv8 <= 16 ? 0 : nv8 <= 32 ? 1 : nv8 <= 64 ? 2 : 3;
    }
    const int nvec = d / 4;
    return nvec <= 16 ? 0 : nvec <= 32 ? 1 : nvec <= 64 ? 2 : nvec <= 128 ? 3 : 4;
}
}  // namespace

int32_t search_form(const mrpt_index* ix, int32_t precision, int32_t k, const float* Q) {
    const int d = ix->d;
    if (precision == MRPT_FP32) {
        const bool vec = (d % 4) == 0 && d <= 1024 && ((uintptr_t)Q % 16) == 0 && ((uintptr_t)ix->X % 16) == 0;
        if (!vec) return -1;
        return 100 + 10 * fp32_layout(d) + r_class(k);
    }
    return (precision == MRPT_FP8_RERANK ? 300 : 200) + pf_layout(precision == MRPT_FP8_RERANK, d);
}

hipError_t launch_search_multi(int32_t form, int32_t d, const SearchItem* items, int32_t nitems, int64_t rows,
                               float recheck_rel, hipStream_t s) {
    if (rows == 0 || nitems == 0) return hipSuccess;
    dim3 grid((unsigned)rows), block(256);
#define MRPT_D32(G, NV, RR) \
    hipLaunchKernelGGL((dist_fp32_multi_kernel<G, NV, RR>), grid, block, 0, s, items, nitems, d)
#define MRPT_D32_R(G, NV)                     \
    switch (form % 10) {                      \
        case 0: MRPT_D32(G, NV, 1); break;    \
        case 1: MRPT_D32(G, NV, 2); break;    \
        case 2: MRPT_D32(G, NV, 4); break;    \
        case 3: MRPT_D32(G, NV, 8); break;    \
        default: MRPT_D32(G, NV, 16); break;  \
    }
#define MRPT_PFM(F, GB, NVB, G2, NV2)                                                                           \
    hipLaunchKernelGGL((dist_prefilter_multi_kernel<F, GB, NVB, G2, NV2>), grid, block, 0, s, items, nitems, d, \
                       recheck_rel)
    if (form >= 100 && form < 200) {
        switch ((form - 100) / 10) {
            case 0: MRPT_D32_R(16, 1); break;
            case 1: MRPT_D32_R(32, 1); break;
            case 2: MRPT_D32_R(64, 1); break;
            case 3: MRPT_D32_R(64, 2); break;
            default: MRPT_D32_R(64, 4); break;
        }
    } else if (form >= 200 && form < 300) {
        switch (form - 200) {
            case 0:
                hipLaunchKernelGGL((dist_prefilter_multi_w7_kernel<kFmtBf16, 16, 1, 32, 1>), grid, block, 0, s,
                                   items, nitems, d, recheck_rel);
                break;
            case 1: MRPT_PFM(kFmtBf16, 32, 1, 64, 1); break;
            case 2: MRPT_PFM(kFmtBf16, 64, 1, 64, 2); break;
            default: MRPT_PFM(kFmtBf16, 64, 2, 64, 4); break;
        }
    } else if (form >= 300 && form < 400) {
        switch (form - 300) {
            case 0:
                hipLaunchKernelGGL((dist_prefilter_multi_w6_kernel<kFmtFp8, 8, 1, 16, 1>), grid, block, 0, s,
                                   items, nitems, d, recheck_rel);
                break;
            case 1:
                hipLaunchKernelGGL((dist_prefilter_multi_w6_kernel<kFmtFp8, 8, 1, 32, 1>), grid, block, 0, s,
                                   items, nitems, d, recheck_rel);
                break;
            case 2: MRPT_PFM(kFmtFp8, 16, 1, 64, 1); break;
            case 3: MRPT_PFM(kFmtFp8, 32, 1, 64, 2); break;
            default: MRPT_PFM(kFmtFp8, 64, 1, 64, 4); break;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef MRPT_PFM
#undef MRPT_D32_R
#undef MRPT_D32
    return hipGetLastError();
}

}  // namespace mrpt
