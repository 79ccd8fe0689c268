// Query-path kernels for gfx950 (wave64).
//
//   route     : sparse projection of a query tile (Sec. II-C: one vector per
//               level, so the T*depth projections of a query are one sparse
//               product) fused with the descent of Alg. 3 (q^T r <= split goes
//               left, Sec. III); split tables staged in LDS.
//   vote      : F(x; q) = number of trees whose leaf holds both x and q, and
//               S = {x : F >= v} (Sec. III-A, Alg. 4), with packed 8-bit
//               counters in LDS over id ranges; a point joins S at the moment
//               its counter reaches v, as in Alg. 4.
//   dist_fp32 : knn(q, k, S) of Alg. 4: gather of the candidate rows, float32
//               squared Euclidean distance (Sec. I-A), wave-level top-k under
//               the order (distance, id), merge across waves.
//   dist_bf16 : bfloat16 prefilter over S, float32 rerank of the best r*k,
//               float64 recheck of the candidates at the k-th boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mrpt_internal.h"

namespace mrpt {
namespace {

constexpr int kWave = 64;
constexpr int32_t kPadId = 0x7F000000;  // ids of empty top-k slots (distance +inf)

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float read_lane_f(float x, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}
__device__ __forceinline__ int read_lane_i(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

// strict order on (distance, id)
__device__ __forceinline__ bool key_less(float da, int32_t ia, float db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

// ---------------------------------------------------------------------------
// Sorted list of the best 64*R (distance, id) pairs held by one wave: entry
// e = lane*R + r lives in register r of that lane.  insert() places a
// wave-uniform candidate at its rank and shifts the tail by one slot.
// ---------------------------------------------------------------------------
template <int R>
struct WaveTopK {
    float d[R];
    int32_t id[R];

    __device__ void init(int32_t pad_base) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            d[r] = INFINITY;
            id[r] = pad_base + lane_id() * R + r;
        }
    }

    // value of entry e (wave-uniform e)
    __device__ void get(int e, float& od, int32_t& oi) const {
        const int rr = e % R, ln = e / R;
        float vd = d[0];
        int32_t vi = id[0];
#pragma unroll
        for (int r = 1; r < R; ++r)
            if (r == rr) { vd = d[r]; vi = id[r]; }
        od = read_lane_f(vd, ln);
        oi = read_lane_i(vi, ln);
    }

    __device__ void insert(float cd, int32_t ci) {
        int pos = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) pos += __popcll(__ballot(key_less(d[r], id[r], cd, ci)));
        const float up_d = __shfl_up(d[R - 1], 1);
        const int32_t up_i = __shfl_up(id[R - 1], 1);
        const int e0 = lane_id() * R;
#pragma unroll
        for (int r = R - 1; r >= 0; --r) {
            const int e = e0 + r;
            const float pd = (r > 0) ? d[r > 0 ? r - 1 : 0] : up_d;
            const int32_t pi = (r > 0) ? id[r > 0 ? r - 1 : 0] : up_i;
            if (e == pos) { d[r] = cd; id[r] = ci; }
            else if (e > pos) { d[r] = pd; id[r] = pi; }
        }
    }

    // write entries [0, cnt) to LDS arrays
    __device__ void store(float* sd, int32_t* si, int cnt) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = lane_id() * R + r;
            if (e < cnt) { sd[e] = d[r]; si[e] = id[r]; }
        }
    }
};

// number of entries of the sorted LDS list (sd, si)[0, cnt) that are < key
__device__ __forceinline__ int count_less(const float* sd, const int32_t* si, int cnt, float kd,
                                          int32_t ki) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key_less(sd[mid], si[mid], kd, ki)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// route: one wave per tree, lanes = 64 queries of a tile; the query tile is
// staged through LDS in feature blocks ([feature][query], padded), the CSR
// rows of the wave's tree are read with scalar loads, every projection is a
// float32 fused multiply-add chain in ascending feature order from +0.
// ---------------------------------------------------------------------------
constexpr int kRouteFB = 32;          // features per staged block
constexpr int kRouteLdsQ = kRouteFB * 65;

template <int MAXL>
__global__ __launch_bounds__(256) void route_kernel(const float* __restrict__ Q, int64_t nq, int32_t d,
                                                    const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const float* __restrict__ splits, int32_t T,
                                                    int32_t depth, int32_t trees_per_block,
                                                    int32_t splits_in_lds, int32_t* __restrict__ leaf) {
    extern __shared__ float route_smem[];
    float* qt = route_smem;                 // [kRouteFB][65]
    float* sp = route_smem + kRouteLdsQ;    // [trees_per_block][nsplit]
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t q0 = (int64_t)blockIdx.x * kWave;
    const int t = uniform((int)blockIdx.y * trees_per_block + w);
    const bool tree_ok = t < T;
    const int nsplit = (1 << depth) - 1;
    const int nthreads = (int)blockDim.x;

    if (splits_in_lds) {
        for (int i = (int)threadIdx.x; i < trees_per_block * nsplit; i += nthreads) {
            const int tw = i / nsplit;
            const int tt = (int)blockIdx.y * trees_per_block + tw;
            sp[i] = tt < T ? splits[(int64_t)tt * nsplit + (i - tw * nsplit)] : 0.0f;
        }
    }

    float acc[MAXL];
    int ptr[MAXL], end[MAXL];
#pragma unroll
    for (int j = 0; j < MAXL; ++j) {
        acc[j] = 0.0f;
        ptr[j] = 0;
        end[j] = 0;
        if (j < depth && tree_ok) {
            ptr[j] = uniform(rowptr[(int64_t)t * depth + j]);
            end[j] = uniform(rowptr[(int64_t)t * depth + j + 1]);
        }
    }

    for (int fb = 0; fb < d; fb += kRouteFB) {
        __syncthreads();
        for (int i = (int)threadIdx.x; i < kWave * kRouteFB; i += nthreads) {
            const int qq = i / kRouteFB, f = i - qq * kRouteFB;
            const int64_t gq = q0 + qq;
            const int gf = fb + f;
            qt[f * 65 + qq] = (gq < nq && gf < d) ? Q[gq * d + gf] : 0.0f;
        }
        __syncthreads();
        const int fe = fb + kRouteFB;
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < depth) {
                int p = ptr[j];
                const int e = end[j];
                float a = acc[j];
                while (p < e) {
                    const int c = col[p];
                    if (c >= fe) break;
                    a = __builtin_fmaf(qt[(c - fb) * 65 + lane], val[p], a);
                    ++p;
                }
                acc[j] = a;
                ptr[j] = p;
            }
        }
    }

    const int64_t q = q0 + lane;
    if (tree_ok && q < nq) {
        int node = 0;
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < depth) {
                const float s = splits_in_lds ? sp[w * nsplit + node] : splits[(int64_t)t * nsplit + node];
                node = (acc[j] <= s) ? 2 * node + 1 : 2 * node + 2;
            }
        }
        leaf[q * T + t] = node - nsplit;
    }
}

// ---------------------------------------------------------------------------
// vote: one workgroup per query.  The T leaf lists (each ascending by id) are
// flattened; thread i keeps entries i, i+B, i+2B, ... in registers (the rest,
// if any, is re-read per pass).  For each range of kVoteChunk ids the packed
// 8-bit LDS counters are cleared and every entry in range is counted with an
// LDS atomic; the thread that moves a counter from v-1 to v appends the id to
// S (wave-aggregated slot reservation).
// ---------------------------------------------------------------------------
constexpr int kVoteBlock = 512;
constexpr int kVoteRegs = 48;

__device__ __forceinline__ void vote_one(int32_t id, int64_t lo, int64_t hi, uint32_t* cnt, int v,
                                         int* nsel, int32_t* out, int64_t cap) {
    bool elect = false;
    if (id >= lo && id < hi) {
        const uint32_t rel = (uint32_t)(id - lo);
        const uint32_t sh = (rel & 3u) * 8u;
        const uint32_t old = atomicAdd(&cnt[rel >> 2], 1u << sh);
        elect = (int)((old >> sh) & 0xffu) + 1 == v;
    }
    const uint64_t m = __ballot(elect);
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(nsel, __popcll(m));
        base = __shfl(base, leader);
        if (elect) {
            const int64_t p = (int64_t)base + __popcll(m & __lanemask_lt());
            if (p < cap) out[p] = id;
        }
    }
}

__global__ __launch_bounds__(kVoteBlock) void vote_kernel(const int32_t* __restrict__ leaf,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t n,
                                                          int32_t T, int32_t v, int32_t chunk,
                                                          int32_t* __restrict__ s_ids, int64_t cap,
                                                          int32_t* __restrict__ s_count) {
    extern __shared__ uint32_t vote_cnt[];   // chunk/4 words
    __shared__ int64_t base[kMaxT];
    __shared__ int32_t pre[kMaxT + 1];
    __shared__ int nsel;
    const int tid = (int)threadIdx.x;
    const int64_t q = blockIdx.x;

    if (tid < T) {
        const int L = leaf[q * T + tid];
        const int b = off[L];
        base[tid] = (int64_t)tid * n + b;
        pre[tid + 1] = off[L + 1] - b;
    }
    if (tid == 0) { pre[0] = 0; nsel = 0; }
    __syncthreads();
    if (tid < kWave) {  // inclusive scan of pre[1..T] by wave 0, 4 entries per lane
        int v4[4], s = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = 1 + tid * 4 + i;
            v4[i] = idx <= T ? pre[idx] : 0;
            s += v4[i];
        }
        int incl = s;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (tid >= o) incl += y;
        }
        int run = incl - s;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = 1 + tid * 4 + i;
            run += v4[i];
            if (idx <= T) pre[idx] = run;
        }
    }
    __syncthreads();
    const int total = pre[T];

    int32_t* out = s_ids + q * cap;
    int32_t ids[kVoteRegs];
#pragma unroll
    for (int r = 0; r < kVoteRegs; ++r) {
        const int f = tid + r * kVoteBlock;
        ids[r] = -1;
        if (f < total) {
            int lo = 0, hi = T;  // largest t with pre[t] <= f
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[mid] <= f) lo = mid; else hi = mid;
            }
            ids[r] = perm[base[lo] + (f - pre[lo])];
        }
    }

    const int words = chunk >> 2;
    for (int64_t lo = 0; lo < n; lo += chunk) {
        const int64_t hi = lo + chunk < n ? lo + chunk : n;
        uint4* c4 = reinterpret_cast<uint4*>(vote_cnt);
        for (int i = tid; i < (words >> 2); i += kVoteBlock) c4[i] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kVoteRegs; ++r) vote_one(ids[r], lo, hi, vote_cnt, v, &nsel, out, cap);
        for (int fb = kVoteRegs * kVoteBlock; fb < total; fb += kVoteBlock) {
            const int f = fb + tid;
            int32_t id = -1;
            if (f < total) {
                int a = 0, b = T;
                while (b - a > 1) {
                    const int mid = (a + b) >> 1;
                    if (pre[mid] <= f) a = mid; else b = mid;
                }
                id = perm[base[a] + (f - pre[a])];
            }
            vote_one(id, lo, hi, vote_cnt, v, &nsel, out, cap);
        }
        __syncthreads();
    }
    if (tid == 0) s_count[q] = nsel < cap ? nsel : (int32_t)cap;
}

// debug: F(x; q) of every listed candidate, by binary search of x in each of
// the query's T leaf lists (independent of the counting kernel)
__global__ __launch_bounds__(256) void vote_counts_kernel(const int32_t* __restrict__ leaf,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t n,
                                                          int32_t T, const int32_t* __restrict__ s_ids,
                                                          int64_t cap, const int32_t* __restrict__ s_count,
                                                          uint8_t* __restrict__ s_votes) {
    const int64_t q = blockIdx.x;
    const int ns = s_count[q];
    for (int i = (int)threadIdx.x; i < ns; i += (int)blockDim.x) {
        const int32_t x = s_ids[q * cap + i];
        int F = 0;
        for (int t = 0; t < T; ++t) {
            const int L = leaf[q * T + t];
            const int32_t* lst = perm + (int64_t)t * n;
            int lo = off[L], hi = off[L + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (lst[mid] < x) lo = mid + 1; else hi = mid;
            }
            F += (lo < off[L + 1] && lst[lo] == x) ? 1 : 0;
        }
        s_votes[q * cap + i] = (uint8_t)F;
    }
}

// ---------------------------------------------------------------------------
// dist_fp32: one workgroup (4 waves) per query.  A group of G lanes holds a
// candidate row as NV float4 per lane; G = 32 for d = 128 (two rows per wave
// per load), U rows per group are in flight.  Each group's squared distance
// (direct differences, per-lane fused accumulation, butterfly reduction) is
// offered to the wave's sorted top-k list; the 4 lists are merged by rank.
// ---------------------------------------------------------------------------
constexpr int kDistWaves = 4;

template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

template <int G, int NV, int R>
__global__ __launch_bounds__(256) void dist_fp32_kernel(const float* __restrict__ X, int32_t d,
                                                        const float* __restrict__ Q,
                                                        const int32_t* __restrict__ s_ids, int64_t cap,
                                                        const int32_t* __restrict__ s_count, int32_t k,
                                                        int32_t* __restrict__ out_idx,
                                                        float* __restrict__ out_dist) {
    constexpr int GPW = kWave / G;
    constexpr int U = (GPW * NV >= 4) ? 4 : (8 / (GPW * NV) > 0 ? 8 / (GPW * NV) : 1);
    __shared__ float md[kDistWaves][kWave * R];
    __shared__ int32_t mi[kDistWaves][kWave * R];
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int g = lane / G, gl = lane - g * G;
    const int64_t q = blockIdx.x;
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
    for (int b0 = 0; b0 < ns; b0 += kStep) {
        int32_t cid[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ci = b0 + (u * kDistWaves + w) * GPW + g;
            cid[u] = ci < ns ? S[ci] : -1;
        }
        float4 xv[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float4* xr = reinterpret_cast<const float4*>(X + (int64_t)(cid[u] < 0 ? 0 : cid[u]) * d);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int vi = gl + i * G;
                xv[u][i] = (cid[u] >= 0 && vi < nvec) ? xr[vi] : qv[i];
            }
        }
        float s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float a = 0.0f;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const float dx = qv[i].x - xv[u][i].x, dy = qv[i].y - xv[u][i].y;
                const float dz = qv[i].z - xv[u][i].z, dw = qv[i].w - xv[u][i].w;
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
// dist_bf16: phase 1 ranks S by ||q||^2 - 2 q.x~ + ||x~||^2 with x~ the
// bfloat16 row (8 values per lane per 16-byte load, float32 accumulation) and
// keeps the best kp = r*k; phase 2 recomputes those kp with float32 direct
// differences from the float32 rows and orders them by (distance, id);
// phase 3 recomputes in float64 every candidate whose float32 distance is
// within recheck_rel of the k-th and orders that window by (float64 distance,
// id).  One workgroup (4 waves) per query.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

template <int GB, int NVB, int RB>
__global__ __launch_bounds__(256) void dist_bf16_kernel(const float* __restrict__ X,
                                                        const uint16_t* __restrict__ Xb,
                                                        const float* __restrict__ xnorm, int32_t d,
                                                        const float* __restrict__ Q,
                                                        const int32_t* __restrict__ s_ids, int64_t cap,
                                                        const int32_t* __restrict__ s_count, int32_t k,
                                                        int32_t kp, float recheck_rel,
                                                        int32_t* __restrict__ out_idx,
                                                        float* __restrict__ out_dist) {
    constexpr int GPW = kWave / GB;
    constexpr int U = (GPW * NVB >= 4) ? 4 : (8 / (GPW * NVB) > 0 ? 8 / (GPW * NVB) : 1);
    __shared__ float md[kDistWaves][kWave * RB];
    __shared__ int32_t mi[kDistWaves][kWave * RB];
    __shared__ int32_t cand[kMaxRerank];      // phase-1 survivors in prefilter rank order
    __shared__ float d32[kMaxRerank];         // their float32 squared distances
    __shared__ double d64[kMaxRerank];        // float64 squared distances (window only)
    __shared__ int32_t order[kMaxRerank];     // rank by (d32, id) -> candidate slot
    __shared__ int32_t final_slot[kMaxK];
    __shared__ int win_lo, win_hi;
    __shared__ float qs[1024 + 64];           // query (float32) for phases 2-3 when d <= 1024

    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int g = lane / GB, gl = lane - g * GB;
    const int64_t q = blockIdx.x;
    const int ns = uniform(s_count[q]);
    const int32_t* S = s_ids + q * cap;
    const int nv8 = d >> 3;
    const float* qrow = Q + q * d;

    for (int i = (int)threadIdx.x; i < d; i += (int)blockDim.x) qs[i] = qrow[i];

    // query slice (8 floats per 16-byte bf16 slot) and ||q||^2
    float qf[NVB][8];
    float qn_part = 0.0f;
#pragma unroll
    for (int i = 0; i < NVB; ++i) {
        const int vi = gl + i * GB;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            qf[i][j] = vi < nv8 ? qrow[vi * 8 + j] : 0.0f;
            qn_part = __builtin_fmaf(qf[i][j], qf[i][j], qn_part);
        }
    }
    const float qn = read_lane_f(group_sum<GB>(qn_part), 0);

    WaveTopK<RB> top;
    top.init(kPadId + w * kWave * RB);
    float tau_d;
    int32_t tau_i;
    top.get(kp - 1, tau_d, tau_i);

    constexpr int kStep = kDistWaves * GPW * U;
    for (int b0 = 0; b0 < ns; b0 += kStep) {
        int32_t cid[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ci = b0 + (u * kDistWaves + w) * GPW + g;
            cid[u] = ci < ns ? S[ci] : -1;
        }
        uint4 xv[U][NVB];
        float xn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = cid[u] < 0 ? 0 : cid[u];
            const uint4* xr = reinterpret_cast<const uint4*>(Xb + row * d);
#pragma unroll
            for (int i = 0; i < NVB; ++i) {
                const int vi = gl + i * GB;
                xv[u][i] = (cid[u] >= 0 && vi < nv8) ? xr[vi] : make_uint4(0u, 0u, 0u, 0u);
            }
            xn[u] = xnorm[row];
        }
        float s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float a = 0.0f;
#pragma unroll
            for (int i = 0; i < NVB; ++i) {
                const uint32_t wv[4] = {xv[u][i].x, xv[u][i].y, xv[u][i].z, xv[u][i].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a = __builtin_fmaf(qf[i][2 * j], bf16_lo(wv[j]), a);
                    a = __builtin_fmaf(qf[i][2 * j + 1], bf16_hi(wv[j]), a);
                }
            }
            const float dot = group_sum<GB>(a);
            s[u] = (qn + xn[u]) - 2.0f * dot;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int gg = 0; gg < GPW; ++gg) {
                const int32_t ci = read_lane_i(cid[u], gg * GB);
                const float cd = read_lane_f(s[u], gg * GB);
                if (ci >= 0 && key_less(cd, ci, tau_d, tau_i)) {
                    top.insert(cd, ci);
                    top.get(kp - 1, tau_d, tau_i);
                }
            }
        }
    }

    // merge the wave lists: the best kp of the prefilter, in rank order
    top.store(md[w], mi[w], kp);
    __syncthreads();
    for (int e = (int)threadIdx.x; e < kDistWaves * kp; e += (int)blockDim.x) {
        const int ww = e / kp, pos = e - ww * kp;
        const float kd = md[ww][pos];
        const int32_t ki = mi[ww][pos];
        int rank = pos;
        for (int o = 0; o < kDistWaves; ++o)
            if (o != ww) rank += count_less(md[o], mi[o], kp, kd, ki);
        if (rank < kp) cand[rank] = kd < INFINITY ? ki : -1;
    }
    __syncthreads();

    // phase 2: float32 direct distances of the survivors, one wave per candidate
    for (int c = w; c < kp; c += kDistWaves) {
        const int32_t id = uniform(cand[c]);
        float r = INFINITY;
        if (id >= 0) {
            const float* xr = X + (int64_t)id * d;
            float a = 0.0f;
            for (int i = lane; i < d; i += kWave) {
                const float df = qs[i] - xr[i];
                a = __builtin_fmaf(df, df, a);
            }
            r = read_lane_f(group_sum<kWave>(a), 0);
        }
        if (lane == 0) d32[c] = r;
    }
    __syncthreads();
    // order by (d32, id); empty slots (id -1, +inf) go last in slot order
    for (int c = (int)threadIdx.x; c < kp; c += (int)blockDim.x) {
        const float kd = d32[c];
        const int32_t ki = cand[c] < 0 ? kPadId + c : cand[c];
        int rank = 0;
        for (int o = 0; o < kp; ++o) {
            const int32_t oi = cand[o] < 0 ? kPadId + o : cand[o];
            rank += key_less(d32[o], oi, kd, ki) ? 1 : 0;
        }
        order[rank] = c;
    }
    __syncthreads();
    // phase 3: float64 recheck of the window around the k-th float32 distance
    if (threadIdx.x == 0) {
        const int kk = k < kp ? k : kp;
        const float dk2 = d32[order[kk - 1]];
        int lo = kk, hi = kk;
        if (dk2 < INFINITY) {
            const float dk = sqrtf(dk2);
            const float tol = recheck_rel * dk;
            lo = kk - 1;
            while (lo > 0 && fabsf(sqrtf(d32[order[lo - 1]]) - dk) <= tol) --lo;
            hi = kk;
            while (hi < kp && d32[order[hi]] < INFINITY && fabsf(sqrtf(d32[order[hi]]) - dk) <= tol) ++hi;
        }
        win_lo = lo;
        win_hi = hi;
    }
    __syncthreads();
    const int wlo = win_lo, whi = win_hi;
    for (int r = wlo + w; r < whi; r += kDistWaves) {
        const int c = uniform(order[r]);
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
    for (int r = (int)threadIdx.x; r < k; r += (int)blockDim.x) {
        if (r < wlo || r >= whi) {
            final_slot[r] = r < kp ? order[r] : -1;
        }
    }
    for (int r = wlo + (int)threadIdx.x; r < whi; r += (int)blockDim.x) {
        const int c = order[r];
        const double kd = d64[c];
        const int32_t ki = cand[c];
        int rank = wlo;
        for (int o = wlo; o < whi; ++o) {
            const int oc = order[o];
            rank += (d64[oc] < kd || (d64[oc] == kd && cand[oc] < ki)) ? 1 : 0;
        }
        if (rank < k) final_slot[rank] = -2 - c;  // marks a rechecked slot
    }
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

__global__ void copy_counts_kernel(const int32_t* __restrict__ src, int64_t nq, int32_t* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) dst[i] = src[i];
}

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

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_route(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const int nsplit = (1 << ix->depth) - 1;
    const int base_lds = kRouteLdsQ * (int)sizeof(float);
    const int limit = lds_per_block_limit();
    int tpb = 4;
    int splits_in_lds = 1;
    while (tpb > 1 && base_lds + tpb * nsplit * (int)sizeof(float) > limit) --tpb;
    if (base_lds + tpb * nsplit * (int)sizeof(float) > limit) { splits_in_lds = 0; tpb = 4; }
    tpb = tpb < ix->T ? tpb : ix->T;
    const size_t lds = (size_t)base_lds + (splits_in_lds ? (size_t)tpb * nsplit * sizeof(float) : 0);
    dim3 grid((unsigned)((nq + kWave - 1) / kWave), (unsigned)((ix->T + tpb - 1) / tpb));
    dim3 block(kWave * tpb);
#define MRPT_ROUTE(ML)                                                                          \
    hipLaunchKernelGGL(route_kernel<ML>, grid, block, lds, s, Q, nq, ix->d, ix->rowptr, ix->col, \
                       ix->val, ix->splits, ix->T, ix->depth, tpb, splits_in_lds, leaf)
    if (ix->depth <= 8) MRPT_ROUTE(8);
    else if (ix->depth <= 12) MRPT_ROUTE(12);
    else if (ix->depth <= 16) MRPT_ROUTE(16);
    else MRPT_ROUTE(24);
#undef MRPT_ROUTE
    return hipGetLastError();
}

hipError_t launch_vote(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                       int64_t cap, int32_t* s_count, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const size_t lds = (size_t)ix->id_chunk;
    hipLaunchKernelGGL(vote_kernel, dim3((unsigned)nq), dim3(kVoteBlock), lds, s, leaf, ix->perm, ix->off,
                       ix->n, ix->T, v, ix->id_chunk, s_ids, cap, s_count);
    return hipGetLastError();
}

hipError_t launch_vote_counts(const mrpt_index* ix, const int32_t* leaf, int64_t nq, const int32_t* s_ids,
                              int64_t cap, const int32_t* s_count, uint8_t* s_votes, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(vote_counts_kernel, dim3((unsigned)nq), dim3(256), 0, s, leaf, ix->perm, ix->off, ix->n,
                       ix->T, s_ids, cap, s_count, s_votes);
    return hipGetLastError();
}

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

hipError_t launch_dist_bf16(const mrpt_index* ix, const float* Q, int64_t nq, const int32_t* s_ids, int64_t cap,
                            const int32_t* s_count, int32_t k, int32_t rerank, float recheck_rel,
                            int32_t* out_idx, float* out_dist, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const int d = ix->d;
    const int kp = k * rerank;
    const int RB = kp <= 64 ? 1 : kp <= 128 ? 2 : kp <= 256 ? 4 : 8;
    dim3 grid((unsigned)nq), block(256);
#define MRPT_BF(GB, NVB, RR)                                                                              \
    hipLaunchKernelGGL((dist_bf16_kernel<GB, NVB, RR>), grid, block, 0, s, ix->X, ix->Xb, ix->xnorm, d, Q, \
                       s_ids, cap, s_count, k, kp, recheck_rel, out_idx, out_dist)
#define MRPT_BF_R(GB, NVB)                 \
    switch (RB) {                          \
        case 1: MRPT_BF(GB, NVB, 1); break; \
        case 2: MRPT_BF(GB, NVB, 2); break; \
        case 4: MRPT_BF(GB, NVB, 4); break; \
        default: MRPT_BF(GB, NVB, 8); break; \
    }
    const int nv8 = d / 8;
    if (nv8 <= 16) { MRPT_BF_R(16, 1); }
    else if (nv8 <= 32) { MRPT_BF_R(32, 1); }
    else if (nv8 <= 64) { MRPT_BF_R(64, 1); }
    else { MRPT_BF_R(64, 2); }
#undef MRPT_BF_R
#undef MRPT_BF
    return hipGetLastError();
}

hipError_t launch_copy_counts(const int32_t* src, int64_t nq, int32_t* dst, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_counts_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, src, nq, dst);
    return hipGetLastError();
}

}  // namespace mrpt
