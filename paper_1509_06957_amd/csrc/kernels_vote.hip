// Vote kernels (Sec. III-A, Alg. 4): for one query, F(x; q) counts the trees
// whose leaf holds both x and q, and x joins the candidate set S when its
// count reaches v (in Alg. 4, at the moment the count becomes v).
//
// Two forms, both one workgroup of 16 waves per CU-resident query:
//
//  * single pass (when a 1-bit map of all n ids fits LDS): the first
//    occurrence of an id sets its bit; later occurrences are compacted per
//    wave and counted in an LDS hash table keyed by id.  The workgroup is
//    persistent over queries and prefetches the next query's leaf windows.
//  * multi pass (any n): packed counters of B bits per id (the smallest width
//    that holds v) over id ranges that fit LDS, one pass per range.
//
// In both, each wave owns trees w, w+16, ...; a tree's leaf list (ascending
// ids, contiguous in that tree's permutation) is read as 64-id windows into
// registers, coalesced.
#include <cstdlib>

#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

using namespace dev;

constexpr int kVoteWaves = 16;
constexpr int kVoteBlock = kVoteWaves * kWave;
constexpr int kVoteSlots = 32;      // register windows per lane

// wave-aggregated append of the ids whose `elect` is set (slot from an LDS counter)
__device__ __forceinline__ void append(bool elect, int32_t id, int* nsel, int32_t* out, int64_t cap) {
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

// ---------------------------------------------------------------------------
// multi-pass form
// ---------------------------------------------------------------------------

// one occurrence of id (rel = id - first id of the pass); true when this
// occurrence is the v-th
template <int B>
__device__ __forceinline__ bool count_id(uint32_t* cnt, uint32_t rel, int v) {
    constexpr uint32_t per = 32u / B;
    const uint32_t word = rel / per;
    const uint32_t sh = (rel % per) * B;
    if constexpr (B == 1) {
        const uint32_t bit = 1u << sh;
        if (cnt[word] & bit) return false;
        return (atomicOr(&cnt[word], bit) & bit) == 0u;
    } else if constexpr (B == 8) {
        if ((int)((cnt[word] >> sh) & 0xffu) >= v) return false;
        const uint32_t old = atomicAdd(&cnt[word], 1u << sh);
        return (int)((old >> sh) & 0xffu) + 1 == v;
    } else {
        constexpr uint32_t mask = (1u << B) - 1u;
        uint32_t old = cnt[word];
        while (true) {
            const int c = (int)((old >> sh) & mask);
            if (c >= v) return false;
            const uint32_t prev = atomicCAS(&cnt[word], old, old + (1u << sh));
            if (prev == old) return c + 1 == v;
            old = prev;
        }
    }
}

// One workgroup per query.  Counters of B bits per id over passes of `chunk`
// ids; after a pass only the touched words are reset.  Windows beyond the
// register budget are re-read in every pass (the array is then cleared in
// full).  With redo_only set, only queries whose count is -1 are processed.
template <int B>
__global__ __launch_bounds__(kVoteBlock) void vote_kernel(const int32_t* __restrict__ leaf,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t n,
                                                          int32_t T, int32_t v, int32_t chunk,
                                                          int32_t* __restrict__ s_ids, int64_t cap,
                                                          int32_t* __restrict__ s_count, int32_t redo_only) {
    extern __shared__ uint32_t vote_cnt[];   // chunk * B / 32 words
    __shared__ int64_t tbase[kMaxT];
    __shared__ int32_t tlen[kMaxT];
    __shared__ int nsel;
    __shared__ int spill;
    constexpr int per = 32 / B;
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int w = uniform(tid >> 6);
    const int64_t q = blockIdx.x;
    const int words = chunk / per;
    if (redo_only && s_count[q] >= 0) return;

    if (tid < T) {
        const int L = leaf[q * T + tid];
        const int b = off[L];
        tbase[tid] = (int64_t)tid * n + b;
        tlen[tid] = off[L + 1] - b;
    }
    if (tid == 0) { nsel = 0; spill = 0; }
    for (int i = tid; i < (words >> 2); i += kVoteBlock)
        reinterpret_cast<uint4*>(vote_cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    // slot s holds window (tree jj, 64-id block uu) of this wave
    int32_t ids[kVoteSlots];
    int jj = w, uu = 0;
#pragma unroll
    for (int s = 0; s < kVoteSlots; ++s) {
        ids[s] = -1;
        if (jj < T) {
            const int len = uniform(tlen[jj]);
            const int e = uu * kWave + lane;
            if (e < len) ids[s] = perm[tbase[jj] + e];
            ++uu;
            if (uu * kWave >= len) { uu = 0; jj += kVoteWaves; }
        }
    }
    const int spill_j = jj, spill_u = uu;   // first window that did not fit
    if (lane == 0 && spill_j < T) spill = 1;
    __syncthreads();
    const bool full_clear = spill != 0;

    int32_t* out = s_ids + q * cap;
    for (int64_t lo = 0; lo < n; lo += chunk) {
        const int64_t hi = lo + chunk < n ? lo + chunk : n;
#pragma unroll
        for (int s = 0; s < kVoteSlots; ++s) {
            const int32_t id = ids[s];
            bool elect = false;
            if (id >= lo && id < hi) elect = count_id<B>(vote_cnt, (uint32_t)(id - lo), v);
            append(elect, id, &nsel, out, cap);
        }
        for (int j2 = spill_j, u2 = spill_u; j2 < T;) {
            int32_t sid[8];                 // 8 windows in flight
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                sid[b] = -1;
                if (j2 < T) {
                    const int len = uniform(tlen[j2]);
                    const int e = u2 * kWave + lane;
                    if (e < len) sid[b] = perm[tbase[j2] + e];
                    ++u2;
                    if (u2 * kWave >= len) { u2 = 0; j2 += kVoteWaves; }
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                bool elect = false;
                if (sid[b] >= lo && sid[b] < hi) elect = count_id<B>(vote_cnt, (uint32_t)(sid[b] - lo), v);
                append(elect, sid[b], &nsel, out, cap);
            }
        }
        if (hi >= n) break;
        __syncthreads();
        if (full_clear) {
            for (int i = tid; i < (words >> 2); i += kVoteBlock)
                reinterpret_cast<uint4*>(vote_cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
        } else {
#pragma unroll
            for (int s = 0; s < kVoteSlots; ++s) {
                const int32_t id = ids[s];
                if (id >= lo && id < hi) vote_cnt[(uint32_t)(id - lo) / per] = 0u;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (tid == 0) s_count[q] = nsel < cap ? nsel : (int32_t)cap;
}

// ---------------------------------------------------------------------------
// single-pass form
// ---------------------------------------------------------------------------
constexpr int kHashEntries = 6144;   // 24 KB of (id + 1) << 8 | count
constexpr int kCompact = 128;        // repeated ids buffered per wave
constexpr int kMapBatch = 8;         // slots whose map updates are issued together

__device__ __forceinline__ uint32_t hash_slot(int32_t id) {
    const uint32_t h = (uint32_t)id * 2654435761u;
    return (uint32_t)(((uint64_t)h * kHashEntries) >> 32);
}

// F(id) after this occurrence (>= 2) for an id whose map bit was already set;
// 0 if the table is full
__device__ __forceinline__ int hash_increment(uint32_t* tab, int32_t id) {
    const uint32_t key = (uint32_t)(id + 1);
    uint32_t h = hash_slot(id);
    for (int probe = 0; probe < kHashEntries; ++probe) {
        uint32_t cur = tab[h];
        if (cur == 0u) {
            const uint32_t prev = atomicCAS(&tab[h], 0u, (key << 8) | 2u);
            if (prev == 0u) return 2;
            cur = prev;
        }
        if ((cur >> 8) == key) {
            const uint32_t old = atomicAdd(&tab[h], 1u);
            return (int)(old & 0xffu) + 1;
        }
        h = h + 1u == (uint32_t)kHashEntries ? 0u : h + 1u;
    }
    return 0;
}

// counts of the buffered repeated ids, all lanes busy; elected ids appended
__device__ __forceinline__ void flush_repeats(const int32_t* buf, int cnt, uint32_t* tab, int v, int* ovf, int* nsel,
                                              int32_t* out, int64_t cap) {
    for (int i = 0; i < cnt; i += kWave) {
        const int j = i + lane_id();
        const int32_t id = j < cnt ? buf[j] : -1;
        int c = -1;
        if (id >= 0) {
            c = hash_increment(tab, id);
            if (c == 0) *ovf = 1;
        }
        append(c == v, id, nsel, out, cap);
    }
}

// First occurrences set a bit of the id map (one LDS atomic OR, no branch);
// a set bit marks a repeated occurrence, which is compacted into the wave's
// buffer and counted in the hash table when the buffer is flushed (then all
// 64 lanes work on repeats).  For v = 1 the map alone decides.  Persistent
// over queries q, q + gridDim.x, ...: while q is counted, the windows of the
// next query and the leaf positions of the one after are in flight.
template <bool HASH>
__global__ __launch_bounds__(kVoteBlock) void vote_map_kernel(const int32_t* __restrict__ leaf,
                                                              const int32_t* __restrict__ perm,
                                                              const int32_t* __restrict__ off, int64_t n,
                                                              int32_t T, int32_t v, int64_t nq, int32_t map_words,
                                                              int32_t* __restrict__ s_ids, int64_t cap,
                                                              int32_t* __restrict__ s_count) {
    extern __shared__ uint32_t map_smem[];   // map [map_words] | table | per-wave buffers
    __shared__ int32_t tbase[2][kMaxT];       // leaf start inside its tree
    __shared__ int32_t tlen[2][kMaxT];
    __shared__ int nsel[2];
    __shared__ int ovf[2];
    constexpr int kTab = HASH ? kHashEntries : 0;
    uint32_t* map = map_smem;
    uint32_t* tab = map_smem + map_words;
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int w = uniform(tid >> 6);
    int32_t* cbuf = reinterpret_cast<int32_t*>(map_smem + map_words + kTab) + w * kCompact;
    const uint32_t dummy = (uint32_t)map_words - 1u;    // a word past every real id
    const int64_t stride = gridDim.x;
    int64_t q = blockIdx.x;
    if (q >= nq) return;

    for (int i = tid; i < ((map_words + kTab) >> 2); i += kVoteBlock)
        reinterpret_cast<uint4*>(map_smem)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int k = 0; k < 2; ++k) {
        const int64_t qq = q + k * stride;
        if (qq < nq && tid < T) {
            const int L = leaf[qq * T + tid];
            const int b = off[L];
            tbase[k][tid] = b;
            tlen[k][tid] = off[L + 1] - b;
        }
    }
    if (tid < 2) { nsel[tid] = 0; ovf[tid] = 0; }
    lds_barrier();

    int32_t ids[kVoteSlots], nid[kVoteSlots];
#define MRPT_LOAD_WINDOWS(DST, BUF)                                              \
    do {                                                                         \
        int jj = w, uu = 0;                                                      \
        _Pragma("unroll") for (int s = 0; s < kVoteSlots; ++s) {                 \
            DST[s] = -1;                                                         \
            if (jj < T) {                                                        \
                const int len = uniform(tlen[BUF][jj]);                          \
                const int e = uu * kWave + lane;                                 \
                if (e < len) DST[s] = perm[(int64_t)jj * n + tbase[BUF][jj] + e]; \
                ++uu;                                                            \
                if (uu * kWave >= len) { uu = 0; jj += kVoteWaves; }             \
            }                                                                    \
        }                                                                        \
    } while (0)
    MRPT_LOAD_WINDOWS(ids, 0);
    int cur = 0;
    while (true) {
        const int nxt = cur ^ 1;
        const int64_t q1 = q + stride, q2 = q + 2 * stride;
        if (q1 < nq) MRPT_LOAD_WINDOWS(nid, nxt);           // in flight while q is counted
        int L2 = 0;
        if (q2 < nq && tid < T) L2 = leaf[q2 * T + tid];     // likewise
        int32_t* out = s_ids + q * cap;
        int* my_nsel = &nsel[cur];
        int pending = 0;                                     // wave-uniform fill of cbuf
#pragma unroll
        for (int s0 = 0; s0 < kVoteSlots; s0 += kMapBatch) {
            uint32_t old[kMapBatch];
#pragma unroll
            for (int g = 0; g < kMapBatch; ++g) {
                const int32_t id = ids[s0 + g];
                const uint32_t word = id >= 0 ? (uint32_t)id >> 5 : dummy;
                old[g] = atomicOr(&map[word], 1u << (id & 31));
            }
#pragma unroll
            for (int g = 0; g < kMapBatch; ++g) {
                const int32_t id = ids[s0 + g];
                const bool seen = id >= 0 && ((old[g] >> (id & 31)) & 1u);
                if constexpr (!HASH) {
                    append(id >= 0 && !seen, id, my_nsel, out, cap);
                } else {
                    const uint64_t m = __ballot(seen);
                    if (m) {
                        const int c = __popcll(m);
                        if (pending + c > kCompact) {
                            flush_repeats(cbuf, pending, tab, v, &ovf[cur], my_nsel, out, cap);
                            pending = 0;
                        }
                        if (seen) cbuf[pending + __popcll(m & __lanemask_lt())] = id;
                        pending += c;
                    }
                }
            }
        }
        if constexpr (HASH) flush_repeats(cbuf, pending, tab, v, &ovf[cur], my_nsel, out, cap);
        lds_barrier();
        if (q2 < nq && tid < T) {                            // buffer cur held q's positions: free now
            const int b = off[L2];
            tbase[cur][tid] = b;
            tlen[cur][tid] = off[L2 + 1] - b;
        }
        if (tid == 0) { nsel[nxt] = 0; ovf[nxt] = 0; }
#pragma unroll
        for (int s = 0; s < kVoteSlots; ++s) map[ids[s] >= 0 ? (uint32_t)ids[s] >> 5 : dummy] = 0u;
        if constexpr (HASH) {
            for (int i = tid; i < (kTab >> 2); i += kVoteBlock)
                reinterpret_cast<uint4*>(tab)[i] = make_uint4(0u, 0u, 0u, 0u);
        }
        lds_barrier();
        if (tid == 0) s_count[q] = ovf[cur] ? -1 : (nsel[cur] < cap ? nsel[cur] : (int32_t)cap);
        if (q1 >= nq) break;
#pragma unroll
        for (int s = 0; s < kVoteSlots; ++s) ids[s] = nid[s];
        cur = nxt;
        q = q1;
    }
#undef MRPT_LOAD_WINDOWS
}

// debug: F(x; q) of every listed candidate, by binary search of x in each of
// the query's T leaf lists (independent of the counting kernels)
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

__global__ void copy_counts_kernel(const int32_t* __restrict__ src, int64_t nq, int32_t* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) dst[i] = src[i];
}

// MRPT_VOTE_KERNEL=0 forces the multi-pass kernel (tuning and tests); the
// default takes the single-pass kernel whenever it fits
bool single_pass_allowed() {
    const char* env = std::getenv("MRPT_VOTE_KERNEL");
    return !(env && *env && std::atoi(env) == 0);
}

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

template <int B>
hipError_t launch_vote_b(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                         int64_t cap, int32_t* s_count, hipStream_t s) {
    constexpr int per = 32 / B;
    const size_t limit = (size_t)std::min(lds_per_block_limit(), 160 * 1024);
    // multi-pass geometry: ids per pass, a multiple of 4 words' worth of ids
    constexpr size_t kStaticMulti = kMaxT * 8 + kMaxT * 4 + 16;
    int64_t chunk = (int64_t)((limit - kStaticMulti) / 16) * 4 * per;
    const int64_t padded = (ix->n + 4 * per - 1) / (4 * per) * (4 * per);
    if (chunk > padded) chunk = padded;
    const int64_t passes = (ix->n + chunk - 1) / chunk;   // same passes, smaller array
    chunk = ((ix->n + passes - 1) / passes + 4 * per - 1) / (4 * per) * (4 * per);
    const size_t multi_lds = (size_t)(chunk / per) * 4;

    // single-pass geometry: map words (with one spare word) + table + buffers
    const bool hash = v >= 2;
    const int64_t map_words = ((ix->n + 31) / 32 + 1 + 3) / 4 * 4;   // the last word is never a real id's
    const size_t map_lds = (size_t)map_words * 4 + (hash ? (size_t)kHashEntries * 4 + kVoteWaves * kCompact * 4 : 0);
    constexpr size_t kStaticMap = 2 * kMaxT * 4 * 2 + 16;
    const int64_t windows = (int64_t)((ix->T + kVoteWaves - 1) / kVoteWaves) * ((ix->max_leaf + kWave - 1) / kWave);
    const bool single = single_pass_allowed() && map_lds + kStaticMap <= limit && windows <= kVoteSlots &&
                        ix->n < (int64_t(1) << 24);
    if (single) {
        const int64_t grid = std::min<int64_t>(nq, device_cus());
#define MRPT_MAP(H)                                                                                               \
    do {                                                                                                          \
        (void)hipFuncSetAttribute((const void*)vote_map_kernel<H>, hipFuncAttributeMaxDynamicSharedMemorySize,     \
                                  (int)map_lds);                                                                  \
        hipLaunchKernelGGL(vote_map_kernel<H>, dim3((unsigned)grid), dim3(kVoteBlock), map_lds, s, leaf, ix->perm, \
                           ix->off, ix->n, ix->T, v, nq, (int32_t)map_words, s_ids, cap, s_count);               \
    } while (0)
        if (hash) MRPT_MAP(true);
        else MRPT_MAP(false);
#undef MRPT_MAP
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !hash) return e;
        // queries whose table overflowed (count -1) are counted again, multi-pass
    }
    (void)hipFuncSetAttribute((const void*)vote_kernel<B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)multi_lds);
    hipLaunchKernelGGL(vote_kernel<B>, dim3((unsigned)nq), dim3(kVoteBlock), multi_lds, s, leaf, ix->perm, ix->off,
                       ix->n, ix->T, v, (int32_t)chunk, s_ids, cap, s_count, single ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_vote(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                       int64_t cap, int32_t* s_count, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    if (v == 1) return launch_vote_b<1>(ix, leaf, nq, v, s_ids, cap, s_count, s);
    if (v <= 3) return launch_vote_b<2>(ix, leaf, nq, v, s_ids, cap, s_count, s);
    if (v <= 15) return launch_vote_b<4>(ix, leaf, nq, v, s_ids, cap, s_count, s);
    return launch_vote_b<8>(ix, leaf, nq, v, s_ids, cap, s_count, s);
}

hipError_t launch_vote_counts(const mrpt_index* ix, const int32_t* leaf, int64_t nq, const int32_t* s_ids,
                              int64_t cap, const int32_t* s_count, uint8_t* s_votes, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(vote_counts_kernel, dim3((unsigned)nq), dim3(256), 0, s, leaf, ix->perm, ix->off, ix->n,
                       ix->T, s_ids, cap, s_count, s_votes);
    return hipGetLastError();
}

hipError_t launch_copy_counts(const int32_t* src, int64_t nq, int32_t* dst, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_counts_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, src, nq, dst);
    return hipGetLastError();
}

}  // namespace mrpt
