// Vote kernel (Sec. III-A, Alg. 4): for one query, F(x; q) counts the trees
// whose leaf holds both x and q, and x joins S when its count reaches v.
//
// One workgroup per query.  Each wave owns trees w, w+NW, ...; their leaf
// lists (ascending ids, contiguous in the tree's permutation) are loaded as
// 64-id windows into registers once.  Counting runs in passes over id ranges
// that fit a packed LDS counter array of B bits per id, where B is the
// smallest width that can hold v (1 bit for v = 1, 2 bits for v <= 3, ...):
// a counter saturates at v, so a point is appended to S exactly once, by the
// thread whose update moves its counter from v-1 to v, as in Alg. 4.  After
// a pass only the words that were touched are reset, so the array is cleared
// in full once per query.  Windows that do not fit the register budget are
// re-read from memory in every pass (and then the array is cleared in full).
#include <cstdlib>

#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

using namespace dev;

constexpr int kVoteWaves = 16;
constexpr int kVoteBlock = kVoteWaves * kWave;
constexpr int kVoteSlots = 32;

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

// wave-aggregated append of the ids whose `elect` is set
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
    // second launch after the single-pass kernel: only queries it gave up on (count -1)
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

    // register windows: slot s holds window (tree jj, 64-id block uu) of this wave
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
            const bool in = id >= lo && id < hi;
            bool elect = false;
            if (in) elect = count_id<B>(vote_cnt, (uint32_t)(id - lo), v);
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
                const bool in = sid[b] >= lo && sid[b] < hi;
                bool elect = false;
                if (in) elect = count_id<B>(vote_cnt, (uint32_t)(sid[b] - lo), v);
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
// Persistent form (every wave's windows fit its registers): one workgroup per
// CU walks the queries blockIdx.x, blockIdx.x + gridDim.x, ...  While it counts
// query q it already fetches the leaf of query q' = q + gridDim.x in every tree
// and the leaf's place in the permutation (during the first pass), so only
// the window loads of q' wait at the start of its turn.
// The counter array is cleared once per workgroup and kept clean by resetting
// the touched words after every pass.  The counter updates of kBatch slots are
// issued together (read, then one update attempt each, then the rare retries)
// so their LDS latencies overlap.
// ---------------------------------------------------------------------------
constexpr int kBatch = 4;

template <int B>
__device__ __forceinline__ void count_batch(const int32_t* ids, int64_t lo, int64_t hi, uint32_t* cnt, int v,
                                            int* nsel, int32_t* out, int64_t cap) {
    constexpr uint32_t per = 32u / B;
    constexpr uint32_t mask = B == 32 ? 0xffffffffu : ((1u << B) - 1u);
    uint32_t word[kBatch], sh[kBatch], cur[kBatch];
    bool act[kBatch], elect[kBatch];
#pragma unroll
    for (int g = 0; g < kBatch; ++g) {
        act[g] = ids[g] >= lo && ids[g] < hi;
        const uint32_t rel = act[g] ? (uint32_t)(ids[g] - lo) : 0u;
        word[g] = rel / per;
        sh[g] = (rel % per) * B;
        elect[g] = false;
    }
#pragma unroll
    for (int g = 0; g < kBatch; ++g) cur[g] = act[g] ? cnt[word[g]] : 0u;
#pragma unroll
    for (int g = 0; g < kBatch; ++g) {
        if (act[g]) {
            const int c = (int)((cur[g] >> sh[g]) & mask);
            if (c >= v) {
                act[g] = false;
            } else if constexpr (B == 1) {
                const uint32_t old = atomicOr(&cnt[word[g]], 1u << sh[g]);
                elect[g] = ((old >> sh[g]) & 1u) == 0u;
                act[g] = false;
            } else if constexpr (B == 8) {
                const uint32_t old = atomicAdd(&cnt[word[g]], 1u << sh[g]);
                elect[g] = (int)((old >> sh[g]) & 0xffu) + 1 == v;
                act[g] = false;
            } else {
                const uint32_t prev = atomicCAS(&cnt[word[g]], cur[g], cur[g] + (1u << sh[g]));
                if (prev == cur[g]) {
                    elect[g] = c + 1 == v;
                    act[g] = false;
                } else {
                    cur[g] = prev;
                }
            }
        }
    }
    if constexpr (B != 1 && B != 8) {
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            while (act[g]) {
                const int c = (int)((cur[g] >> sh[g]) & mask);
                if (c >= v) break;
                const uint32_t prev = atomicCAS(&cnt[word[g]], cur[g], cur[g] + (1u << sh[g]));
                if (prev == cur[g]) {
                    elect[g] = c + 1 == v;
                    break;
                }
                cur[g] = prev;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < kBatch; ++g) append(elect[g], ids[g], nsel, out, cap);
}

template <int B>
__global__ __launch_bounds__(kVoteBlock) void vote_persistent_kernel(const int32_t* __restrict__ leaf,
                                                                     const int32_t* __restrict__ perm,
                                                                     const int32_t* __restrict__ off, int64_t n,
                                                                     int32_t T, int32_t v, int32_t chunk,
                                                                     int64_t nq, int32_t* __restrict__ s_ids,
                                                                     int64_t cap, int32_t* __restrict__ s_count) {
    extern __shared__ uint32_t vote_cnt[];   // chunk * B / 32 words
    __shared__ int64_t tbase[2][kMaxT];
    __shared__ int32_t tlen[2][kMaxT];
    __shared__ int nsel[2];
    constexpr int per = 32 / B;
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int w = uniform(tid >> 6);
    const int words = chunk / per;
    int64_t q = blockIdx.x;
    if (q >= nq) return;

    for (int i = tid; i < (words >> 2); i += kVoteBlock)
        reinterpret_cast<uint4*>(vote_cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (tid < T) {
        const int L = leaf[q * T + tid];
        const int b = off[L];
        tbase[0][tid] = (int64_t)tid * n + b;
        tlen[0][tid] = off[L + 1] - b;
    }
    if (tid == 0) nsel[0] = 0;
    lds_barrier();

    int32_t ids[kVoteSlots];
    int cur = 0;
    while (true) {
        {
            int jj = w, uu = 0;
#pragma unroll
            for (int s = 0; s < kVoteSlots; ++s) {
                ids[s] = -1;
                if (jj < T) {
                    const int len = uniform(tlen[cur][jj]);
                    const int e = uu * kWave + lane;
                    if (e < len) ids[s] = perm[tbase[cur][jj] + e];
                    ++uu;
                    if (uu * kWave >= len) { uu = 0; jj += kVoteWaves; }
                }
            }
        }
        const int64_t qn = q + gridDim.x;
        const bool has_next = qn < nq;
        const int nxt = cur ^ 1;
        int Ln = 0;
        if (has_next && tid < T) Ln = leaf[qn * T + tid];   // in flight during pass 0
        int32_t* out = s_ids + q * cap;
        int pass = 0;
        for (int64_t lo = 0; lo < n; lo += chunk, ++pass) {
            const int64_t hi = lo + chunk < n ? lo + chunk : n;
            int* my_nsel = &nsel[cur];
#pragma unroll
            for (int s0 = 0; s0 < kVoteSlots; s0 += kBatch) {
                int32_t part[kBatch];
#pragma unroll
                for (int g = 0; g < kBatch; ++g) part[g] = ids[s0 + g];
                count_batch<B>(part, lo, hi, vote_cnt, v, my_nsel, out, cap);
            }
            lds_barrier();
            if (pass == 0 && has_next) {
                if (tid < T) {
                    const int b = off[Ln];
                    tbase[nxt][tid] = (int64_t)tid * n + b;
                    tlen[nxt][tid] = off[Ln + 1] - b;
                }
                if (tid == 0) nsel[nxt] = 0;
            }
#pragma unroll
            for (int s = 0; s < kVoteSlots; ++s) {
                const int32_t id = ids[s];
                if (id >= lo && id < hi) vote_cnt[(uint32_t)(id - lo) / per] = 0u;
            }
            lds_barrier();
        }
        if (tid == 0) s_count[q] = nsel[cur] < cap ? nsel[cur] : (int32_t)cap;
        if (!has_next) break;
        cur = nxt;
        q = qn;
    }
}

// ---------------------------------------------------------------------------
// Wave form: one wave per query, with a private slice of LDS, so waves never
// wait for each other and a CU keeps ~20 queries in flight.  Lane l follows
// the leaf lists of trees l, l+64, ... with a cursor; the id space is walked in
// ranges of `range` ids whose counters (B bits each) fill the wave's slice.
// In a range every lane reads the next 4 ids of each of its lists (ascending,
// so the ids of the range are a prefix), counts the prefix, and advances its
// cursors; the loop ends when no list has an id left in the range.
// ---------------------------------------------------------------------------
constexpr int kWaveWin = 4;            // ids read per list per step
constexpr int kWavesPerBlock = 4;

template <int B, int SPL>
__global__ __launch_bounds__(kWavesPerBlock * kWave) void vote_wave_kernel(
    const int32_t* __restrict__ leaf, const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
    int64_t n, int32_t T, int32_t v, int32_t range, int32_t words_per_wave, int64_t nq,
    int32_t* __restrict__ s_ids, int64_t cap, int32_t* __restrict__ s_count) {
    extern __shared__ uint32_t wave_cnt[];
    constexpr uint32_t per = 32u / B;
    constexpr uint32_t mask = B == 32 ? 0xffffffffu : ((1u << B) - 1u);
    const int lane = lane_id();
    const int w = uniform((int)(threadIdx.x >> 6));
    const int64_t q = (int64_t)blockIdx.x * kWavesPerBlock + w;
    if (q >= nq) return;                          // whole wave; no workgroup barrier below
    uint32_t* cnt = wave_cnt + (size_t)w * words_per_wave;

    int64_t base[SPL];
    int len[SPL], cur[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const int t = lane + s * kWave;
        base[s] = 0;
        len[s] = 0;
        cur[s] = 0;
        if (t < T) {
            const int L = leaf[q * T + t];
            const int b = off[L];
            base[s] = (int64_t)t * n + b;
            len[s] = off[L + 1] - b;
        }
    }
    int32_t* out = s_ids + q * cap;
    int nsel = 0;                                 // wave-uniform
    for (int64_t lo = 0; lo < n; lo += range) {
        const int64_t hi = lo + range < n ? lo + range : n;
        for (int i = lane; i < (words_per_wave >> 2); i += kWave)
            reinterpret_cast<uint4*>(cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
        bool active[SPL];
#pragma unroll
        for (int s = 0; s < SPL; ++s) active[s] = cur[s] < len[s];
        while (true) {
            bool any = false;
#pragma unroll
            for (int s = 0; s < SPL; ++s) any |= active[s];
            if (!__any(any)) break;
            int32_t id[SPL][kWaveWin];
#pragma unroll
            for (int s = 0; s < SPL; ++s)
#pragma unroll
                for (int j = 0; j < kWaveWin; ++j)
                    id[s][j] = (active[s] && cur[s] + j < len[s]) ? perm[base[s] + cur[s] + j] : INT32_MAX;
            // the prefix below hi of each window is this range's share of the list
            uint32_t word[SPL][kWaveWin], sh[SPL][kWaveWin], val[SPL][kWaveWin];
            bool act[SPL][kWaveWin], elect[SPL][kWaveWin];
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                int used = 0;
#pragma unroll
                for (int j = 0; j < kWaveWin; ++j) {
                    act[s][j] = id[s][j] < hi;
                    used += act[s][j] ? 1 : 0;
                    const uint32_t rel = act[s][j] ? (uint32_t)(id[s][j] - lo) : 0u;
                    word[s][j] = rel / per;
                    sh[s][j] = (rel % per) * B;
                    elect[s][j] = false;
                }
                cur[s] += used;
                active[s] = active[s] && used == kWaveWin && cur[s] < len[s];
            }
#pragma unroll
            for (int s = 0; s < SPL; ++s)
#pragma unroll
                for (int j = 0; j < kWaveWin; ++j) val[s][j] = act[s][j] ? cnt[word[s][j]] : 0u;
#pragma unroll
            for (int s = 0; s < SPL; ++s)
#pragma unroll
                for (int j = 0; j < kWaveWin; ++j) {
                    if (!act[s][j]) continue;
                    const int c = (int)((val[s][j] >> sh[s][j]) & mask);
                    if (c >= v) {
                        act[s][j] = false;
                    } else if constexpr (B == 1) {
                        const uint32_t old = atomicOr(&cnt[word[s][j]], 1u << sh[s][j]);
                        elect[s][j] = ((old >> sh[s][j]) & 1u) == 0u;
                        act[s][j] = false;
                    } else if constexpr (B == 8) {
                        const uint32_t old = atomicAdd(&cnt[word[s][j]], 1u << sh[s][j]);
                        elect[s][j] = (int)((old >> sh[s][j]) & 0xffu) + 1 == v;
                        act[s][j] = false;
                    } else {
                        const uint32_t prev = atomicCAS(&cnt[word[s][j]], val[s][j], val[s][j] + (1u << sh[s][j]));
                        if (prev == val[s][j]) {
                            elect[s][j] = c + 1 == v;
                            act[s][j] = false;
                        } else {
                            val[s][j] = prev;
                        }
                    }
                }
            if constexpr (B != 1 && B != 8) {
#pragma unroll
                for (int s = 0; s < SPL; ++s)
#pragma unroll
                    for (int j = 0; j < kWaveWin; ++j) {
                        while (act[s][j]) {
                            const int c = (int)((val[s][j] >> sh[s][j]) & mask);
                            if (c >= v) break;
                            const uint32_t prev =
                                atomicCAS(&cnt[word[s][j]], val[s][j], val[s][j] + (1u << sh[s][j]));
                            if (prev == val[s][j]) {
                                elect[s][j] = c + 1 == v;
                                break;
                            }
                            val[s][j] = prev;
                        }
                    }
            }
#pragma unroll
            for (int s = 0; s < SPL; ++s)
#pragma unroll
                for (int j = 0; j < kWaveWin; ++j) {
                    const uint64_t m = __ballot(elect[s][j]);
                    if (m) {
                        if (elect[s][j]) {
                            const int64_t p = (int64_t)nsel + __popcll(m & __lanemask_lt());
                            if (p < cap) out[p] = id[s][j];
                        }
                        nsel += __popcll(m);
                    }
                }
        }
    }
    if (lane == 0) s_count[q] = nsel < cap ? nsel : (int32_t)cap;
}

// ---------------------------------------------------------------------------
// Single-pass form (all n ids fit a 1-bit LDS map): the first occurrence of an
// id sets its bit; a repeated id goes to an open-addressing LDS hash table that
// holds (id + 1) << 8 | count for the ids seen at least twice.  F(x) is thus
// 1 for ids only in the map and the table count otherwise, and the occurrence
// that makes it v appends x to S (for v = 1, the one that sets the bit).  If
// the table fills up the query's count is stored as -1 and the query is redone
// by the multi-pass kernel.  The workgroup is persistent over queries q,
// q + gridDim.x, ...: while it counts q, the leaf windows of the next query and
// the leaf positions of the one after are already being fetched.
// ---------------------------------------------------------------------------
constexpr int kHashLog2 = 13;   // 8192 entries, 32 KB

__device__ __forceinline__ uint32_t hash_slot(int32_t id) {
    return ((uint32_t)id * 2654435761u) >> (32 - kHashLog2);
}

// F(id) after this occurrence (>= 2) for an id whose map bit was already set;
// 0 if the table is full
__device__ __forceinline__ int hash_increment(uint32_t* tab, int32_t id) {
    constexpr uint32_t kMask = (1u << kHashLog2) - 1u;
    const uint32_t key = (uint32_t)(id + 1);
    uint32_t h = hash_slot(id);
    for (int probe = 0; probe <= (int)kMask; ++probe) {
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
        h = (h + 1u) & kMask;
    }
    return 0;
}

template <bool HASH>
__global__ __launch_bounds__(kVoteBlock) void vote_bitmap_kernel(const int32_t* __restrict__ leaf,
                                                                 const int32_t* __restrict__ perm,
                                                                 const int32_t* __restrict__ off, int64_t n,
                                                                 int32_t T, int32_t v, int64_t nq, int32_t bm_words,
                                                                 int32_t* __restrict__ s_ids, int64_t cap,
                                                                 int32_t* __restrict__ s_count) {
    extern __shared__ uint32_t bm_smem[];   // bitmap [bm_words], then the table
    __shared__ int32_t tbase[2][kMaxT];   // leaf start inside its tree
    __shared__ int32_t tlen[2][kMaxT];
    __shared__ int nsel[2];
    __shared__ int ovf[2];
    constexpr int kTab = HASH ? (1 << kHashLog2) : 0;
    uint32_t* bm = bm_smem;
    uint32_t* tab = bm_smem + bm_words;
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int w = uniform(tid >> 6);
    const int64_t stride = gridDim.x;
    int64_t q = blockIdx.x;
    if (q >= nq) return;

    const int clear_words = bm_words + kTab;   // multiple of 4
    for (int i = tid; i < (clear_words >> 2); i += kVoteBlock)
        reinterpret_cast<uint4*>(bm_smem)[i] = make_uint4(0u, 0u, 0u, 0u);
    // leaf positions of the first two queries
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
#define MRPT_LOAD_WINDOWS(DST, BUF)                                          \
    do {                                                                     \
        int jj = w, uu = 0;                                                  \
        _Pragma("unroll") for (int s = 0; s < kVoteSlots; ++s) {             \
            DST[s] = -1;                                                     \
            if (jj < T) {                                                    \
                const int len = uniform(tlen[BUF][jj]);                      \
                const int e = uu * kWave + lane;                             \
                if (e < len) DST[s] = perm[(int64_t)jj * n + tbase[BUF][jj] + e]; \
                ++uu;                                                        \
                if (uu * kWave >= len) { uu = 0; jj += kVoteWaves; }         \
            }                                                                \
        }                                                                    \
    } while (0)
    MRPT_LOAD_WINDOWS(ids, 0);
    int cur = 0;
    while (true) {
        const int nxt = cur ^ 1;
        const int64_t q1 = q + stride, q2 = q + 2 * stride;
        if (q1 < nq) MRPT_LOAD_WINDOWS(nid, nxt);            // in flight while q is counted
        int L2 = 0;
        if (q2 < nq && tid < T) L2 = leaf[q2 * T + tid];      // likewise
        int32_t* out = s_ids + q * cap;
        int* my_nsel = &nsel[cur];
#pragma unroll
        for (int s0 = 0; s0 < kVoteSlots; s0 += kBatch) {
            uint32_t old[kBatch];
            bool elect[kBatch];
#pragma unroll
            for (int g = 0; g < kBatch; ++g) {
                const int32_t id = ids[s0 + g];
                old[g] = id >= 0 ? atomicOr(&bm[(uint32_t)id >> 5], 1u << (id & 31)) : 0u;
            }
#pragma unroll
            for (int g = 0; g < kBatch; ++g) {
                const int32_t id = ids[s0 + g];
                const bool seen = id >= 0 && ((old[g] >> (id & 31)) & 1u);
                elect[g] = id >= 0 && !seen && v == 1;
                if (HASH && seen) {
                    const int c = hash_increment(tab, id);
                    if (c == 0) ovf[cur] = 1;
                    elect[g] = c == v;
                }
            }
#pragma unroll
            for (int g = 0; g < kBatch; ++g) append(elect[g], ids[s0 + g], my_nsel, out, cap);
        }
        lds_barrier();
        if (q2 < nq && tid < T) {                             // buffer cur held q's positions: free now
            const int b = off[L2];
            tbase[cur][tid] = b;
            tlen[cur][tid] = off[L2 + 1] - b;
        }
        if (tid == 0) { nsel[nxt] = 0; ovf[nxt] = 0; }
#pragma unroll
        for (int s = 0; s < kVoteSlots; ++s)
            if (ids[s] >= 0) bm[(uint32_t)ids[s] >> 5] = 0u;
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

__global__ void copy_counts_kernel(const int32_t* __restrict__ src, int64_t nq, int32_t* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) dst[i] = src[i];
}

// Which vote kernel runs: 3 = single pass with the id map (default, when n
// fits), 2 = one wave per query, 1 = persistent multi-pass, 0 = one workgroup
// per query.  MRPT_VOTE_KERNEL selects another for tuning; all compute the
// same S.
int vote_kernel_choice() {
    const char* env = std::getenv("MRPT_VOTE_KERNEL");
    const int choice = (env && *env) ? std::atoi(env) : 3;
    return (choice < 0 || choice > 3) ? 3 : choice;
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

// the single-pass kernel, then the multi-pass one for the queries whose hash
// table overflowed; false if the id map does not fit
template <int B>
bool launch_vote_single_pass(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                             int64_t cap, int32_t* s_count, int64_t chunk, size_t multi_lds, hipStream_t s,
                             hipError_t* err) {
    constexpr size_t kStatic = 2 * kMaxT * 4 * 2 + 16;
    const bool hash = v >= 2;
    const int64_t bm_words = ((ix->n + 31) / 32 + 3) / 4 * 4;
    const size_t lds = (size_t)(bm_words + (hash ? (1 << kHashLog2) : 0)) * 4;
    const int64_t windows = (int64_t)((ix->T + kVoteWaves - 1) / kVoteWaves) * ((ix->max_leaf + kWave - 1) / kWave);
    if (lds + kStatic > (size_t)std::min(lds_per_block_limit(), 160 * 1024) || windows > kVoteSlots ||
        ix->n >= (int64_t(1) << 24))
        return false;
    const int64_t grid = std::min<int64_t>(nq, device_cus());
    if (hash) {
        (void)hipFuncSetAttribute((const void*)vote_bitmap_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(vote_bitmap_kernel<true>, dim3((unsigned)grid), dim3(kVoteBlock), lds, s, leaf, ix->perm,
                           ix->off, ix->n, ix->T, v, nq, (int32_t)bm_words, s_ids, cap, s_count);
        *err = hipGetLastError();
        if (*err != hipSuccess) return true;
        (void)hipFuncSetAttribute((const void*)vote_kernel<B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)multi_lds);
        hipLaunchKernelGGL(vote_kernel<B>, dim3((unsigned)nq), dim3(kVoteBlock), multi_lds, s, leaf, ix->perm,
                           ix->off, ix->n, ix->T, v, (int32_t)chunk, s_ids, cap, s_count, 1);
    } else {
        (void)hipFuncSetAttribute((const void*)vote_bitmap_kernel<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(vote_bitmap_kernel<false>, dim3((unsigned)grid), dim3(kVoteBlock), lds, s, leaf, ix->perm,
                           ix->off, ix->n, ix->T, v, nq, (int32_t)bm_words, s_ids, cap, s_count);
    }
    *err = hipGetLastError();
    return true;
}

template <int B>
hipError_t launch_vote_b(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                         int64_t cap, int32_t* s_count, hipStream_t s) {
    constexpr int per = 32 / B;
    constexpr size_t kStatic = 2 * (kMaxT * 8 + kMaxT * 4) + 16;
    // 16 waves of ~100 VGPRs hold a CU: the workgroup may take all of its LDS
    const size_t budget = (size_t)std::min(lds_per_block_limit(), 160 * 1024) - kStatic;
    // ids per pass: a multiple of 4 words' worth of ids, at most what the budget holds
    int64_t chunk = (int64_t)(budget / 16) * 4 * per;
    const int64_t padded = (ix->n + 4 * per - 1) / (4 * per) * (4 * per);
    if (chunk > padded) chunk = padded;
    // same number of passes, smaller array
    const int64_t passes = (ix->n + chunk - 1) / chunk;
    chunk = ((ix->n + passes - 1) / passes + 4 * per - 1) / (4 * per) * (4 * per);
    const size_t lds = (size_t)(chunk / per) * 4;
    // windows per wave: its trees times the 64-id windows of the longest leaf
    const int64_t windows = (int64_t)((ix->T + kVoteWaves - 1) / kVoteWaves) * ((ix->max_leaf + kWave - 1) / kWave);
    if (vote_kernel_choice() == 3) {
        hipError_t err = hipSuccess;
        if (launch_vote_single_pass<B>(ix, leaf, nq, v, s_ids, cap, s_count, chunk, lds, s, &err)) return err;
    }
    if (vote_kernel_choice() == 2) {
        // one wave per query: an 8 KB counter slice per wave
        constexpr int64_t kSliceBytes = 8192;
        const int64_t range_max = kSliceBytes * 8 / B;
        int64_t range = std::min<int64_t>(range_max, (ix->n + 4 * per - 1) / (4 * per) * (4 * per));
        const int32_t words = (int32_t)(range / per);
        const size_t lds_w = (size_t)words * 4 * kWavesPerBlock;
        const unsigned grid = (unsigned)((nq + kWavesPerBlock - 1) / kWavesPerBlock);
        const int spl = (ix->T + kWave - 1) / kWave;
#define MRPT_VW(SPL)                                                                                          \
    do {                                                                                                      \
        (void)hipFuncSetAttribute((const void*)vote_wave_kernel<B, SPL>,                                      \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_w);                    \
        hipLaunchKernelGGL((vote_wave_kernel<B, SPL>), dim3(grid), dim3(kWavesPerBlock * kWave), lds_w, s, leaf, \
                           ix->perm, ix->off, ix->n, ix->T, v, (int32_t)range, words, nq, s_ids, cap, s_count);  \
    } while (0)
        switch (spl) {
            case 1: MRPT_VW(1); break;
            case 2: MRPT_VW(2); break;
            case 3: MRPT_VW(3); break;
            default: MRPT_VW(4); break;
        }
#undef MRPT_VW
        return hipGetLastError();
    }
    if (windows <= kVoteSlots && vote_kernel_choice() == 1) {
        const int64_t grid = std::min<int64_t>(nq, device_cus());
        (void)hipFuncSetAttribute((const void*)vote_persistent_kernel<B>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(vote_persistent_kernel<B>, dim3((unsigned)grid), dim3(kVoteBlock), lds, s, leaf, ix->perm,
                           ix->off, ix->n, ix->T, v, (int32_t)chunk, nq, s_ids, cap, s_count);
        return hipGetLastError();
    }
    (void)hipFuncSetAttribute((const void*)vote_kernel<B>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(vote_kernel<B>, dim3((unsigned)nq), dim3(kVoteBlock), lds, s, leaf, ix->perm, ix->off, ix->n,
                       ix->T, v, (int32_t)chunk, s_ids, cap, s_count, 0);
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
