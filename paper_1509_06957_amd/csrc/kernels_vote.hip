// Vote kernels (Sec. III-A, Alg. 4): for one query, F(x; q) counts the trees
// whose leaf holds both x and q, and x joins the candidate set S when its
// count reaches v (in Alg. 4, at the moment the count becomes v).
//
// Two forms, both one workgroup of 16 waves per CU-resident query:
//
//  * single pass (when a 1-bit map of all n ids fits LDS): the first
//    occurrence of an id sets its bit; repeated occurrences are queued, and
//    the queue is run through the map again, v - 1 times, to find the ids
//    with F >= v.  The workgroup is persistent over queries and has the next
//    query's leaf windows in flight while it counts.
//  * multi pass (any n): packed counters of B bits per id (the smallest width
//    that holds v) over id ranges that fit LDS, one pass per range; it also
//    recounts the queries whose repeat queue overflowed.
//
// A tree's leaf list (ascending ids, contiguous in that tree's permutation)
// is read as 64-id windows into registers, coalesced.
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

// The queries a multi-pass workgroup counts.  Counting all queries: q =
// blockIdx.x, + gridDim.x, ... .  Recounting (redo_only): the workgroup owns
// the per = ceil(nq / gridDim.x) <= 1024 queries from blockIdx.x * per (the
// grid is at least ceil(nq / 1024) and about one workgroup per CU, so many
// overflows still spread over the chip), reads their counts in one coalesced
// load and keeps those marked -1 (queue overflow) in `list`.  Returns how
// many queries the workgroup takes; query `it` is redo_query(...).
__device__ __forceinline__ int64_t redo_select(bool redo_only, int64_t nq, const int32_t* __restrict__ s_count,
                                               int32_t* list, int* n) {
    if (!redo_only) return blockIdx.x < nq ? (nq - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
    const int tid = (int)threadIdx.x;
    if (tid == 0) *n = 0;
    __syncthreads();
    const int64_t per = (nq + gridDim.x - 1) / gridDim.x;
    const int64_t qq = (int64_t)blockIdx.x * per + tid;
    if (tid < per && qq < nq && s_count[qq] < 0) list[atomicAdd(n, 1)] = tid;
    __syncthreads();
    return *n;
}

__device__ __forceinline__ int64_t redo_query(bool redo_only, int64_t it, const int32_t* list, int64_t nq) {
    return redo_only ? (int64_t)blockIdx.x * ((nq + gridDim.x - 1) / gridDim.x) + list[it]
                     : (int64_t)blockIdx.x + it * gridDim.x;
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

// One workgroup per query (queries blockIdx.x, + gridDim.x, ...).  Counters
// of B bits per id over passes of `chunk` ids; after a pass only the touched
// words are reset.  Windows beyond the
// register budget are re-read in every pass (the array is then cleared in
// full).  With redo_only set, only queries whose count is -1 are processed.
template <int B>
__global__ __launch_bounds__(kVoteBlock) void vote_kernel(const int32_t* __restrict__ leaf,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t n, int64_t ld,
                                                          int32_t T, int32_t v, int64_t nq, int32_t chunk,
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
    const int words = chunk / per;
    __shared__ int32_t redo_list[kVoteBlock];
    __shared__ int redo_n;
    const int64_t nwork = redo_select(redo_only != 0, nq, s_count, redo_list, &redo_n);
    for (int64_t it = 0; it < nwork; ++it) {
    const int64_t q = redo_query(redo_only != 0, it, redo_list, nq);

    if (tid < T) {
        const int L = leaf[q * T + tid];
        const int b = off[L];
        tbase[tid] = (int64_t)tid * ld + b;
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
    __syncthreads();                        // shared state is reused by the next query
    }
}

// ---------------------------------------------------------------------------
// multi-pass form with a leaf directory
// ---------------------------------------------------------------------------
// A leaf's ids are ascending, so the ids of one pass [lo, hi) are one slice
// of it.  The directory holds, for tree t, leaf L and boundary j, the position
// of the leaf's first id >= min(j * grain, n); passes start and end on
// boundaries, so every pass reads exactly its slice of each of the query's T
// leaves and each id is read once per query instead of once per pass.
__global__ void vote_dir_build_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
                                      int64_t n, int64_t ld, int32_t nleaf, int32_t nb, int32_t grain, int64_t total,
                                      int32_t* __restrict__ dir) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total) return;
    const int32_t j = (int32_t)(x % nb);
    const int64_t tl = x / nb;
    const int32_t L = (int32_t)(tl % nleaf);
    const int64_t t = tl / nleaf;
    const int32_t* ids = perm + t * ld + off[L];
    const int64_t target = (int64_t)j * grain < n ? (int64_t)j * grain : n;
    int32_t lo = 0, hi = off[L + 1] - off[L];   // first position whose id >= target
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (ids[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    dir[x] = lo;
}

// ---------------------------------------------------------------------------
// single-pass form (n < 2^24 and the id map fits LDS; windows in registers)
// ---------------------------------------------------------------------------
// A 1-bit map over the ids answers "seen before?" with one LDS atomic OR per
// id occurrence.  Reading a query's windows through the map leaves the first
// occurrence of every id in the map and queues each repeated occurrence
// (an id with F = f is queued f - 1 times).  For v = 1 the first occurrences
// are S.  For v >= 2 the queue is run through the map v - 1 more times:
// each of the first v - 2 runs blanks the first queued occurrence of every
// id, so after j runs an id with F = f has f - 1 - j occurrences left, and
// the last run elects the first remaining occurrence of every id, i.e.
// exactly the ids with F >= v, each once.  No clear is needed between runs:
// after the window pass every queued id's bit is set, so the first run finds
// first occurrences by clearing bits (atomic AND), the next by setting them
// again (atomic OR), and so on, since the ids a run examines are exactly ids
// the previous run examined (their bits all flipped by it).  The queue is a few thousand
// entries, so these runs use all 1024 threads and cost little.  A query whose
// queue overflows gets count -1 and is recounted by the multi-pass kernel.
//
// The workgroup is persistent over the queries g, g + G, ...: while query q
// is counted, the leaf windows of the next query (registers), the leaf
// offsets of the one after and the leaf numbers of the third are in flight.
// A query's T * wpl windows (tree u / wpl, 64-id part u % wpl) are dealt
// round-robin over the 16 waves: slot s of wave w is window w + 16 s.  Every
// slot issues one load per lane with no branch around it (so the compiler
// can count the loads in flight): a lane beyond its leaf, or a slot beyond
// the last tree, reads the padding entry n + 32 lane of perm row 0, which
// holds that value; such ids are never queued or elected, and their map bits
// lie in spare words past the ids, a different word for every lane.  Loads address perm by a 32-bit byte offset
// from its base.  Two queries are counted per loop turn, so the windows in
// flight and the windows counted swap register arrays instead of moving.
// slots whose map updates are issued together (13: the two batches of a
// 25-slot wave, the sift-like shape, without spilling the batch's lane masks
// out of scalar registers; 5 took 4 % longer there)
constexpr int kMapBatch = 13;
constexpr int kPosBufs = 3;          // leaf position buffers of the pipeline

// number of set bits of m below this lane, plus base
__device__ __forceinline__ uint32_t rank_below(uint64_t m, uint32_t base) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
}

// tot places reserved on the LDS counter *fill, its old value returned to
// the wave: lane 0 adds tot, lanes 1..63 add 0 to spare words of their own,
// so the add is one full-wave LDS atomic with no branch around it
__device__ __forceinline__ uint32_t reserve(int* fill, int* spare, int tot) {
    const int lane = lane_id();
    const int old = atomicAdd(lane == 0 ? fill : spare + lane, lane == 0 ? tot : 0);
    return (uint32_t)__builtin_amdgcn_readfirstlane(old);
}

// The ids of NB slots whose lanes pass the test (old & bit) != 0 (REPEAT) or
// == 0 (first occurrence), real ids only (id < n32), stored at consecutive
// places of out from one reservation on *fill.  Places at or beyond cap are
// dropped; the caller sees that as *fill > cap.  The per-lane test is written
// out where it is used: a bool kept across the stores' branches would be
// rebuilt from a vector 0/1 value.
template <bool REPEAT, int NB>
__device__ __forceinline__ void append_batch(const uint32_t (&ob)[NB], const int32_t (&id)[NB], int32_t n32,
                                             int* fill, int* spare, int32_t* out, uint32_t cap) {
    uint64_t m[NB];
    int tot = 0;
#pragma unroll
    for (int g = 0; g < NB; ++g) {
        m[g] = __builtin_amdgcn_ballot_w64(REPEAT ? ob[g] != 0u : ob[g] == 0u) &
               __builtin_amdgcn_ballot_w64(id[g] < n32);
        tot += __popcll(m[g]);
    }
    if (tot == 0) return;
    const uint32_t base = reserve(fill, spare, tot);
    if (base + (uint32_t)tot <= cap) {
        int32_t* o = out + base;
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            if ((REPEAT ? ob[g] != 0u : ob[g] == 0u) && id[g] < n32) o[rank_below(m[g], 0u)] = id[g];
            o += __popcll(m[g]);
        }
    } else {
        uint32_t at0 = base;
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            if ((REPEAT ? ob[g] != 0u : ob[g] == 0u) && id[g] < n32) {
                const uint32_t at = rank_below(m[g], at0);
                if (at < cap) out[at] = id[g];
            }
            at0 += (uint32_t)__popcll(m[g]);
        }
    }
}

// Per-slot window descriptors of wave w of NW, one slot per lane (lanes >=
// S unused): part = 64-id part of the window in its leaf (-1 past the last
// tree) and tp = tree | 64 * part << 8.  Computed once per kernel.
template <int NW>
__device__ __forceinline__ void slot_table(int w, int T, int wpl, int& part64, int& tp) {
    const int u = w + NW * lane_id();
    const int t = u / wpl, part = u - t * wpl;
    part64 = t < T ? part * kWave : -1;
    tp = t < T ? (t | (part * kWave) << 8) : 0;
}

// the windows of one query, lane s holding slot s's: first = perm index of
// its first id, avail = ids in it (0 past the last tree).  The leaf positions
// hold each tree's leaf as (perm index of its first id, length).  One LDS
// read of them per wave; the slots read these back with readlane.
__device__ __forceinline__ void slot_windows(const int2* __restrict__ tpos, int part64, int slot_tp, int& first,
                                             int& avail) {
    const int2 bl = tpos[slot_tp & 255];
    first = part64 + bl.x;
    avail = part64 < 0 ? 0 : bl.y - (slot_tp >> 8);
}

template <int S>
__device__ __forceinline__ void load_windows(int32_t (&dst)[S], const int32_t* __restrict__ perm, uint32_t pad4,
                                             int first_v, int avail_v) {
    const int lane = lane_id();
    const uint32_t lane4 = (uint32_t)lane * 4u;
    const char* base = reinterpret_cast<const char*>(perm);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        // byte offset from the start of perm (T * ld * 4 < 2^32): the slot's
        // entry for lanes inside the window, the lane's padding entry else
        const uint32_t first4 = (uint32_t)__builtin_amdgcn_readlane(first_v, s) * 4u;
        const int avail = __builtin_amdgcn_readlane(avail_v, s);
        const uint32_t at = lane < avail ? first4 + lane4 : pad4;
        dst[s] = *reinterpret_cast<const int32_t*>(base + at);
    }
}

// One workgroup per query (queries blockIdx.x, + gridDim.x, ...); 8-bit
// counters over passes of `chunk` ids (a multiple of the grain), cleared in
// full before each pass.  A count never exceeds T <= 255, so one atomic add
// per id suffices: the id is elected by the add that finds v - 1.  Wave w
// takes trees w, w + 16, ... and reads each slice in 64-id windows,
// kDirWindows in flight, whose atomics are then issued together; their
// elections are stored from one reservation.  The loads need no bounds
// branch: a window reaches at most 63 entries past its slice, which stay
// inside the tree's perm row (n ids, then padding).  With redo_only set, only
// queries whose count is -1 are processed.
constexpr int kDirWindows = 16;

__global__ __launch_bounds__(kVoteBlock) void vote_dir_kernel(
    const int32_t* __restrict__ leaf, const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
    const int32_t* __restrict__ dir, int32_t nleaf, int32_t nb, int32_t grain, int64_t n, int64_t ld, int32_t T,
    int32_t v, int64_t nq, int32_t chunk, int32_t* __restrict__ s_ids, int64_t cap, int32_t* __restrict__ s_count,
    int32_t redo_only) {
    extern __shared__ uint32_t vote_cnt[];   // chunk / 4 words, one byte per id
    __shared__ int64_t tbase[kMaxT];         // perm index of the leaf's first id
    __shared__ int64_t tslice[kMaxT];        // this pass: perm index of the slice, its length
    __shared__ int32_t tlen[kMaxT];
    __shared__ int nsel;
    __shared__ int spare[kWave];             // targets of the reservations' idle lanes
    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int w = uniform(tid >> 6);
    const int words = chunk >> 2;
    const uint32_t hit = (uint32_t)(v - 1);
    const uint32_t cap32 = (uint32_t)(cap < INT32_MAX ? cap : INT32_MAX);
    __shared__ int32_t redo_list[kVoteBlock];
    __shared__ int redo_n;
    const int64_t nwork = redo_select(redo_only != 0, nq, s_count, redo_list, &redo_n);
    for (int64_t it = 0; it < nwork; ++it) {
        const int64_t q = redo_query(redo_only != 0, it, redo_list, nq);
        // thread t < T follows tree t's slice boundaries, one pass ahead: a
        // pass's slice starts where the previous one ended
        int64_t row = 0;
        int32_t cut_lo = 0, cut_hi = 0;
        if (tid < T) {
            const int L = leaf[q * T + tid];
            tbase[tid] = (int64_t)tid * ld + off[L];
            row = ((int64_t)tid * nleaf + L) * nb;
            const int64_t hi0 = chunk < n ? chunk : n;
            cut_lo = dir[row];
            cut_hi = dir[row + (hi0 == n ? nb - 1 : (int)(hi0 / grain))];
        }
        if (tid == 0) nsel = 0;
        int32_t* out = s_ids + q * cap;
        for (int64_t lo = 0; lo < n; lo += chunk) {
            const int64_t hi = lo + chunk < n ? lo + chunk : n;
            __syncthreads();                 // the previous pass is done with the counters
            for (int i = tid; i < (words >> 2); i += kVoteBlock)
                reinterpret_cast<uint4*>(vote_cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
            if (tid < T) {
                tslice[tid] = tbase[tid] + cut_lo;
                tlen[tid] = cut_hi - cut_lo;
                cut_lo = cut_hi;
                if (hi < n) {                // the next pass's end, loaded during this pass
                    const int64_t hi2 = hi + chunk < n ? hi + chunk : n;
                    cut_hi = dir[row + (hi2 == n ? nb - 1 : (int)(hi2 / grain))];
                }
            }
            __syncthreads();
            // this wave's slices (trees w, w + 16, ...; at most 16): lane j
            // holds slice j's start and length and, after an inclusive scan,
            // the end of its windows in the wave's window sequence
            const int ntw = T > w ? (T - w + kVoteWaves - 1) / kVoteWaves : 0;
            int64_t sbase = 0;
            int slen = 0, nwin = 0;
            if (lane < ntw) {
                const int t = w + kVoteWaves * lane;
                sbase = tslice[t];
                slen = tlen[t];
                nwin = (slen + kWave - 1) / kWave;
            }
            int wend = nwin;
#pragma unroll
            for (int o = 1; o < kVoteWaves; o <<= 1) {
                const int y = __shfl_up(wend, o);
                if (lane >= o) wend += y;
            }
            const int nwin_all = __builtin_amdgcn_readlane(wend, kVoteWaves - 1);
            for (int r0 = 0; r0 < nwin_all; r0 += kWave) {   // wave-uniform
                // lane s describes window r0 + s: its slice j (the number of
                // slices that end at or before it) and its place in the slice
                const int wi = r0 + lane;
                int j = 0;
#pragma unroll
                for (int jj = 0; jj < kVoteWaves; ++jj) j += __builtin_amdgcn_readlane(wend, jj) <= wi ? 1 : 0;
                const int jc = j < kVoteWaves ? j : kVoteWaves - 1;
                const int64_t b0 = __shfl(sbase, jc);
                const int l0 = __shfl(slen, jc);
                const int k0 = wi - (__shfl(wend, jc) - __shfl(nwin, jc));
                const int64_t first = b0 + (int64_t)k0 * kWave;
                const int first_lo = (int)(uint32_t)first, first_hi = (int)(first >> 32);
                const int avail_v = wi < nwin_all ? min(kWave, l0 - k0 * kWave) : 0;
                const int nw = nwin_all - r0 < kWave ? nwin_all - r0 : kWave;
                // windows g0 .. g0 + 15 of this round into dst: their ids, or
                // -1; a window reads at most 63 entries past its slice, which
                // stay inside the tree's perm row
                auto load = [&](int32_t (&dst)[kDirWindows], int g0) {
#pragma unroll
                    for (int b = 0; b < kDirWindows; ++b) {
                        dst[b] = -1;
                        if (g0 + b < nw) {   // wave-uniform
                            const int64_t f = ((int64_t)__builtin_amdgcn_readlane(first_hi, g0 + b) << 32) |
                                              (uint32_t)__builtin_amdgcn_readlane(first_lo, g0 + b);
                            const int avail = __builtin_amdgcn_readlane(avail_v, g0 + b);
                            const int32_t x = perm[f + lane];
                            if (lane < avail) dst[b] = x;
                        }
                    }
                };
                // count the windows in `cur` while the next 16 load into `nxt`
                auto count = [&](int32_t (&cur)[kDirWindows], int32_t (&nxt)[kDirWindows], int g0) -> bool {
                    const bool more = g0 + kDirWindows < nw;
                    if (more) load(nxt, g0 + kDirWindows);
                    uint32_t ob[kDirWindows];    // nonzero: this occurrence is the v-th
#pragma unroll
                    for (int b = 0; b < kDirWindows; ++b) {
                        // (every id of a slice lies in [lo, hi); the bound keeps
                        // the counter index inside the array regardless)
                        const uint32_t rel = (uint32_t)(cur[b] - lo);
                        ob[b] = 0u;
                        if (cur[b] >= 0 && rel < (uint32_t)chunk) {
                            const uint32_t sh = (rel & 3u) * 8u;
                            ob[b] = ((atomicAdd(&vote_cnt[rel >> 2], 1u << sh) >> sh) & 0xffu) == hit ? 1u : 0u;
                        }
                    }
                    append_batch<true, kDirWindows>(ob, cur, INT32_MAX, &nsel, spare, out, cap32);
                    return more;
                };
                int32_t sa[kDirWindows], sb[kDirWindows];
                load(sa, 0);
                for (int g0 = 0; count(sa, sb, g0) && count(sb, sa, g0 + kDirWindows); g0 += 2 * kDirWindows) {
                }
            }
        }
        __syncthreads();
        if (tid == 0) s_count[q] = nsel < cap ? nsel : (int32_t)cap;
        __syncthreads();                     // shared state is reused by the next query
    }
}

// One run over the queue: every id's first remaining occurrence flips its
// bit (CLEARING: set -> clear, else clear -> set; exactly one occurrence of
// each id finds the old state) and is blanked (~e), or, on the last run,
// elected.  Wave w takes entries w * 256 + 4096 j + [0, 256), four per lane:
// the four loads, then the four atomics, are issued back to back.  Lanes
// without an entry send a no-op atomic to their own spare word, so no branch
// surrounds the atomics.
constexpr int kRerunUnroll = 4;

template <bool CLEARING, int NW>
__device__ __forceinline__ void rerun(uint32_t* map, int32_t* queue, int qn, bool last, int w, int32_t n32,
                                      int* nsel, int* spare, int32_t* out, uint32_t cap) {
    constexpr int R = kRerunUnroll;
    const int lane = lane_id();
    for (int base = w * kWave * R; base < qn; base += NW * kWave * R) {   // wave-uniform trip count
        int32_t e[R];
        uint32_t f[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = base + j * kWave + lane;
            e[j] = i < qn ? queue[i] : -1;
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool live = e[j] >= 0;
            const uint32_t bit = live ? 1u << (e[j] & 31) : 0u;
            uint32_t* word = live ? &map[(uint32_t)e[j] >> 5] : reinterpret_cast<uint32_t*>(spare + lane);
            const uint32_t old = CLEARING ? atomicAnd(word, ~bit) : atomicOr(word, bit);
            f[j] = CLEARING ? (old & bit) : (~old & bit);   // nonzero: the first remaining occurrence
        }
        if (!last) {
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (f[j] != 0u) queue[base + j * kWave + lane] = ~e[j];
        } else {
            append_batch<true, R>(f, e, n32, nsel, spare, out, cap);
        }
    }
}

// LDS: map [map_words] | queue [qcap] | leaf positions [kPosBufs][kMaxT]
//      (int2) | qfill, nsel, 2 unused | kWave spare words
//
// The body serves one query call (MULTI false: `one` describes it, rows are
// its queries) or several calls of one geometry (MULTI true: equal T and
// windows per leaf; row r is query r - row0 of item row_item[r], and the map
// and queue are laid out for the largest index).  Every row's item gives its
// index arrays, n, v and outputs; the map is clear again after every query
// (each query clears the words its index's ids use).  NW waves per
// workgroup: 16 (one workgroup per CU), or 8 where two workgroups' maps and
// queues fit LDS together.
template <int S, bool QUEUE, bool MULTI, int NW>
__device__ __forceinline__ void vote_map_body(const VoteItem& one, const VoteItem* __restrict__ items,
                                              const int32_t* __restrict__ row_item, int64_t nrows, int32_t T,
                                              int32_t wpl, int32_t map_words, int32_t qcap) {
    extern __shared__ __align__(16) uint32_t map_smem[];
    uint32_t* map = map_smem;
    int32_t* queue = reinterpret_cast<int32_t*>(map_smem + map_words);
    int2 (*tpos)[kMaxT] = reinterpret_cast<int2 (*)[kMaxT]>(queue + qcap);
    int* flags = reinterpret_cast<int*>(tpos + kPosBufs);
    int* qfill = flags;
    int* nsel = flags + 1;
    int* spare = flags + 4;   // kWave words, targets of the reservations' idle lanes
    const int tid = (int)threadIdx.x;
    const int w = uniform(tid >> 6);
    const int64_t G = gridDim.x;
    int64_t q = blockIdx.x;
    if (q >= nrows) return;
    // the call that row r belongs to (rows past the last clamp to the last
    // row: their loads stay in range and their values are never used)
    auto item = [&](int64_t r) -> const VoteItem& {
        if constexpr (MULTI) return items[row_item[r < nrows ? r : nrows - 1]];
        else return one;
    };
    int part64, slot_tp;
    slot_table<NW>(w, T, wpl, part64, slot_tp);

    for (int i = tid; i < (map_words >> 2); i += NW * kWave)
        reinterpret_cast<uint4*>(map_smem)[i] = make_uint4(0u, 0u, 0u, 0u);
    // leaf position of tree tid in the query of row r (tid < T): perm index
    // of the leaf's first id, and its length
    auto position = [&](int64_t r, int L) -> int2 {
        const VoteItem& it = item(r);
        const int b = it.off[L];
        return make_int2((int)((int64_t)tid * it.ld) + b, it.off[L + 1] - b);
    };
    auto leaf_of = [&](int64_t r) -> int {
        const VoteItem& it = item(r);
        return it.leaf[(r - it.row0) * T + tid];
    };
    int Lnext = 0;                            // leaf numbers of the query two ahead
    if (tid < T) {
        // every buffer holds in-range positions (empty ones for absent
        // queries): windows are loaded without checking that the query exists
#pragma unroll
        for (int k = 0; k < kPosBufs; ++k) {
            const int64_t qq = q + k * G;
            int2 p = make_int2(0, 0);
            if (k < 2 && qq < nrows) p = position(qq, leaf_of(qq));
            tpos[k][tid] = p;
        }
        if (q + 2 * G < nrows) Lnext = leaf_of(q + 2 * G);
    }
    if (tid == 0) { *qfill = 0; *nsel = 0; }
    __syncthreads();

    // each lane's padding id in a map word of its own (no bank conflicts)
    auto pad4_of = [&](const VoteItem& it) -> uint32_t { return (uint32_t)(it.n + 32 * lane_id()) * 4u; };
    int32_t ids[S], nid[S];
    {
        int first_v, avail_v;
        slot_windows(tpos[0], part64, slot_tp, first_v, avail_v);
        const VoteItem& it = item(q);
        load_windows<S>(ids, it.perm, pad4_of(it), first_v, avail_v);
    }
    int cur = 0;
    // one query: count the windows in `win`, load the next query's into
    // `nxt`; false after the last query of this workgroup
    auto step = [&](int32_t (&win)[S], int32_t (&nxt)[S]) -> bool {
        const int64_t q1 = q + G, q2 = q + 2 * G, q3 = q + 3 * G;
        const int b1 = cur == kPosBufs - 1 ? 0 : cur + 1;
        const int b2 = b1 == kPosBufs - 1 ? 0 : b1 + 1;
        // (past the last query the buffer holds stale or empty positions: the
        // loads stay in range and their values are never used)
        {
            int first_v, avail_v;
            slot_windows(tpos[b1], part64, slot_tp, first_v, avail_v);
            const VoteItem& it1 = item(q1);
            load_windows<S>(nxt, it1.perm, pad4_of(it1), first_v, avail_v);
        }
        int2 pnext = make_int2(0, 0);
        int Lnn = 0;
        if (tid < T) {
            if (q2 < nrows) pnext = position(q2, Lnext);
            if (q3 < nrows) Lnn = leaf_of(q3);
        }
        const VoteItem& it = item(q);
        const int32_t n32 = it.n;
        const int64_t lq = q - it.row0;
        const int32_t cap32 = (int32_t)std::min<int64_t>(it.cap, INT32_MAX);
        int32_t* out = it.s_ids + lq * it.cap;

        // the windows through the map: first occurrences (v = 1: S) or repeats
        // (a batch past slot S - 1 is cut short: its conditions are
        // compile-time constants once the loops are unrolled)
#pragma unroll
        for (int s0 = 0; s0 < S; s0 += kMapBatch) {
            constexpr int NB = kMapBatch;
            uint32_t ob[NB];
            int32_t bid[NB];
#pragma unroll
            for (int g = 0; g < NB; ++g) {
                ob[g] = 0u;
                bid[g] = n32;   // an absent slot: never real, never stored
                if (s0 + g < S) {
                    const int32_t id = win[s0 + g];
                    const uint32_t bit = 1u << (id & 31);
                    ob[g] = atomicOr(&map[id >> 5], bit) & bit;
                    bid[g] = id;
                }
            }
            if constexpr (QUEUE) append_batch<true, NB>(ob, bid, n32, qfill, spare, queue, (uint32_t)qcap);
            else append_batch<false, NB>(ob, bid, n32, nsel, spare, out, (uint32_t)cap32);
        }
        lds_barrier();                        // the map pass of q is complete
        if constexpr (QUEUE) {
            const int qn = min(*qfill, qcap);
            for (int level = 2; level <= it.v; ++level) {
                const bool last = level == it.v;
                // runs 2, 4, ...: the bits of the queued ids start set
                if ((level & 1) == 0) rerun<true, NW>(map, queue, qn, last, w, n32, nsel, spare, out, (uint32_t)cap32);
                else rerun<false, NW>(map, queue, qn, last, w, n32, nsel, spare, out, (uint32_t)cap32);
                lds_barrier();
            }
        }
        // buffer b2 last served the query before q, whose windows are loaded
        if (tid < T && q2 < nrows) tpos[b2][tid] = pnext;
        if (tid == 0) {
            // a queue that overflowed (more reserved than qcap) marks the query
            it.s_count[lq] = *qfill > qcap ? -1 : (*nsel < it.cap ? *nsel : (int32_t)it.cap);
            *qfill = 0;
            *nsel = 0;
        }
        for (int i = tid; i < (it.map_words >> 2); i += NW * kWave)
            reinterpret_cast<uint4*>(map_smem)[i] = make_uint4(0u, 0u, 0u, 0u);
        lds_barrier();
        if (q1 >= nrows) return false;
        Lnext = Lnn;
        cur = b1;
        q = q1;
        return true;
    };
    while (step(ids, nid) && step(nid, ids)) {
    }
}

template <int S, bool QUEUE, int NW>
__global__ __launch_bounds__(NW * kWave) void vote_map_kernel(VoteItem one, int64_t nq, int32_t T, int32_t wpl,
                                                              int32_t map_words, int32_t qcap) {
    vote_map_body<S, QUEUE, false, NW>(one, nullptr, nullptr, nq, T, wpl, map_words, qcap);
}

// several query calls of one geometry in one persistent launch
template <int S, bool QUEUE, int NW>
__global__ __launch_bounds__(NW * kWave) void vote_map_multi_kernel(const VoteItem* __restrict__ items,
                                                                    const int32_t* __restrict__ row_item,
                                                                    int64_t nrows, int32_t T, int32_t wpl,
                                                                    int32_t map_words, int32_t qcap) {
    vote_map_body<S, QUEUE, true, NW>(VoteItem(), items, row_item, nrows, T, wpl, map_words, qcap);
}

// debug: F(x; q) of every listed candidate, by binary search of x in each of
// the query's T leaf lists (independent of the counting kernels)
__global__ __launch_bounds__(256) void vote_counts_kernel(const int32_t* __restrict__ leaf,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ off, int64_t ld,
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
            const int32_t* lst = perm + (int64_t)t * ld;
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

// MRPT_VOTE_KERNEL=0 forces the multi-pass kernel (tuning and tests); by
// default the single-pass kernel runs wherever it fits
// MRPT_VOTE_KERNEL: unset, automatic; 0, the multi-pass kernel (with the
// leaf directory when the index has one; set at build time it also makes the
// build create the directory); 1, the multi-pass kernel without directory
int vote_kernel_override() {
    const char* env = std::getenv("MRPT_VOTE_KERNEL");
    if (!env || !*env) return -1;
    const int x = std::atoi(env);
    return x == 0 || x == 1 ? x : -1;
}

size_t vote_lds_limit() { return (size_t)std::min(lds_per_block_limit(), 160 * 1024); }

// single-pass geometry: map words (ids 0 .. n + 2047: real ids, then the
// empty lanes' ids n + 32 lane), the repeat queue in what LDS has left
struct SingleGeometry {
    bool ok;
    int32_t wpl;
    int64_t slots, map_words, qcap;
    size_t lds;
};

constexpr size_t kMapTail = sizeof(int2) * kPosBufs * kMaxT + 16 + 4 * kWave;   // positions, flags, spare

// the LDS one workgroup of nw waves may take: all of it at 16 waves, half at
// 8 (two workgroups per CU)
size_t vote_lds_budget(int nw) { return nw == kVoteWaves ? vote_lds_limit() : vote_lds_limit() / 2; }

SingleGeometry single_geometry(const mrpt_index* ix, bool queued, int nw = kVoteWaves) {
    SingleGeometry g;
    const size_t limit = vote_lds_budget(nw);
    g.wpl = (ix->max_leaf + kWave - 1) / kWave;
    g.slots = ((int64_t)ix->T * g.wpl + nw - 1) / nw;
    g.map_words = ((ix->n + kVoteSlots * kWave) / 32 + 1 + 3) / 4 * 4;
    const int64_t room = ((int64_t)limit - (int64_t)kMapTail - g.map_words * 4) / 4;
    g.qcap = queued ? std::min<int64_t>(room, (int64_t)ix->T * ix->max_leaf) / 4 * 4 : 0;
    // MRPT_VOTE_QUEUE_CAP lowers the queue capacity (tests: queries then
    // overflow and are recounted by a multi-pass kernel)
    const char* cap_env = std::getenv("MRPT_VOTE_QUEUE_CAP");
    if (queued && cap_env && *cap_env && std::atoll(cap_env) > 0)
        g.qcap = std::min<int64_t>(g.qcap, std::atoll(cap_env) / 4 * 4);
    g.ok = g.slots <= kVoteSlots && ix->n < (int64_t(1) << 24) &&
           (int64_t)ix->T * ix->perm_ld < (int64_t(1) << 30) && room >= 0 && (!queued || g.qcap >= 1024);
    g.lds = (size_t)(g.map_words + g.qcap) * 4 + kMapTail;
    return g;
}

// waves per workgroup of the single-pass kernel for this index: 8 (two
// workgroups per CU, whose fixed per-query costs overlap) when the map, the
// windows and a queue that holds every repeat of a query, or 4,096 of them,
// fit half of LDS; else 16.  pinned: 16, or 8 wherever the 8-wave geometry
// fits at all (its smaller queue may overflow: those queries are recounted)
int single_waves(const mrpt_index* ix, bool queued, int32_t pinned = 0) {
    if (pinned == kVoteWaves) return kVoteWaves;
    const SingleGeometry g8 = single_geometry(ix, queued, 8);
    if (pinned == 8) return g8.ok ? 8 : kVoteWaves;
    const int64_t most = (int64_t)ix->T * ix->max_leaf - ix->n / ((int64_t)1 << ix->depth);
    return g8.ok && (!queued || g8.qcap >= std::min<int64_t>(most, 4096)) ? 8 : kVoteWaves;
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
// recount_only: no single-pass launch; the multi-pass kernel counts again
// the queries marked as overflowed (count -1) by an earlier single-pass one
hipError_t launch_vote_b(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                         int64_t cap, int32_t* s_count, hipStream_t s, const LaunchCfg& cfg,
                         bool recount_only = false) {
    constexpr int per = 32 / B;
    const size_t limit = vote_lds_limit();
    // a pinned choice first (multi-pass: with the directory when there is
    // one), else the environment override, else automatic
    const int mode = recount_only ? -1 : cfg.vote_kernel == 2 ? 0 : cfg.vote_kernel == 1 ? -1 : vote_kernel_override();
    const bool queued = v >= 2;   // repeats are queued and rerun
    const int nw = single_waves(ix, queued, cfg.vote_waves);
    const SingleGeometry sg = single_geometry(ix, queued, nw);
    const bool single = recount_only || (mode < 0 && sg.ok);
    if (single && !recount_only) {
        const int wpl = sg.wpl;
        const int64_t slots = sg.slots, map_words = sg.map_words, qcap = sg.qcap;
        const size_t lds = sg.lds;
        const int64_t grid = std::min<int64_t>(nq, (int64_t)device_cus() * (kVoteWaves / nw));
        VoteItem one;
        one.leaf = leaf;
        one.perm = ix->perm;
        one.off = ix->off;
        one.s_ids = s_ids;
        one.s_count = s_count;
        one.cap = cap;
        one.ld = ix->perm_ld;
        one.row0 = 0;
        one.n = (int32_t)ix->n;
        one.v = v;
        one.map_words = (int32_t)map_words;
#define MRPT_MAP_W(SS, H, NW)                                                                                    \
    do {                                                                                                         \
        (void)hipFuncSetAttribute((const void*)vote_map_kernel<SS, H, NW>,                                       \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                         \
        hipLaunchKernelGGL((vote_map_kernel<SS, H, NW>), dim3((unsigned)grid), dim3((NW) * kWave), lds, s, one,   \
                           nq, ix->T, wpl, (int32_t)map_words, (int32_t)qcap);                                   \
    } while (0)
#define MRPT_MAP(SS, H)                      \
    do {                                     \
        if (nw == 8) MRPT_MAP_W(SS, H, 8);   \
        else MRPT_MAP_W(SS, H, kVoteWaves);  \
    } while (0)
        // the smallest instantiated slot count that holds the windows: every
        // slot costs its loads and map updates even when it is empty
#define MRPT_MAP_S(SS)                                                                                           \
    if (slots <= SS) {                                                                                           \
        if (queued) MRPT_MAP(SS, true);                                                                          \
        else MRPT_MAP(SS, false);                                                                                \
    } else
        MRPT_MAP_S(4) MRPT_MAP_S(8) MRPT_MAP_S(13) MRPT_MAP_S(16) MRPT_MAP_S(20) MRPT_MAP_S(25) MRPT_MAP_S(28) {
            if (queued) MRPT_MAP(kVoteSlots, true);
            else MRPT_MAP(kVoteSlots, false);
        }
#undef MRPT_MAP_S
#undef MRPT_MAP
#undef MRPT_MAP_W
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !queued) return e;
        // a query queues sum(F - 1) <= T * max_leaf - (its first leaf's size)
        // ids; when the queue holds that many, none can overflow
        const int64_t most = (int64_t)ix->T * ix->max_leaf - ix->n / ((int64_t)1 << ix->depth);
        if (qcap >= most) return e;
        // queries whose queue overflowed (count -1) are counted again, multi-pass
    }
    // a recount workgroup checks up to 1024 queries' counts at once and
    // counts those that overflowed; about one workgroup per CU
    const int64_t grid = single ? std::max<int64_t>((nq + kVoteBlock - 1) / kVoteBlock, std::min<int64_t>(nq, device_cus()))
                                : nq;

    if (ix->vdir && mode != 1) {
        // passes on directory boundaries, a multiple of the grain each; one
        // byte per id
        constexpr size_t fixed = kMaxT * (8 + 8 + 4) + 16 + 4 * kWave + 4 * kVoteBlock + 256;   // static LDS
        const int64_t most = (int64_t)((limit - fixed) / 16) * 4 * 4;
        int64_t chunk = most / kDirGrain * kDirGrain;
        if (chunk >= kDirGrain) {
            const int64_t passes = (ix->n + chunk - 1) / chunk;
            chunk = ((ix->n + passes - 1) / passes + kDirGrain - 1) / kDirGrain * kDirGrain;
            const size_t lds = (size_t)chunk;
            (void)hipFuncSetAttribute((const void*)vote_dir_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
            hipLaunchKernelGGL(vote_dir_kernel, dim3((unsigned)grid), dim3(kVoteBlock), lds, s, leaf, ix->perm,
                               ix->off, ix->vdir, ix->nleaf, ix->vdir_nb, kDirGrain, ix->n, ix->perm_ld, ix->T, v,
                               nq, (int32_t)chunk, s_ids, cap, s_count, single ? 1 : 0);
            return hipGetLastError();
        }
    }
    // multi-pass geometry for `fixed` bytes of static LDS: ids per pass, a
    // multiple of 4 words' worth of ids, and the number of passes
    constexpr size_t fixed = kMaxT * 8 + kMaxT * 4 + 16 + 4 * kVoteBlock + 256;   // static LDS, aligned
    int64_t chunk = (int64_t)((limit - fixed) / 16) * 4 * per;
    const int64_t padded = (ix->n + 4 * per - 1) / (4 * per) * (4 * per);
    if (chunk > padded) chunk = padded;
    const int64_t passes = (ix->n + chunk - 1) / chunk;   // same passes, smaller array
    chunk = ((ix->n + passes - 1) / passes + 4 * per - 1) / (4 * per) * (4 * per);
    const size_t multi_lds = (size_t)(chunk / per) * 4;
    (void)hipFuncSetAttribute((const void*)vote_kernel<B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)multi_lds);
    hipLaunchKernelGGL(vote_kernel<B>, dim3((unsigned)grid), dim3(kVoteBlock), multi_lds, s, leaf, ix->perm, ix->off,
                       ix->n, ix->perm_ld, ix->T, v, nq, (int32_t)chunk, s_ids, cap, s_count, single ? 1 : 0);
    return hipGetLastError();
}

// the slot counts the single-pass kernel is instantiated for
constexpr int kSlotClasses[] = {4, 8, 13, 16, 20, 25, 28, kVoteSlots};

}  // namespace

// ((((slot class * 2 + queued) * 2 + eight waves) * 256 + T) * 65536 + windows per leaf
int64_t vote_form(const mrpt_index* ix, int32_t v, const LaunchCfg& cfg) {
    const int mode = cfg.vote_kernel == 2 ? 0 : cfg.vote_kernel == 1 ? -1 : vote_kernel_override();
    const bool queued = v >= 2;
    const int nw = single_waves(ix, queued, cfg.vote_waves);
    const SingleGeometry sg = single_geometry(ix, queued, nw);
    if (mode >= 0 || !sg.ok) return -1;
    int c = 0;
    while (kSlotClasses[c] < sg.slots) ++c;
    return ((((int64_t)c * 2 + (queued ? 1 : 0)) * 2 + (nw == 8 ? 1 : 0)) * 256 + ix->T) * 65536 + sg.wpl;
}

namespace {
int form_waves(int64_t form) { return ((form / 65536 / 256) & 1) != 0 ? 8 : kVoteWaves; }
bool form_queued(int64_t form) { return ((form / 65536 / 256 / 2) & 1) != 0; }
int form_slot_class(int64_t form) { return (int)(form / 65536 / 256 / 4); }
}  // namespace

int32_t vote_map_words(const mrpt_index* ix) { return (int32_t)single_geometry(ix, false).map_words; }

int64_t vote_most_queued(const mrpt_index* ix) {
    return (int64_t)ix->T * ix->max_leaf - ix->n / ((int64_t)1 << ix->depth);
}

int64_t vote_multi_qcap(int64_t form, int32_t map_words, int64_t most_occurrences) {
    const int64_t room = ((int64_t)vote_lds_budget(form_waves(form)) - (int64_t)kMapTail - (int64_t)map_words * 4) / 4;
    int64_t qcap = std::min<int64_t>(room, most_occurrences) / 4 * 4;
    const char* cap_env = std::getenv("MRPT_VOTE_QUEUE_CAP");
    if (cap_env && *cap_env && std::atoll(cap_env) > 0) qcap = std::min<int64_t>(qcap, std::atoll(cap_env) / 4 * 4);
    return qcap >= 1024 ? qcap : -1;
}

hipError_t launch_vote_multi(int64_t form, int32_t map_words, int64_t qcap, const VoteItem* items,
                             const int32_t* row_item, int64_t nrows, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    const int32_t wpl = (int32_t)(form % 65536);
    const int32_t T = (int32_t)((form / 65536) % 256);
    const int nw = form_waves(form);
    const bool queued = form_queued(form);
    const int c = form_slot_class(form);
    const size_t lds = (size_t)(map_words + qcap) * 4 + kMapTail;
    const int64_t grid = std::min<int64_t>(nrows, (int64_t)device_cus() * (kVoteWaves / nw));
#define MRPT_MAPM_W(SS, H, NW)                                                                               \
    do {                                                                                                     \
        (void)hipFuncSetAttribute((const void*)vote_map_multi_kernel<SS, H, NW>,                             \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                     \
        hipLaunchKernelGGL((vote_map_multi_kernel<SS, H, NW>), dim3((unsigned)grid), dim3((NW) * kWave), lds, \
                           s, items, row_item, nrows, T, wpl, map_words, (int32_t)qcap);                     \
    } while (0)
#define MRPT_MAPM(SS, H)                      \
    do {                                      \
        if (nw == 8) MRPT_MAPM_W(SS, H, 8);   \
        else MRPT_MAPM_W(SS, H, kVoteWaves);  \
    } while (0)
#define MRPT_MAPM_C(CI, SS)                       \
    case CI:                                      \
        if (queued) MRPT_MAPM(SS, true);          \
        else MRPT_MAPM(SS, false);                \
        break;
    switch (c) {
        MRPT_MAPM_C(0, 4) MRPT_MAPM_C(1, 8) MRPT_MAPM_C(2, 13) MRPT_MAPM_C(3, 16) MRPT_MAPM_C(4, 20)
        MRPT_MAPM_C(5, 25) MRPT_MAPM_C(6, 28) default:
            if (queued) MRPT_MAPM(kVoteSlots, true);
            else MRPT_MAPM(kVoteSlots, false);
    }
#undef MRPT_MAPM_C
#undef MRPT_MAPM
#undef MRPT_MAPM_W
    return hipGetLastError();
}

hipError_t launch_vote_recount(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                               int64_t cap, int32_t* s_count, hipStream_t s) {
    if (nq == 0 || v == 1) return hipSuccess;
    const LaunchCfg cfg;
    if (v <= 3) return launch_vote_b<2>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg, true);
    if (v <= 15) return launch_vote_b<4>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg, true);
    return launch_vote_b<8>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg, true);
}

hipError_t launch_vote(const mrpt_index* ix, const int32_t* leaf, int64_t nq, int32_t v, int32_t* s_ids,
                       int64_t cap, int32_t* s_count, hipStream_t s, const LaunchCfg& cfg) {
    if (nq == 0) return hipSuccess;
    if (v == 1) return launch_vote_b<1>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg);
    if (v <= 3) return launch_vote_b<2>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg);
    if (v <= 15) return launch_vote_b<4>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg);
    return launch_vote_b<8>(ix, leaf, nq, v, s_ids, cap, s_count, s, cfg);
}

hipError_t build_vote_directory(mrpt_index* ix, int64_t* tally) {
    // the multi-pass kernels serve this index when the single-pass one cannot
    // (or when the multi-pass kernel is forced); one pass needs no directory
    const bool multi = vote_kernel_override() == 0 || !single_geometry(ix, false).ok ||
                       !single_geometry(ix, true).ok;
    if (!multi || ix->n <= kDirGrain) return hipSuccess;
    const int32_t nb = (int32_t)((ix->n + kDirGrain - 1) / kDirGrain + 1);
    const int64_t total = (int64_t)ix->T * ix->nleaf * nb;
    hipError_t e = hipMalloc((void**)&ix->vdir, (size_t)total * sizeof(int32_t));
    if (e != hipSuccess) {
        ix->vdir = nullptr;
        return e;
    }
    if (tally) *tally += total * (int64_t)sizeof(int32_t);
    ix->vdir_nb = nb;
    const unsigned threads = 256;
    hipLaunchKernelGGL(vote_dir_build_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0,
                       nullptr, ix->perm, ix->off, ix->n, ix->perm_ld, ix->nleaf, nb, kDirGrain, total, ix->vdir);
    return hipGetLastError();
}

hipError_t launch_vote_counts(const mrpt_index* ix, const int32_t* leaf, int64_t nq, const int32_t* s_ids,
                              int64_t cap, const int32_t* s_count, uint8_t* s_votes, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(vote_counts_kernel, dim3((unsigned)nq), dim3(256), 0, s, leaf, ix->perm, ix->off, ix->perm_ld,
                       ix->T, s_ids, cap, s_count, s_votes);
    return hipGetLastError();
}

hipError_t launch_copy_counts(const int32_t* src, int64_t nq, int32_t* dst, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_counts_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, src, nq, dst);
    return hipGetLastError();
}

}  // namespace mrpt
