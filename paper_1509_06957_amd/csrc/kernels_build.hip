// Index build on the GPU (Alg. 1 grow_trees, Alg. 2 grow_tree; Sec. II-A
// median splits, Sec. II-C one projection vector per level).
//
// Trees are grown in groups.  For a group the data are projected onto all of
// its vectors at once (project_kernel, the float32 fused multiply-add chain
// in ascending feature order that the queries use), then level by level
// every node of every tree of the group is cut by rank: the ceil(m/2)
// smallest of the node's keys (projection, id) form the left child, the rest
// the right one.  A key is a 64-bit word, the projection's order bits
// above the id (idb = bits of n - 1 of them), so the order of keys is the
// order (projection, id), and all keys of a tree are distinct.  The split
// stored for queries is the largest left value for odd m and the float32
// midpoint of the two middle values for even m.  Finally each leaf is sorted
// by id.
//
// The cut of a level needs only the ceil(m/2)-th key of each node, not the
// order inside it: a radix select finds that key digit by digit (8 bits per
// pass, from the top: a histogram of the current digit over the keys that
// match the digits found so far, then the bin that holds the wanted rank),
// and one partition pass moves the keys at or below it to the node's front.
// A node stops early when the wanted rank is the last key of its bin: the
// bin then goes left whole, and its lower digits need no pass.
// Nodes of more than kCutSmallMax keys are cut by many workgroups each
// (global histograms, one pass per digit); smaller ones by one workgroup
// per node with its keys in LDS.  The order inside a child is left to the
// atomics that place the keys: nothing depends on it, since the next level
// cuts by rank again and the leaves end sorted by id.  A segmented radix
// sort (rocPRIM) of each level, which orders every node completely, is
// kept as the alternative (MRPT_BUILD_SORT=1); both give the same trees.
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <cstdlib>
#include <vector>

#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

using dev::kWave;

// monotone map of a float32 (zero canonicalised to +0) onto uint32 order
__device__ __forceinline__ uint32_t order_bits(float p) {
    const uint32_t u = __float_as_uint(p == 0.0f ? 0.0f : p);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_order_bits(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// keys of level lv: tree tl = blockIdx.y of the group, position i (the id at
// that position after the previous level's sort, or i itself at level 0)
__global__ void level_keys_kernel(const float* __restrict__ P, int32_t depth, int32_t lv, int64_t n, int32_t idb,
                                  const uint64_t* __restrict__ prev, uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t tl = blockIdx.y;
    const int64_t at = tl * n + i;
    const uint32_t id = prev ? (uint32_t)(prev[at] & ((uint64_t(1) << idb) - 1)) : (uint32_t)i;
    const float p = P[(tl * depth + lv) * n + id];
    keys[at] = ((uint64_t)order_bits(p) << idb) | id;
}

// split of node s of level lv in tree tl = blockIdx.y, from its sorted keys
__global__ void level_splits_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ node_off,
                                    int32_t lv, int64_t n, int32_t idb, int64_t nsplit, float* __restrict__ splits) {
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int nodes = 1 << lv;
    if (s >= nodes) return;
    const int64_t tl = blockIdx.y;
    const int64_t b = node_off[s], m = node_off[s + 1] - b;
    const int64_t nl = (m + 1) / 2;
    const uint64_t* k = keys + tl * n + b;
    const float left_max = from_order_bits((uint32_t)(k[nl - 1] >> idb));
    float split = left_max;
    if ((m & 1) == 0) {
        const float right_min = from_order_bits((uint32_t)(k[nl] >> idb));
        const float sum = left_max + right_min;
        split = sum * 0.5f;
    }
    splits[tl * nsplit + (nodes - 1) + s] = split;
}

// ids of the sorted keys into the perm rows of the group (row stride ld)
__global__ void perm_rows_kernel(const uint64_t* __restrict__ keys, int64_t n, int32_t idb, int64_t ld,
                                 int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t tl = blockIdx.y;
    perm[tl * ld + i] = (int32_t)(keys[tl * n + i] & ((uint64_t(1) << idb) - 1));
}

// identity ids (depth 0: one leaf holding every point, ascending)
__global__ void iota_keys_kernel(int64_t n, uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[(int64_t)blockIdx.y * n + i] = (uint64_t)i;
}

// ---------------------------------------------------------------------------
// Cut by rank: radix select of the ceil(m/2)-th key of every node, then a
// partition.  A node is (tree tl, node j of the level): positions
// [node_off[j], node_off[j + 1]) of row tl of the key array, global node
// index tl * nodes + j, so the nodes of all trees are consecutive ranges of
// the group's key array, in the order of their global index.
// ---------------------------------------------------------------------------
constexpr int kCutSmallMax = 8192;   // nodes up to this size: one workgroup, keys in LDS
constexpr int kCutChunk = 4096;      // keys per workgroup of the large-node passes
constexpr int kCutThreads = 256;
constexpr int kCutDigit = 8;         // bits per radix-select pass
constexpr int kCutBins = 1 << kCutDigit;

// per node: the select's prefix (digits found so far, in place) and the rank
// still wanted among the keys that match it; then the partition's fills and
// the smallest key of the right child
struct CutNode {
    unsigned long long prefix;
    unsigned long long krem;
    unsigned long long fill_l, fill_r;
    unsigned long long right_min;
    unsigned long long left_max;
    int32_t shift;               // digits at and above it decide the cut; -1 while open
    int32_t pad_;
};

// the largest / smallest value over the wave's lanes
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int o) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long t = shfl_xor_u64(v, o);
        v = t > v ? t : v;
    }
    return v;
}
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long t = shfl_xor_u64(v, o);
        v = t < v ? t : v;
    }
    return v;
}

__global__ void cut_init_kernel(CutNode* __restrict__ st, int64_t gnodes, const int64_t* __restrict__ node_off,
                                int32_t nodes) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= gnodes) return;
    const int j = (int)(g % nodes);
    const int64_t m = node_off[j + 1] - node_off[j];
    st[g].prefix = 0ull;
    st[g].krem = (unsigned long long)((m + 1) / 2);
    st[g].fill_l = 0ull;
    st[g].fill_r = 0ull;
    st[g].right_min = ~0ull;
    st[g].left_max = 0ull;
    st[g].shift = -1;
}

// the first node of the chunk starting at position p0 of the key array, and
// the first position past it (every large node is longer than a chunk, so a
// chunk meets at most two nodes: g0 and g0 + 1)
__device__ __forceinline__ void chunk_nodes(int64_t p0, int64_t n, const int64_t* __restrict__ node_off,
                                            int32_t nodes, int64_t& g0, int64_t& b1) {
    const int64_t tl = p0 / n, pos = p0 - tl * n;
    int lo = 0, hi = nodes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (node_off[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    g0 = tl * nodes + lo;
    b1 = tl * n + node_off[lo + 1];
}

// the histogram of the digit [shift, top) over the keys whose bits at and
// above `top` equal their node's prefix
__global__ __launch_bounds__(kCutThreads) void cut_hist_kernel(const uint64_t* __restrict__ keys, int64_t total,
                                                                int64_t n, const int64_t* __restrict__ node_off,
                                                                int32_t nodes, const CutNode* __restrict__ st,
                                                                int32_t top, int32_t shift,
                                                                uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[2][kCutBins];
    __shared__ int64_t s_g0, s_b1;
    const int tid = (int)threadIdx.x;
    for (int i = tid; i < 2 * kCutBins; i += kCutThreads) h[i / kCutBins][i % kCutBins] = 0u;
    const int64_t p0 = (int64_t)blockIdx.x * kCutChunk;
    if (tid == 0) {
        int64_t g0, b1;
        chunk_nodes(p0, n, node_off, nodes, g0, b1);
        s_g0 = g0;
        s_b1 = b1;
    }
    __syncthreads();
    const int64_t g0 = s_g0, b1 = s_b1;
    const bool two = b1 < total && b1 < p0 + kCutChunk;
    // a decided node takes no more histograms: its keys are not read
    const bool open0 = st[g0].shift < 0;
    const bool open1 = two && st[g0 + 1].shift < 0;
    if (!open0 && !open1) return;
    const uint64_t pre0 = st[g0].prefix;
    const uint64_t pre1 = two ? st[g0 + 1].prefix : 0ull;
    const uint32_t mask = (1u << (top - shift)) - 1u;
    const int64_t pbeg = open0 ? p0 : b1;                       // the open nodes' positions
    const int64_t pend = open1 ? p0 + kCutChunk : (b1 < p0 + kCutChunk ? b1 : p0 + kCutChunk);
    for (int e = 0; e < kCutChunk / kCutThreads; ++e) {
        const int64_t p = p0 + e * kCutThreads + tid;
        if (p >= total) break;
        if (p < pbeg || p >= pend) continue;
        const uint64_t k = keys[p];
        const int slot = p >= b1 ? 1 : 0;
        if (((k ^ (slot ? pre1 : pre0)) >> top) == 0) atomicAdd(&h[slot][(uint32_t)(k >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int i = tid; i < 2 * kCutBins; i += kCutThreads) {
        const int slot = i / kCutBins;
        const uint32_t c = h[slot][i % kCutBins];
        if (c != 0u) atomicAdd(&hist[(g0 + slot) * kCutBins + i % kCutBins], c);
    }
}

// one wave picks a digit: the bin of h (kCutBins counts) that holds rank
// *krem, whose count below is taken off *krem and whose value goes into
// *prefix at `shift`; h is cleared for the next pass.  When the wanted rank
// is the bin's last key, every key of the bin goes left and the cut is
// decided: *done = shift (the node's keys compare with the prefix from
// that bit up; the lower digits need no more passes)
__device__ __forceinline__ void pick_digit(uint32_t* h, unsigned long long* prefix, unsigned long long* krem,
                                           int32_t shift, int32_t* done) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    constexpr int per = kCutBins / kWave;
    uint32_t c[per];
    uint32_t sum = 0u;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        c[j] = h[lane * per + j];
        sum += c[j];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    const uint64_t want = *krem;
    const uint32_t excl = incl - sum;
    if ((uint64_t)excl < want && want <= (uint64_t)incl) {
        uint32_t below = excl;
        int b = per - 1;
#pragma unroll
        for (int j = 0; j < per; ++j) {
            if (below + c[j] >= want) {
                b = j;
                break;
            }
            below += c[j];
        }
        *krem = want - below;
        *prefix |= (unsigned long long)(lane * per + b) << shift;
        if (c[b] == want - below) *done = shift;
    }
#pragma unroll
    for (int j = 0; j < per; ++j) h[lane * per + j] = 0u;
}

__global__ __launch_bounds__(kWave) void cut_pick_kernel(uint32_t* __restrict__ hist, CutNode* __restrict__ st,
                                                          int32_t shift) {
    const int64_t g = blockIdx.x;
    if (st[g].shift >= 0) return;   // decided: its bins stay zero
    pick_digit(hist + g * kCutBins, &st[g].prefix, &st[g].krem, shift, &st[g].shift);
}

// the partition of large nodes: keys at or below the node's selected key
// (its prefix, complete after the last pass) to the front ceil(m/2)
// places, the rest behind them; the right child's smallest key is kept
__global__ __launch_bounds__(kCutThreads) void cut_partition_kernel(const uint64_t* __restrict__ keys, int64_t total,
                                                                     int64_t n, const int64_t* __restrict__ node_off,
                                                                     int32_t nodes, CutNode* __restrict__ st,
                                                                     uint64_t* __restrict__ out) {
    constexpr int E = kCutChunk / kCutThreads;
    __shared__ uint32_t cnt[2][2];
    __shared__ unsigned long long base[2][2], rmin[2], lmax[2];
    __shared__ int64_t s_g0, s_b1;
    const int tid = (int)threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * kCutChunk;
    if (tid == 0) {
        int64_t g0, b1;
        chunk_nodes(p0, n, node_off, nodes, g0, b1);
        s_g0 = g0;
        s_b1 = b1;
        cnt[0][0] = cnt[0][1] = cnt[1][0] = cnt[1][1] = 0u;
        rmin[0] = rmin[1] = ~0ull;
        lmax[0] = lmax[1] = 0ull;
    }
    __syncthreads();
    const int64_t g0 = s_g0, b1 = s_b1;
    const bool two = b1 < total && b1 < p0 + kCutChunk;
    // a key goes right when its bits from the node's deciding digit up
    // exceed the selected prefix's
    const int r0 = st[g0].shift < 0 ? 0 : st[g0].shift;
    const int r1 = two ? (st[g0 + 1].shift < 0 ? 0 : st[g0 + 1].shift) : 0;
    const uint64_t t0 = st[g0].prefix >> r0;
    const uint64_t t1 = two ? st[g0 + 1].prefix >> r1 : 0ull;
    uint64_t k[E];
    uint32_t at[E];
    unsigned long long mn[2] = {~0ull, ~0ull}, mx[2] = {0ull, 0ull};   // per slot, this thread's keys
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t p = p0 + e * kCutThreads + tid;
        at[e] = 0u;
        k[e] = 0ull;
        if (p < total) {
            k[e] = keys[p];
            const int slot = p >= b1 ? 1 : 0;
            const bool right = (k[e] >> (slot ? r1 : r0)) > (slot ? t1 : t0);
            at[e] = atomicAdd(&cnt[slot][right ? 1 : 0], 1u);
            if (right) mn[slot] = k[e] < mn[slot] ? k[e] : mn[slot];
            else mx[slot] = k[e] > mx[slot] ? k[e] : mx[slot];
        }
    }
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
        const unsigned long long wmn = wave_min_u64(mn[slot]), wmx = wave_max_u64(mx[slot]);
        if ((tid & (kWave - 1)) == 0) {
            if (wmn != ~0ull) atomicMin(&rmin[slot], wmn);
            if (wmx != 0ull) atomicMax(&lmax[slot], wmx);
        }
    }
    __syncthreads();
    if (tid < 4) {
        const int slot = tid >> 1, side = tid & 1;
        if (slot == 0 || two)
            base[slot][side] = cnt[slot][side] == 0u
                                   ? 0ull
                                   : atomicAdd(side ? &st[g0 + slot].fill_r : &st[g0 + slot].fill_l,
                                               (unsigned long long)cnt[slot][side]);
    } else if (tid < 6) {
        const int slot = tid - 4;
        if ((slot == 0 || two) && rmin[slot] != ~0ull) atomicMin(&st[g0 + slot].right_min, rmin[slot]);
    } else if (tid < 8) {
        const int slot = tid - 6;
        if ((slot == 0 || two) && cnt[slot][0] != 0u) atomicMax(&st[g0 + slot].left_max, lmax[slot]);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t p = p0 + e * kCutThreads + tid;
        if (p < total) {
            const int slot = p >= b1 ? 1 : 0;
            const int64_t g = g0 + slot;
            const int64_t tl = g / nodes;
            const int j = (int)(g - tl * nodes);
            const int64_t lo = node_off[j], m = node_off[j + 1] - lo;
            const bool right = (k[e] >> (slot ? r1 : r0)) > (slot ? t1 : t0);
            const int64_t place = (right ? (m + 1) / 2 + (int64_t)base[slot][1] : (int64_t)base[slot][0]) + at[e];
            // exactly ceil(m/2) keys are at or below the selected one (the
            // keys of a tree are distinct), so every place is inside the
            // node; the test only keeps a wrong selection inside it too
            if (place < m) out[tl * n + lo + place] = k[e];
        }
    }
}

// split of every node from its selected key and its right child's smallest
// key (the same float32 arithmetic as the split from sorted keys)
__global__ void cut_splits_kernel(const CutNode* __restrict__ st, int64_t gnodes, const int64_t* __restrict__ node_off,
                                  int32_t nodes, int32_t lv, int32_t idb, int64_t nsplit,
                                  float* __restrict__ splits) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= gnodes) return;
    const int64_t tl = g / nodes;
    const int j = (int)(g - tl * nodes);
    const int64_t m = node_off[j + 1] - node_off[j];
    const float left_max = from_order_bits((uint32_t)(st[g].left_max >> idb));
    float split = left_max;
    if ((m & 1) == 0) {
        const float right_min = from_order_bits((uint32_t)(st[g].right_min >> idb));
        const float sum = left_max + right_min;
        split = sum * 0.5f;
    }
    splits[tl * nsplit + ((1 << lv) - 1) + j] = split;
}

// a small node (at most kCutSmallMax keys) cut by one workgroup of NT
// threads: its keys in LDS, the select's passes over them there, the
// partition written out, the split stored
template <int NT>
__global__ __launch_bounds__(NT) void cut_small_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                       const int64_t* __restrict__ node_off, int32_t nodes,
                                                       int32_t lv, int32_t top_bits, int32_t idb, int64_t nsplit,
                                                       uint64_t* __restrict__ out, float* __restrict__ splits) {
    extern __shared__ unsigned long long kv[];
    __shared__ uint32_t h[kCutBins];
    __shared__ unsigned long long s_prefix, s_krem, s_rmin, s_lmax;
    __shared__ uint32_t s_cnt[2];
    __shared__ int32_t s_shift;
    const int tid = (int)threadIdx.x;
    const int64_t g = blockIdx.x;
    const int64_t tl = g / nodes;
    const int j = (int)(g - tl * nodes);
    const int64_t lo = node_off[j];
    const int m = (int)(node_off[j + 1] - lo);
    const uint64_t* src = keys + tl * n + lo;
    for (int i = tid; i < m; i += NT) kv[i] = src[i];
    for (int i = tid; i < kCutBins; i += NT) h[i] = 0u;
    if (tid == 0) {
        s_prefix = 0ull;
        s_krem = (unsigned long long)((m + 1) / 2);
        s_rmin = ~0ull;
        s_lmax = 0ull;
        s_cnt[0] = s_cnt[1] = 0u;
        s_shift = -1;
    }
    __syncthreads();
    for (int top = top_bits; top > 0 && s_shift < 0; top -= kCutDigit) {
        const int shift = top > kCutDigit ? top - kCutDigit : 0;
        const uint32_t mask = (1u << (top - shift)) - 1u;
        const uint64_t pre = s_prefix;
        for (int i = tid; i < m; i += NT) {
            const uint64_t k = kv[i];
            if (((k ^ pre) >> top) == 0) atomicAdd(&h[(uint32_t)(k >> shift) & mask], 1u);
        }
        __syncthreads();
        if (tid < kWave) pick_digit(h, &s_prefix, &s_krem, shift, &s_shift);
        __syncthreads();
    }
    // a key goes left when its bits from the deciding digit up are at most
    // the selected prefix's (all bits when every pass ran)
    const int rs = s_shift < 0 ? 0 : s_shift;
    const uint64_t sel = s_prefix >> rs;
    const int nl = (m + 1) / 2;
    uint64_t* dst = out + tl * n + lo;
    unsigned long long mn = ~0ull, mx = 0ull;   // this thread's keys: smallest right, largest left
    for (int i = tid; i < m; i += NT) {
        const uint64_t k = kv[i];
        // (places stay inside the node even for a wrong selection)
        if ((k >> rs) <= sel) {
            const uint32_t at = atomicAdd(&s_cnt[0], 1u);
            if ((int)at < nl) dst[at] = k;
            mx = k > mx ? k : mx;
        } else {
            const uint32_t at = atomicAdd(&s_cnt[1], 1u);
            if ((int)at < m - nl) dst[nl + at] = k;
            mn = k < mn ? k : mn;
        }
    }
    mn = wave_min_u64(mn);
    mx = wave_max_u64(mx);
    if ((tid & (kWave - 1)) == 0) {
        if (mn != ~0ull) atomicMin(&s_rmin, mn);
        if (mx != 0ull) atomicMax(&s_lmax, mx);
    }
    __syncthreads();
    if (tid == 0) {
        const float left_max = from_order_bits((uint32_t)(s_lmax >> idb));
        float split = left_max;
        if ((m & 1) == 0) {
            const float right_min = from_order_bits((uint32_t)(s_rmin >> idb));
            const float sum = left_max + right_min;
            split = sum * 0.5f;
        }
        splits[tl * nsplit + ((1 << lv) - 1) + j] = split;
    }
}

}  // namespace

size_t device_build_bytes_per_tree(int64_t n, int32_t depth) {
    return (size_t)n * (4 * (size_t)std::max(depth, 1) + 2 * sizeof(uint64_t));
}

hipError_t grow_trees_device(mrpt_index* ix, int32_t t0, int32_t g, const std::vector<std::vector<int64_t>>& level_off,
                             float* P, uint64_t* keys_a, uint64_t* keys_b, void*& temp, size_t& temp_bytes,
                             int32_t* seg_off, int64_t* node_off, hipStream_t s) {
    const int64_t n = ix->n;
    const int32_t depth = ix->depth;
    const int64_t nsplit = ((int64_t)1 << depth) - 1;
    const unsigned threads = 256;
    const dim3 rows((unsigned)((n + threads - 1) / threads), (unsigned)g);
    // bits of the largest id (at least 1): the keys' low field
    int32_t idb = 1;
    while (idb < 31 && ((n - 1) >> idb) != 0) ++idb;
    hipError_t e;
    if ((e = launch_project(ix, ix->X, n, t0 * depth, g * depth, P, s)) != hipSuccess) return e;

    // temporary device memory of at least `need` bytes in `temp` (grown
    // after the stream has drained, never shrunk)
    auto ensure_temp = [&](size_t need) -> hipError_t {
        if (need <= temp_bytes) return hipSuccess;
        hipError_t err;
        if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
        if (temp && (err = hipFree(temp)) != hipSuccess) return err;
        temp = nullptr;
        temp_bytes = 0;
        if ((err = hipMalloc(&temp, need)) != hipSuccess) return err;
        temp_bytes = need;
        return hipSuccess;
    };

    // segmented sort over the nodes of every tree of the group (offsets into
    // the group's key array); level `lv` = depth sorts leaves by id
    auto sort_level = [&](int lv, const uint64_t* in, uint64_t* out, unsigned begin_bit,
                          unsigned end_bit) -> hipError_t {
        const std::vector<int64_t>& lo = level_off[lv];
        const int nodes = 1 << lv;
        std::vector<int32_t> off((size_t)g * nodes + 1);
        for (int32_t tl = 0; tl < g; ++tl)
            for (int j = 0; j < nodes; ++j) off[(size_t)tl * nodes + j] = (int32_t)(tl * n + lo[j]);
        off[(size_t)g * nodes] = (int32_t)(g * n);
        hipError_t err = hipMemcpy(seg_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (err != hipSuccess) return err;
        size_t need = 0;
        err = rocprim::segmented_radix_sort_keys(nullptr, need, in, out, (unsigned)(g * n), (unsigned)(g * nodes),
                                                 seg_off, seg_off + 1, begin_bit, end_bit, s);
        if (err != hipSuccess) return err;
        if ((err = ensure_temp(need)) != hipSuccess) return err;
        return rocprim::segmented_radix_sort_keys(temp, need, in, out, (unsigned)(g * n), (unsigned)(g * nodes),
                                                  seg_off, seg_off + 1, begin_bit, end_bit, s);
    };

    // the cut of level lv by rank (node offsets already in node_off): keys
    // of `in` partitioned into `out`, splits stored; false when the level's
    // shape is outside what the select kernels assume (then it is sorted)
    const int top_bits = 32 + idb;
    float* tree_splits = ix->splits + (int64_t)t0 * nsplit;
    auto cut_level = [&](int lv, const uint64_t* in, uint64_t* out, bool* done) -> hipError_t {
        *done = false;
        const std::vector<int64_t>& lo = level_off[lv];
        const int nodes = 1 << lv;
        const int64_t gnodes = (int64_t)g * nodes, total = (int64_t)g * n;
        int64_t minm = n, maxm = 0;
        for (int j = 0; j < nodes; ++j) {
            minm = std::min<int64_t>(minm, lo[j + 1] - lo[j]);
            maxm = std::max<int64_t>(maxm, lo[j + 1] - lo[j]);
        }
        hipError_t err;
        const unsigned cut_threads = (unsigned)kCutThreads;
        const dim3 node_grid((unsigned)((gnodes + cut_threads - 1) / cut_threads));
        if (maxm > kCutSmallMax) {
            if (minm <= kCutChunk) return hipSuccess;
            const size_t st_bytes = ((size_t)gnodes * sizeof(CutNode) + 255) / 256 * 256;
            if ((err = ensure_temp(st_bytes + (size_t)gnodes * kCutBins * sizeof(uint32_t))) != hipSuccess)
                return err;
            CutNode* st = static_cast<CutNode*>(temp);
            uint32_t* hist = reinterpret_cast<uint32_t*>(static_cast<char*>(temp) + st_bytes);
            if ((err = hipMemsetAsync(hist, 0, (size_t)gnodes * kCutBins * sizeof(uint32_t), s)) != hipSuccess)
                return err;
            hipLaunchKernelGGL(cut_init_kernel, node_grid, dim3(cut_threads), 0, s, st, gnodes, node_off, nodes);
            const dim3 chunks((unsigned)((total + kCutChunk - 1) / kCutChunk));
            for (int top = top_bits; top > 0; top -= kCutDigit) {
                const int shift = top > kCutDigit ? top - kCutDigit : 0;
                hipLaunchKernelGGL(cut_hist_kernel, chunks, dim3(cut_threads), 0, s, in, total, n, node_off, nodes,
                                   st, top, shift, hist);
                hipLaunchKernelGGL(cut_pick_kernel, dim3((unsigned)gnodes), dim3(kWave), 0, s, hist, st, shift);
            }
            hipLaunchKernelGGL(cut_partition_kernel, chunks, dim3(cut_threads), 0, s, in, total, n, node_off, nodes,
                               st, out);
            hipLaunchKernelGGL(cut_splits_kernel, node_grid, dim3(cut_threads), 0, s, st, gnodes, node_off, nodes,
                               lv, idb, nsplit, tree_splits);
        } else {
            const int nt = maxm <= 1024 ? 64 : maxm <= 4096 ? 256 : 512;
            if (gnodes * nt >= (int64_t(1) << 32)) return hipSuccess;
            const size_t lds = (size_t)maxm * sizeof(uint64_t);
#define MRPT_CUT_SMALL(NT)                                                                                     \
    do {                                                                                                       \
        (void)hipFuncSetAttribute((const void*)cut_small_kernel<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                  (int)lds);                                                                   \
        hipLaunchKernelGGL(cut_small_kernel<NT>, dim3((unsigned)gnodes), dim3(NT), lds, s, in, n, node_off, nodes, \
                           lv, top_bits, idb, nsplit, out, tree_splits);                                        \
    } while (0)
            if (nt == 64) MRPT_CUT_SMALL(64);
            else if (nt == 256) MRPT_CUT_SMALL(256);
            else MRPT_CUT_SMALL(512);
#undef MRPT_CUT_SMALL
        }
        *done = true;
        return hipGetLastError();
    };

    // MRPT_BUILD_SORT=1: every level by the segmented sort
    const char* sort_env = std::getenv("MRPT_BUILD_SORT");
    const bool sort_levels = sort_env && std::atoi(sort_env) == 1;

    // each level: keys from the previous level's cut keys (in keys_b) into
    // keys_a, then the cut of keys_a back into keys_b
    for (int32_t lv = 0; lv < depth; ++lv) {
        hipLaunchKernelGGL(level_keys_kernel, rows, dim3(threads), 0, s, P, depth, lv, n, idb,
                           lv == 0 ? (const uint64_t*)nullptr : keys_b, keys_a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const std::vector<int64_t>& lo = level_off[lv];
        if ((e = hipMemcpy(node_off, lo.data(), lo.size() * sizeof(int64_t), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return e;
        bool cut = false;
        if (!sort_levels && (e = cut_level(lv, keys_a, keys_b, &cut)) != hipSuccess) return e;
        if (cut) continue;
        if ((e = sort_level(lv, keys_a, keys_b, 0, 32 + (unsigned)idb)) != hipSuccess) return e;
        const int nodes = 1 << lv;
        hipLaunchKernelGGL(level_splits_kernel, dim3((unsigned)((nodes + threads - 1) / threads), (unsigned)g),
                           dim3(threads), 0, s, keys_b, node_off, lv, n, idb, nsplit, tree_splits);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const uint64_t* ids = keys_a;
    if (depth == 0) {
        hipLaunchKernelGGL(iota_keys_kernel, rows, dim3(threads), 0, s, n, keys_a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        // leaves: ids ascending (the key's low idb bits)
        if ((e = sort_level(depth, keys_b, keys_a, 0, (unsigned)idb)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(perm_rows_kernel, rows, dim3(threads), 0, s, ids, n, idb, ix->perm_ld,
                       ix->perm + (int64_t)t0 * ix->perm_ld);
    return hipGetLastError();
}

}  // namespace mrpt
