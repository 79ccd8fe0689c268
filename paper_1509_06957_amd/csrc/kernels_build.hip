// Index build on the GPU (Alg. 1 grow_trees, Alg. 2 grow_tree; Sec. II-A
// median splits, Sec. II-C one projection vector per level).
//
// Trees are grown in groups.  For a group the data are projected onto all of
// its vectors at once (project_kernel, the float32 fused multiply-add chain
// in ascending feature order that the queries use), then level by level
// every node of every tree of the group is cut by rank: the node's keys
// (projection, id) are sorted within the node and its first ceil(m/2) keys
// form the left child.  A key is a 64-bit word, the projection's order bits
// above the id (idb = bits of n - 1 of them), so one segmented radix sort of
// its 32 + idb low bits over all nodes of the group does the cut of a whole
// level, ties broken by id.  The split stored for queries
// is the largest left value for odd m and the float32 midpoint of the two
// middle values for even m.  Finally each leaf is sorted by id.
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <vector>

#include "device_common.h"
#include "mrpt_internal.h"

namespace mrpt {
namespace {

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
        if (need > temp_bytes) {
            if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
            if (temp && (err = hipFree(temp)) != hipSuccess) return err;
            temp = nullptr;
            temp_bytes = 0;
            if ((err = hipMalloc(&temp, need)) != hipSuccess) return err;
            temp_bytes = need;
        }
        return rocprim::segmented_radix_sort_keys(temp, need, in, out, (unsigned)(g * n), (unsigned)(g * nodes),
                                                  seg_off, seg_off + 1, begin_bit, end_bit, s);
    };

    // each level: keys from the previous level's sorted keys (in keys_b) into
    // keys_a, then the sort of keys_a back into keys_b
    for (int32_t lv = 0; lv < depth; ++lv) {
        hipLaunchKernelGGL(level_keys_kernel, rows, dim3(threads), 0, s, P, depth, lv, n, idb,
                           lv == 0 ? (const uint64_t*)nullptr : keys_b, keys_a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = sort_level(lv, keys_a, keys_b, 0, 32 + (unsigned)idb)) != hipSuccess) return e;
        const std::vector<int64_t>& lo = level_off[lv];
        if ((e = hipMemcpy(node_off, lo.data(), lo.size() * sizeof(int64_t), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return e;
        const int nodes = 1 << lv;
        hipLaunchKernelGGL(level_splits_kernel, dim3((unsigned)((nodes + threads - 1) / threads), (unsigned)g),
                           dim3(threads), 0, s, keys_b, node_off, lv, n, idb, nsplit,
                           ix->splits + (int64_t)t0 * nsplit);
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
