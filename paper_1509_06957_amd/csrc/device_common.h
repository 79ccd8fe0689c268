// Device helpers shared by the query kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace mrpt {
namespace dev {

constexpr int kWave = 64;
constexpr int32_t kPadId = 0x7F000000;  // ids of empty top-k slots (distance +inf)

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// value known to be equal in all lanes, kept in a scalar register
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float read_lane_f(float x, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}
__device__ __forceinline__ int read_lane_i(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

// workgroup barrier that orders LDS accesses only: outstanding global loads
// stay in flight across it (a full __syncthreads waits for them)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// strict order on (distance, id): the order in which k-NN results are ranked
__device__ __forceinline__ bool key_less(float da, int32_t ia, float db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

// sum over aligned groups of G lanes (butterfly)
template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
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

    // entry e (wave-uniform e)
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

    // entries [0, cnt) to LDS arrays
    __device__ void store(float* sd, int32_t* si, int cnt) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = lane_id() * R + r;
            if (e < cnt) { sd[e] = d[r]; si[e] = id[r]; }
        }
    }
};

// number of entries of the sorted LDS list (sd, si)[0, cnt) that are < key
__device__ __forceinline__ int count_less(const float* sd, const int32_t* si, int cnt, float kd, int32_t ki) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key_less(sd[mid], si[mid], kd, ki)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace dev

// per-block LDS limit of the current device (bytes)
int lds_per_block_limit();

}  // namespace mrpt
