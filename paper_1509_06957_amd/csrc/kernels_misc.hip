// Build-time and utility kernels: finiteness scan, and the bfloat16 and fp8
// copies of the data that the prefilter arms read.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mrpt_internal.h"

namespace mrpt {
namespace {

__global__ void check_finite_kernel(const float* __restrict__ A, int64_t count, int32_t* __restrict__ flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = __builtin_bit_cast(uint32_t, A[i]);
        bad |= ((b & 0x7f800000u) == 0x7f800000u) ? 1 : 0;
    }
    if (__ballot(bad != 0) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// round-to-nearest-even float32 -> bfloat16 (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t b = __builtin_bit_cast(uint32_t, x);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// one wave per row: lanes over columns
__global__ __launch_bounds__(256) void quantize_bf16_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                            uint16_t* __restrict__ Xb) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); row < n; row += waves) {
        const float* xr = X + row * d;
        uint16_t* br = Xb + row * d;
        for (int i = lane; i < d; i += 64) br[i] = to_bf16(xr[i]);
    }
}

}  // namespace

hipError_t launch_check_finite(const float* A, int64_t count, int32_t* flag, hipStream_t s) {
    if (count == 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, count, flag);
    return hipGetLastError();
}

// FP8 (e4m3) rows with a per-row scale: scale = max|x| / 240 (0 rows: 1), the
// codes are x / scale rounded to nearest by the hardware conversion (|x /
// scale| <= 240 is finite in both e4m3 encodings), and norm = scale^2 *
// sum(decode(code)^2) in float32, so that the prefilter's ||x^||^2 is the
// squared norm of exactly the row it decodes (stored: recomputing it per
// candidate costs the fp8 prefilter more than the load).  Scale and norm sit
// side by side (one float2 per row), so a candidate costs one 8-byte load
// beyond its codes rather than two scattered 4-byte ones.  One wave per row,
// d % 4 == 0.
__global__ __launch_bounds__(256) void quantize_fp8_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                           uint8_t* __restrict__ X8, float2* __restrict__ sn8) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); row < n; row += waves) {
        const float4* xr = reinterpret_cast<const float4*>(X + row * d);
        uint32_t* cr = reinterpret_cast<uint32_t*>(X8 + row * d);
        const int nv = d >> 2;
        float mx = 0.0f;
        for (int i = lane; i < nv; i += 64) {
            const float4 v = xr[i];
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        const float scale = mx > 0.0f ? mx / 240.0f : 1.0f;
        float acc = 0.0f;
        for (int i = lane; i < nv; i += 64) {
            const float4 v = xr[i];
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(v.x / scale, v.y / scale, 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(v.z / scale, v.w / scale, w, true);
            cr[i] = (uint32_t)w;
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
            acc = __builtin_fmaf(lo[0], lo[0], acc);
            acc = __builtin_fmaf(lo[1], lo[1], acc);
            acc = __builtin_fmaf(hi[0], hi[0], acc);
            acc = __builtin_fmaf(hi[1], hi[1], acc);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) sn8[row] = make_float2(scale, (scale * scale) * acc);
    }
}

hipError_t launch_quantize_fp8(const float* X, int64_t n, int32_t d, uint8_t* X8, float2* sn8, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(quantize_fp8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, X8, sn8);
    return hipGetLastError();
}

namespace {

// job blockIdx.y: words [0, words) from src to dst, grid-stride over x
__global__ __launch_bounds__(256) void copy_jobs_kernel(const CopyJob* __restrict__ jobs) {
    const CopyJob j = jobs[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < j.words; i += stride) j.dst[i] = j.src[i];
}

}  // namespace

hipError_t launch_copy_jobs(const CopyJob* jobs, int32_t njobs, int64_t max_words, hipStream_t s) {
    if (njobs == 0 || max_words == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((max_words + 255) / 256, 128);
    hipLaunchKernelGGL(copy_jobs_kernel, dim3((unsigned)blocks, (unsigned)njobs), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_quantize_bf16(const float* X, int64_t n, int32_t d, uint16_t* Xb, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(quantize_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d, Xb);
    return hipGetLastError();
}

}  // namespace mrpt
