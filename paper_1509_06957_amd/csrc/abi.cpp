// C ABI of libmrpt: argument checks, index lifetime, workspace, and the
// order of kernel launches of one query call (Alg. 4: route every query in
// every tree, vote, exact search in S).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <new>

#include "mrpt_internal.h"

namespace mrpt {

namespace {
thread_local std::string g_error;
// workspace bound per query call (larger batches run in several sub-batches);
// MRPT_WORKSPACE_LIMIT (bytes) overrides it
size_t workspace_limit() {
    const char* env = std::getenv("MRPT_WORKSPACE_LIMIT");
    if (env && *env) {
        const long long v = std::atoll(env);
        if (v > 0) return (size_t)v;
    }
    return size_t(4) << 30;
}

template <class T>
hipError_t dev_alloc(T** p, size_t count, int64_t* tally) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e == hipSuccess && tally) *tally += (int64_t)(count * sizeof(T));
    return e;
}

void dev_release(mrpt_index* ix) {
    void* ptrs[] = {ix->X, ix->Xb, ix->X8, ix->sn8, ix->rowptr, ix->col, ix->val,
                    ix->splits, ix->perm, ix->off, ix->vdir, ix->ws.base};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (ix->ws.done) (void)hipEventDestroy(ix->ws.done);
}

// the device that holds p (device or managed memory), or -1 for host memory
// and pointers HIP does not know
int pointer_device(const void* p) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return -1;
    return attr.device;
}

bool is_device_pointer(const void* p) { return pointer_device(p) >= 0; }

mrpt_status check_index(const mrpt_index* ix) {
    if (!ix) return fail(MRPT_EINVAL, "index is NULL");
    return MRPT_OK;
}

mrpt_status check_query_args(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                             const void* out_idx, const void* out_dist) {
    MRPT_TRY(check_index(ix));
    if (nq < 0) return fail(MRPT_EINVAL, "nq = %lld < 0", (long long)nq);
    if (k < 1 || k > kMaxK || (int64_t)k > ix->n)
        return fail(MRPT_EINVAL, "k = %d outside [1, min(n, %d)]", k, kMaxK);
    if (v < 1 || v > ix->T) return fail(MRPT_EINVAL, "v = %d outside [1, T = %d]", v, ix->T);
    if (nq > 0 && (!Q || !out_idx || !out_dist)) return fail(MRPT_EINVAL, "NULL query or output pointer");
    if (nq > 0) {
        const void* ptrs[] = {Q, out_idx, out_dist};
        const char* names[] = {"Q", "out_idx", "out_dist"};
        for (int i = 0; i < 3; ++i)
            if (pointer_device(ptrs[i]) != ix->device)
                return fail(MRPT_EINVAL, "%s must be device memory of the index's device %d", names[i], ix->device);
    }
    return MRPT_OK;
}

// bytes of a query workspace for nb queries at candidate cap `cap`; with
// base given, also lays the workspace out there (leaf | s_ids | s_count |
// flag, each 256-byte aligned)
size_t workspace_layout(const mrpt_index* ix, int64_t nb, int64_t cap, void* base, Workspace* ws) {
    const size_t leaf_b = ((size_t)nb * ix->T * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t ids_b = ((size_t)nb * (size_t)cap * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t cnt_b = ((size_t)nb * sizeof(int32_t) + 255) & ~size_t(255);
    if (base && ws) {
        char* b = (char*)base;
        ws->leaf = (int32_t*)b;
        ws->s_ids = (int32_t*)(b + leaf_b);
        ws->s_count = (int32_t*)(b + leaf_b + ids_b);
        ws->flag = (int32_t*)(b + leaf_b + ids_b + cnt_b);
    }
    return leaf_b + ids_b + cnt_b + 256;
}

// workspace for nb queries at candidate cap `cap` (caller holds ix->mu)
mrpt_status ensure_workspace(mrpt_index* ix, int64_t nb, int64_t cap) {
    const size_t need = workspace_layout(ix, nb, cap, nullptr, nullptr);
    if (!ix->ws.done) MRPT_HIP_TRY(hipEventCreateWithFlags(&ix->ws.done, hipEventDisableTiming));
    if (need > ix->ws.bytes) {
        MRPT_HIP_TRY(hipEventSynchronize(ix->ws.done));
        if (ix->ws.base) MRPT_HIP_TRY(hipFree(ix->ws.base));
        ix->ws.base = nullptr;
        ix->ws.bytes = 0;
        if (hipMalloc(&ix->ws.base, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MRPT_ENOMEM, "workspace of %zu bytes", need);
        }
        ix->ws.bytes = need;
    }
    (void)workspace_layout(ix, nb, cap, ix->ws.base, &ix->ws);
    return MRPT_OK;
}

size_t build_limit() {
    const char* env = std::getenv("MRPT_BUILD_LIMIT");
    if (env && *env) {
        const long long v = std::atoll(env);
        if (v > 0) return (size_t)v;
    }
    return (size_t)8 << 30;
}

// grows all trees on the device in groups that fit build_limit() of scratch
mrpt_status build_trees_on_device(mrpt_index* ix) {
    const int64_t n = ix->n;
    const int32_t depth = ix->depth, T = ix->T;
    std::vector<std::vector<int64_t>> level_off((size_t)depth + 1);
    for (int32_t lv = 0; lv <= depth; ++lv) leaf_offsets(n, lv, level_off[lv]);
    const size_t per_tree = device_build_bytes_per_tree(n, depth);
    int64_t g = std::max<int64_t>(1, (int64_t)(build_limit() / per_tree));
    g = std::min<int64_t>({g, (int64_t)T, (int64_t)((int64_t(1) << 31) - 1) / n});   // int32 key offsets
    float* P = nullptr;
    uint64_t *ka = nullptr, *kb = nullptr;
    int32_t* seg = nullptr;
    int64_t* node = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    auto release = [&]() {
        for (void* p : {(void*)P, (void*)ka, (void*)kb, (void*)seg, (void*)node, temp})
            if (p) (void)hipFree(p);
    };
    const size_t nodes = (size_t)1 << depth;
    hipError_t e = hipMalloc((void**)&P, (size_t)g * std::max(depth, 1) * n * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ka, (size_t)g * n * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&kb, (size_t)g * n * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&seg, ((size_t)g * nodes + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&node, (nodes + 1) * sizeof(int64_t));
    if (e != hipSuccess) {
        release();
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MRPT_ENOMEM : MRPT_EDEVICE, "device build scratch: %s",
                    hipGetErrorString(e));
    }
    for (int32_t t0 = 0; t0 < T && e == hipSuccess; t0 += (int32_t)g) {
        const int32_t gg = (int32_t)std::min<int64_t>(g, T - t0);
        e = grow_trees_device(ix, t0, gg, level_off, P, ka, kb, temp, temp_bytes, seg, node, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    release();
    if (e != hipSuccess) return fail(MRPT_EDEVICE, "device build: %s", hipGetErrorString(e));
    return MRPT_OK;
}

int64_t candidate_cap(const mrpt_index* ix, int32_t v) {
    const int64_t bound = (int64_t)ix->T * ix->max_leaf / v;
    return std::max<int64_t>(1, std::min<int64_t>(ix->n, bound));
}

int64_t batch_size(const mrpt_index* ix, int64_t nq, int64_t cap) {
    const int64_t per_q = (int64_t)(ix->T + cap + 1) * (int64_t)sizeof(int32_t);
    const int64_t nb = std::max<int64_t>(1, (int64_t)workspace_limit() / per_q);
    return std::min(nq, nb);
}

// the precision arm and its parameters against the index
mrpt_status check_arm(const mrpt_index* cix, int32_t k, const mrpt_query_opts& o) {
    if (o.precision != MRPT_FP32 && o.precision != MRPT_BF16_RERANK && o.precision != MRPT_FP8_RERANK)
        return fail(MRPT_EINVAL, "unknown precision %d", o.precision);
    if (o.precision == MRPT_FP8_RERANK && !cix->X8)
        return fail(MRPT_EINVAL, "the fp8 arm needs d %% 16 == 0 and d <= 1024 (d = %d)", cix->d);
    if (o.precision != MRPT_FP32) {
        if (o.rerank_factor < 1 || (int64_t)o.rerank_factor * k > kMaxRerank)
            return fail(MRPT_EINVAL, "rerank_factor*k = %lld outside [1, %d]",
                        (long long)o.rerank_factor * k, kMaxRerank);
        if (!(o.recheck_rel >= 0.0f) || !std::isfinite(o.recheck_rel))
            return fail(MRPT_EINVAL, "recheck_rel must be finite and >= 0");
        if (cix->d % 8 != 0 || cix->d > 1024)
            return fail(MRPT_EINVAL, "the prefilter arms need d %% 8 == 0 and d <= 1024 (d = %d)", cix->d);
    }
    return MRPT_OK;
}

// the kernels of one query batch of m <= workspace queries, in stream order:
// routing (Alg. 3), voting (Alg. 4), exact search in S.  Kernel launches
// only (no allocation, copy, memset or synchronisation), so a stream capture
// can record it.
hipError_t enqueue_batch(const mrpt_index* ix, const Workspace& ws, const float* Qb, int64_t m, int32_t k,
                         int32_t v, int64_t cap, const mrpt_query_opts& o, int32_t* out_idx, float* out_dist,
                         hipStream_t s, bool mark_stages, const LaunchCfg& cfg = LaunchCfg()) {
    auto mark = [&](int i) -> hipError_t {
        if (!mark_stages || !o.stage_events || !o.stage_events[i]) return hipSuccess;
        return hipEventRecord((hipEvent_t)o.stage_events[i], s);
    };
    hipError_t e;
    if ((e = mark(0)) != hipSuccess) return e;
    if ((e = launch_route(ix, Qb, m, ws.leaf, s, cfg)) != hipSuccess) return e;
    if ((e = mark(1)) != hipSuccess) return e;
    if ((e = launch_vote(ix, ws.leaf, m, v, ws.s_ids, cap, ws.s_count, s, cfg)) != hipSuccess) return e;
    if ((e = mark(2)) != hipSuccess) return e;
    if (o.precision == MRPT_FP32)
        e = launch_dist_fp32(ix, Qb, m, ws.s_ids, cap, ws.s_count, k, out_idx, out_dist, s);
    else
        e = launch_dist_prefilter(ix, o.precision == MRPT_FP8_RERANK ? 1 : 0, Qb, m, ws.s_ids, cap, ws.s_count, k,
                                  o.rerank_factor, o.recheck_rel, out_idx, out_dist, s);
    if (e != hipSuccess) return e;
    return mark(3);
}

mrpt_status query_impl(const mrpt_index* cix, const float* Q, int64_t nq, int32_t k, int32_t v, int32_t* out_idx,
                       float* out_dist, const mrpt_query_opts* opts, void* stream) {
    clear_error();
    MRPT_TRY(check_query_args(cix, Q, nq, k, v, out_idx, out_dist));
    mrpt_query_opts o;
    mrpt_default_opts(&o);
    if (opts) o = *opts;
    MRPT_TRY(check_arm(cix, k, o));
    if (nq == 0) return MRPT_OK;
    if (o.s_count && pointer_device(o.s_count) != cix->device)
        return fail(MRPT_EINVAL, "s_count must be device memory of the index's device %d", cix->device);
    mrpt_index* ix = const_cast<mrpt_index*>(cix);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    const int64_t cap = candidate_cap(ix, v);
    const int64_t nb = batch_size(ix, nq, cap);
    MRPT_TRY(ensure_workspace(ix, nb, cap));
    MRPT_HIP_TRY(hipStreamWaitEvent(s, ix->ws.done, 0));
    if (o.check_finite) {
        MRPT_HIP_TRY(hipMemsetAsync(ix->ws.flag, 0, sizeof(int32_t), s));
        MRPT_HIP_TRY(launch_check_finite(Q, nq * (int64_t)ix->d, ix->ws.flag, s));
        int32_t h = 0;
        MRPT_HIP_TRY(hipMemcpyAsync(&h, ix->ws.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MRPT_HIP_TRY(hipStreamSynchronize(s));
        if (h) return fail(MRPT_ENONFINITE, "query matrix holds NaN or Inf");
    }
    for (int64_t q0 = 0; q0 < nq; q0 += nb) {
        const int64_t m = std::min(nb, nq - q0);
        MRPT_HIP_TRY(enqueue_batch(ix, ix->ws, Q + q0 * ix->d, m, k, v, cap, o, out_idx + q0 * k,
                                   out_dist + q0 * k, s, q0 == 0));
        if (o.s_count) MRPT_HIP_TRY(launch_copy_counts(ix->ws.s_count, m, o.s_count + q0, s));
    }
    MRPT_HIP_TRY(hipEventRecord(ix->ws.done, s));
    return MRPT_OK;
}

// ---------------------------------------------------------------- allocation-free queries
// The temporaries of mrpt_query_noalloc (leaf ids, candidate lists and
// counts, projections, the finiteness flag) live in the file-scope array
// `scratch` below, one copy per GPU.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in): it takes the device
// address once per device from hipGetSymbolAddress.
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

__global__ void zero_flag_kernel(int32_t* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

mrpt_status noalloc_impl(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v, int32_t* out_idx,
                         float* out_dist, const mrpt_query_opts* opts, void* stream);

}  // namespace

mrpt_status fail(mrpt_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

void clear_error() { g_error.clear(); }

}  // namespace mrpt

static __device__ __align__(256) unsigned char scratch[MRPT_NOALLOC_SCRATCH_BYTES];

namespace mrpt {
namespace {

// the device address of `scratch` on the current device (taken on the first
// call per device and kept)
mrpt_status scratch_address(int device, char** out) {
    if (device < 0 || device >= (int)(sizeof(g_scratch_ptr) / sizeof(g_scratch_ptr[0])))
        return fail(MRPT_EDEVICE, "device %d beyond the scratch table", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MRPT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
        }
        g_scratch_ptr[device] = p;
    }
    *out = (char*)g_scratch_ptr[device];
    return MRPT_OK;
}

mrpt_status noalloc_impl(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v, int32_t* out_idx,
                         float* out_dist, const mrpt_query_opts* opts, void* stream) {
    clear_error();
    MRPT_TRY(check_query_args(ix, Q, nq, k, v, out_idx, out_dist));
    mrpt_query_opts o;
    mrpt_default_opts(&o);
    if (opts) o = *opts;
    MRPT_TRY(check_arm(ix, k, o));
    if (nq == 0) return MRPT_OK;
    if (o.s_count && pointer_device(o.s_count) != ix->device)
        return fail(MRPT_EINVAL, "s_count must be device memory of the index's device %d", ix->device);
    const size_t limit = MRPT_NOALLOC_SCRATCH_BYTES;
    const int64_t cap = candidate_cap(ix, v);
    const size_t one = workspace_layout(ix, 1, cap, nullptr, nullptr);
    if (one > limit)
        return fail(MRPT_EINVAL, "one query's temporaries take %zu bytes, beyond the %zu-byte scratch of "
                    "mrpt_query_noalloc (T * ceil(n / 2^depth) / v candidates)", one, limit);
    // the most queries whose temporaries fit the scratch
    int64_t nb = std::min<int64_t>(nq, (int64_t)(limit / one));
    while (nb < nq && workspace_layout(ix, nb + 1, cap, nullptr, nullptr) <= limit) ++nb;
    while (nb > 1 && workspace_layout(ix, nb, cap, nullptr, nullptr) > limit) --nb;
    hipStream_t s = (hipStream_t)stream;
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    char* base = nullptr;
    MRPT_TRY(scratch_address(ix->device, &base));
    Workspace ws;
    (void)workspace_layout(ix, nb, cap, base, &ws);
    if (o.check_finite) {
        // the flag is cleared by a kernel (no memset node where a caller captures)
        hipLaunchKernelGGL(zero_flag_kernel, dim3(1), dim3(64), 0, s, ws.flag);
        MRPT_HIP_TRY(hipGetLastError());
        MRPT_HIP_TRY(launch_check_finite(Q, nq * (int64_t)ix->d, ws.flag, s));
        int32_t h = 0;
        MRPT_HIP_TRY(hipMemcpyAsync(&h, ws.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MRPT_HIP_TRY(hipStreamSynchronize(s));
        if (h) return fail(MRPT_ENONFINITE, "query matrix holds NaN or Inf");
    }
    for (int64_t q0 = 0; q0 < nq; q0 += nb) {
        const int64_t m = std::min(nb, nq - q0);
        MRPT_HIP_TRY(enqueue_batch(ix, ws, Q + q0 * ix->d, m, k, v, cap, o, out_idx + q0 * k, out_dist + q0 * k, s,
                                   q0 == 0));
        if (o.s_count) MRPT_HIP_TRY(launch_copy_counts(ws.s_count, m, o.s_count + q0, s));
    }
    return MRPT_OK;
}

}  // namespace
}  // namespace mrpt

// A recorded query plan: one workspace per batch in one allocation, and the
// graph of all batches' kernels (chains of batches, one per branch).
struct mrpt_plan {
    int device = 0;
    void* ws_base = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~mrpt_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ws_base) (void)hipFree(ws_base);
    }
};

using namespace mrpt;

extern "C" {

const char* mrpt_last_error(void) { return g_error.c_str(); }

void mrpt_default_opts(mrpt_query_opts* o) {
    if (!o) return;
    o->precision = MRPT_FP32;
    o->rerank_factor = 4;
    o->recheck_rel = 1e-6f;
    o->check_finite = 0;
    o->s_count = nullptr;
    o->stage_events = nullptr;
}

void mrpt_default_build_opts(mrpt_build_opts* o) {
    if (!o) return;
    o->on_device = 1;
    o->exact_nnz = 0;
}

mrpt_status mrpt_build(const float* data, int64_t n, int32_t d, int32_t T, int32_t depth, float a, uint64_t seed,
                       mrpt_index** out) {
    return mrpt_build_ex(data, n, d, T, depth, a, seed, nullptr, out);
}

mrpt_status mrpt_build_ex(const float* data, int64_t n, int32_t d, int32_t T, int32_t depth, float a,
                          uint64_t seed, const mrpt_build_opts* opts, mrpt_index** out) {
    clear_error();
    mrpt_build_opts bo;
    mrpt_default_build_opts(&bo);
    if (opts) bo = *opts;
    if (!out) return fail(MRPT_EINVAL, "out is NULL");
    if (!data) return fail(MRPT_EINVAL, "data is NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(MRPT_EINVAL, "n = %lld outside [1, 2^31)", (long long)n);
    if (d < 1 || d > 65535) return fail(MRPT_EINVAL, "d = %d outside [1, 65535]", d);
    if (T < 1 || T > kMaxT) return fail(MRPT_EINVAL, "T = %d outside [1, %d]", T, kMaxT);
    if (depth < 0 || depth > kMaxDepth) return fail(MRPT_EINVAL, "depth = %d outside [0, %d]", depth, kMaxDepth);
    if ((int64_t(1) << depth) > n) return fail(MRPT_EINVAL, "2^depth = %lld exceeds n = %lld",
                                              (long long)(int64_t(1) << depth), (long long)n);
    if (!(a > 0.0f && a <= 1.0f)) return fail(MRPT_EINVAL, "a = %g outside (0, 1]", (double)a);
    if (!is_device_pointer(data)) return fail(MRPT_EINVAL, "data must be device memory");

    std::unique_ptr<mrpt_index> ix;
    try {
        ix.reset(new mrpt_index());
    } catch (const std::bad_alloc&) {
        return fail(MRPT_ENOMEM, "host allocation of the index");
    }
    ix->n = n; ix->d = d; ix->T = T; ix->depth = depth; ix->a = a; ix->seed = seed;
    ix->nleaf = 1 << depth;
    ix->max_leaf = (int32_t)((n + ix->nleaf - 1) / ix->nleaf);
    ix->id_chunk = (int32_t)std::min<int64_t>(n, 77 * 1024 * 8);
    MRPT_HIP_TRY(hipGetDevice(&ix->device));

    struct Guard {
        mrpt_index* p;
        ~Guard() { if (p) dev_release(p); }
    } guard{ix.get()};

    const size_t nd = (size_t)n * (size_t)d;
    auto oom = [&](hipError_t e, const char* what) -> mrpt_status {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MRPT_ENOMEM : MRPT_EDEVICE, "allocating %s: %s", what,
                    hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = dev_alloc(&ix->X, nd, &ix->device_bytes)) != hipSuccess) return oom(e, "data copy");
    MRPT_HIP_TRY(hipMemcpy(ix->X, data, nd * sizeof(float), hipMemcpyDeviceToDevice));
    {
        int32_t* flag = nullptr;
        MRPT_HIP_TRY(hipMalloc((void**)&flag, sizeof(int32_t)));
        hipError_t e1 = hipMemset(flag, 0, sizeof(int32_t));
        if (e1 == hipSuccess) e1 = launch_check_finite(ix->X, (int64_t)nd, flag, nullptr);
        int32_t h = 0;
        if (e1 == hipSuccess) e1 = hipMemcpy(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost);
        (void)hipFree(flag);
        MRPT_HIP_TRY(e1);
        if (h) return fail(MRPT_ENONFINITE, "data holds NaN or Inf");
    }

    generate_projection(d, T, depth, a, seed, bo.exact_nnz != 0, ix->h_rowptr, ix->h_col, ix->h_val);
    for (size_t r = 0; r + 1 < ix->h_rowptr.size(); ++r)
        ix->max_row_nnz = std::max(ix->max_row_nnz, ix->h_rowptr[r + 1] - ix->h_rowptr[r]);
    // the GPU build projects the data with the query path's projection kernel
    const bool on_device = bo.on_device != 0;
    ix->built_on_device = on_device ? 1 : 0;
    HostTrees trees;
    if (on_device) {
        leaf_offsets(n, depth, trees.off);
    } else {
        std::vector<float> hX;
        try {
            hX.resize(nd);
        } catch (const std::bad_alloc&) {
            return fail(MRPT_ENOMEM, "host copy of the data (%zu bytes)", nd * sizeof(float));
        }
        MRPT_HIP_TRY(hipMemcpy(hX.data(), ix->X, nd * sizeof(float), hipMemcpyDeviceToHost));
        grow_trees_host(hX.data(), n, d, T, depth, ix->h_rowptr, ix->h_col, ix->h_val, trees);
    }
    ix->h_off = trees.off;

    const size_t nnz = ix->h_col.size();
    const size_t nsplit = ((size_t)1 << depth) - 1;
    if ((e = dev_alloc(&ix->rowptr, ix->h_rowptr.size(), &ix->device_bytes)) != hipSuccess) return oom(e, "rowptr");
    if ((e = dev_alloc(&ix->col, std::max<size_t>(nnz, 1), &ix->device_bytes)) != hipSuccess) return oom(e, "col");
    if ((e = dev_alloc(&ix->val, std::max<size_t>(nnz, 1), &ix->device_bytes)) != hipSuccess) return oom(e, "val");
    if ((e = dev_alloc(&ix->splits, std::max<size_t>((size_t)T * nsplit, 1), &ix->device_bytes)) != hipSuccess)
        return oom(e, "splits");
    ix->perm_ld = n + kPermPad;
    if ((e = dev_alloc(&ix->perm, (size_t)T * (size_t)ix->perm_ld, &ix->device_bytes)) != hipSuccess)
        return oom(e, "perm");
    if ((e = dev_alloc(&ix->off, (size_t)ix->nleaf + 1, &ix->device_bytes)) != hipSuccess) return oom(e, "offsets");
    if ((e = dev_alloc(&ix->Xb, nd, &ix->device_bytes)) != hipSuccess) return oom(e, "bfloat16 data");
    const bool fp8 = d % 16 == 0 && d <= 1024;
    if (fp8) {
        if ((e = dev_alloc(&ix->X8, nd, &ix->device_bytes)) != hipSuccess) return oom(e, "fp8 data");
        if ((e = dev_alloc(&ix->sn8, (size_t)n, &ix->device_bytes)) != hipSuccess) return oom(e, "fp8 scales");
    }

    MRPT_HIP_TRY(hipMemcpy(ix->rowptr, ix->h_rowptr.data(), ix->h_rowptr.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
    if (nnz) {
        MRPT_HIP_TRY(hipMemcpy(ix->col, ix->h_col.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        MRPT_HIP_TRY(hipMemcpy(ix->val, ix->h_val.data(), nnz * sizeof(float), hipMemcpyHostToDevice));
    }
    if (!on_device) {
        if (nsplit)
            MRPT_HIP_TRY(hipMemcpy(ix->splits, trees.splits.data(), (size_t)T * nsplit * sizeof(float),
                                   hipMemcpyHostToDevice));
        MRPT_HIP_TRY(hipMemcpy2D(ix->perm, (size_t)ix->perm_ld * sizeof(int32_t), trees.perm.data(),
                                 (size_t)n * sizeof(int32_t), (size_t)n * sizeof(int32_t), (size_t)T,
                                 hipMemcpyHostToDevice));
    }
    {
        std::vector<int32_t> pad((size_t)T * kPermPad);
        for (size_t i = 0; i < pad.size(); ++i) pad[i] = (int32_t)(n + (int64_t)(i % kPermPad));
        MRPT_HIP_TRY(hipMemcpy2D(ix->perm + n, (size_t)ix->perm_ld * sizeof(int32_t), pad.data(),
                                 (size_t)kPermPad * sizeof(int32_t), (size_t)kPermPad * sizeof(int32_t), (size_t)T,
                                 hipMemcpyHostToDevice));
    }
    std::vector<int32_t> off32(ix->h_off.begin(), ix->h_off.end());
    MRPT_HIP_TRY(hipMemcpy(ix->off, off32.data(), off32.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (on_device) MRPT_TRY(build_trees_on_device(ix.get()));
    MRPT_HIP_TRY(launch_quantize_bf16(ix->X, n, d, ix->Xb, nullptr));
    if (fp8) MRPT_HIP_TRY(launch_quantize_fp8(ix->X, n, d, ix->X8, ix->sn8, nullptr));
    if ((e = build_vote_directory(ix.get(), &ix->device_bytes)) != hipSuccess) return oom(e, "leaf directory");
    MRPT_HIP_TRY(hipDeviceSynchronize());

    guard.p = nullptr;
    *out = ix.release();
    return MRPT_OK;
}

mrpt_status mrpt_query(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v, int32_t* out_idx,
                       float* out_dist, void* stream) {
    return query_impl(ix, Q, nq, k, v, out_idx, out_dist, nullptr, stream);
}

mrpt_status mrpt_query_ex(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v, int32_t* out_idx,
                          float* out_dist, const mrpt_query_opts* opts, void* stream) {
    return query_impl(ix, Q, nq, k, v, out_idx, out_dist, opts, stream);
}

mrpt_status mrpt_query_noalloc(const mrpt_index* ix, const float* Q, int64_t nq, int32_t k, int32_t v,
                               int32_t* out_idx, float* out_dist, const mrpt_query_opts* opts, void* stream) {
    return noalloc_impl(ix, Q, nq, k, v, out_idx, out_dist, opts, stream);
}

void mrpt_free(mrpt_index* ix) {
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    (void)hipDeviceSynchronize();
    dev_release(ix);
    delete ix;
}

mrpt_status mrpt_index_info(const mrpt_index* ix, mrpt_index_desc* out) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (!out) return fail(MRPT_EINVAL, "out is NULL");
    out->n = ix->n; out->d = ix->d; out->T = ix->T; out->depth = ix->depth;
    out->a = ix->a; out->seed = ix->seed;
    out->nnz = (int64_t)ix->h_col.size();
    out->max_leaf = ix->max_leaf;
    out->id_chunk = ix->id_chunk;
    out->device_bytes = ix->device_bytes;
    out->built_on_device = ix->built_on_device;
    out->max_row_nnz = ix->max_row_nnz;
    return MRPT_OK;
}

mrpt_status mrpt_export_projection(const mrpt_index* ix, int32_t* rowptr, int32_t* col, float* val) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (!rowptr || (!ix->h_col.empty() && (!col || !val))) return fail(MRPT_EINVAL, "NULL output pointer");
    std::memcpy(rowptr, ix->h_rowptr.data(), ix->h_rowptr.size() * sizeof(int32_t));
    if (!ix->h_col.empty()) {
        std::memcpy(col, ix->h_col.data(), ix->h_col.size() * sizeof(int32_t));
        std::memcpy(val, ix->h_val.data(), ix->h_val.size() * sizeof(float));
    }
    return MRPT_OK;
}

mrpt_status mrpt_export_tree(const mrpt_index* ix, int32_t t, float* splits, int32_t* perm) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (t < 0 || t >= ix->T) return fail(MRPT_EINVAL, "tree %d outside [0, %d)", t, ix->T);
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    const size_t nsplit = ((size_t)1 << ix->depth) - 1;
    if (splits && nsplit)
        MRPT_HIP_TRY(hipMemcpy(splits, ix->splits + (size_t)t * nsplit, nsplit * sizeof(float),
                               hipMemcpyDeviceToHost));
    if (perm)
        MRPT_HIP_TRY(hipMemcpy(perm, ix->perm + (size_t)t * ix->perm_ld, (size_t)ix->n * sizeof(int32_t),
                               hipMemcpyDeviceToHost));
    return MRPT_OK;
}

mrpt_status mrpt_export_leaf_offsets(const mrpt_index* ix, int64_t* off) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (!off) return fail(MRPT_EINVAL, "off is NULL");
    std::memcpy(off, ix->h_off.data(), ix->h_off.size() * sizeof(int64_t));
    return MRPT_OK;
}

mrpt_status mrpt_debug_leaves(const mrpt_index* ix, const float* Q, int64_t nq, int32_t* leaf, void* stream) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (nq < 0) return fail(MRPT_EINVAL, "nq < 0");
    if (nq > 0 && (!Q || !leaf)) return fail(MRPT_EINVAL, "NULL pointer");
    if (nq == 0) return MRPT_OK;
    mrpt_index* mix = const_cast<mrpt_index*>(ix);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(mix->mu);
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    MRPT_TRY(ensure_workspace(mix, nq, 1));
    MRPT_HIP_TRY(hipStreamWaitEvent(s, mix->ws.done, 0));
    MRPT_HIP_TRY(launch_route(ix, Q, nq, leaf, s));
    MRPT_HIP_TRY(hipEventRecord(mix->ws.done, s));
    return MRPT_OK;
}

mrpt_status mrpt_debug_votes(const mrpt_index* cix, const float* Q, int64_t nq, int32_t v, int32_t* s_count,
                             int32_t* s_ids, uint8_t* s_votes, int64_t cap, void* stream) {
    clear_error();
    MRPT_TRY(check_index(cix));
    if (nq < 0) return fail(MRPT_EINVAL, "nq < 0");
    if (v < 1 || v > cix->T) return fail(MRPT_EINVAL, "v = %d outside [1, T]", v);
    if (nq > 0 && (!Q || !s_count || !s_ids)) return fail(MRPT_EINVAL, "NULL pointer");
    if (cap < candidate_cap(cix, v))
        return fail(MRPT_EINVAL, "cap = %lld below the candidate bound %lld", (long long)cap,
                    (long long)candidate_cap(cix, v));
    if (nq == 0) return MRPT_OK;
    mrpt_index* ix = const_cast<mrpt_index*>(cix);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    MRPT_TRY(ensure_workspace(ix, nq, 1));
    MRPT_HIP_TRY(hipStreamWaitEvent(s, ix->ws.done, 0));
    MRPT_HIP_TRY(launch_route(ix, Q, nq, ix->ws.leaf, s));
    MRPT_HIP_TRY(launch_vote(ix, ix->ws.leaf, nq, v, s_ids, cap, s_count, s));
    if (s_votes) MRPT_HIP_TRY(launch_vote_counts(ix, ix->ws.leaf, nq, s_ids, cap, s_count, s_votes, s));
    MRPT_HIP_TRY(hipEventRecord(ix->ws.done, s));
    return MRPT_OK;
}

mrpt_status mrpt_debug_prefilter(const mrpt_index* cix, const float* Q, int64_t nq, int32_t k, int32_t v,
                                 const mrpt_query_opts* opts, int32_t* s_count, int32_t* keep_ids, void* stream) {
    clear_error();
    MRPT_TRY(check_query_args(cix, Q, nq, k, v, keep_ids, keep_ids));
    mrpt_query_opts o;
    mrpt_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision == MRPT_FP32) return fail(MRPT_EINVAL, "the prefilter hook needs a prefilter arm");
    MRPT_TRY(check_arm(cix, k, o));
    if (nq > 0 && !s_count) return fail(MRPT_EINVAL, "s_count is NULL");
    if (nq == 0) return MRPT_OK;
    mrpt_index* ix = const_cast<mrpt_index*>(cix);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    const int64_t cap = candidate_cap(ix, v);
    const int64_t nb = batch_size(ix, nq, cap);
    MRPT_TRY(ensure_workspace(ix, nb, cap));
    MRPT_HIP_TRY(hipStreamWaitEvent(s, ix->ws.done, 0));
    const int32_t kp = o.rerank_factor * k;
    for (int64_t q0 = 0; q0 < nq; q0 += nb) {
        const int64_t m = std::min(nb, nq - q0);
        const float* Qb = Q + q0 * ix->d;
        MRPT_HIP_TRY(launch_route(ix, Qb, m, ix->ws.leaf, s));
        MRPT_HIP_TRY(launch_vote(ix, ix->ws.leaf, m, v, ix->ws.s_ids, cap, ix->ws.s_count, s));
        MRPT_HIP_TRY(launch_dist_prefilter(ix, o.precision == MRPT_FP8_RERANK ? 1 : 0, Qb, m, ix->ws.s_ids, cap,
                                           ix->ws.s_count, k, o.rerank_factor, o.recheck_rel, nullptr, nullptr, s,
                                           keep_ids + q0 * kp));
        MRPT_HIP_TRY(launch_copy_counts(ix->ws.s_count, m, s_count + q0, s));
    }
    MRPT_HIP_TRY(hipEventRecord(ix->ws.done, s));
    return MRPT_OK;
}

mrpt_status mrpt_debug_lowp_rows(const mrpt_index* ix, int32_t precision, int64_t row0, int64_t nrows, void* rows,
                                 float* scale_norm, void* stream) {
    clear_error();
    MRPT_TRY(check_index(ix));
    if (row0 < 0 || nrows < 0 || row0 + nrows > ix->n)
        return fail(MRPT_EINVAL, "rows [%lld, %lld) outside [0, n = %lld)", (long long)row0,
                    (long long)(row0 + nrows), (long long)ix->n);
    if (precision != MRPT_BF16_RERANK && precision != MRPT_FP8_RERANK)
        return fail(MRPT_EINVAL, "precision %d has no low-precision rows", precision);
    if (precision == MRPT_FP8_RERANK && !ix->X8)
        return fail(MRPT_EINVAL, "the index has no fp8 rows (d %% 16 != 0 or d > 1024)");
    if (nrows == 0) return MRPT_OK;
    if (!rows) return fail(MRPT_EINVAL, "rows is NULL");
    hipStream_t s = (hipStream_t)stream;
    MRPT_HIP_TRY(hipSetDevice(ix->device));
    const size_t nd = (size_t)nrows * (size_t)ix->d;
    if (precision == MRPT_BF16_RERANK) {
        MRPT_HIP_TRY(hipMemcpyAsync(rows, ix->Xb + (size_t)row0 * ix->d, nd * sizeof(uint16_t),
                                    hipMemcpyDeviceToDevice, s));
    } else {
        MRPT_HIP_TRY(hipMemcpyAsync(rows, ix->X8 + (size_t)row0 * ix->d, nd, hipMemcpyDeviceToDevice, s));
        if (scale_norm)
            MRPT_HIP_TRY(hipMemcpyAsync(scale_norm, ix->sn8 + row0, (size_t)nrows * sizeof(float2),
                                        hipMemcpyDeviceToDevice, s));
    }
    return MRPT_OK;
}

int64_t mrpt_candidate_cap(const mrpt_index* ix, int32_t v) {
    if (!ix || v < 1) return 0;
    return candidate_cap(ix, v);
}

void mrpt_default_plan_opts(mrpt_plan_opts* o) {
    if (!o) return;
    o->precision = MRPT_FP32;
    o->rerank_factor = 4;
    o->recheck_rel = 1e-6f;
    o->branches = 4;
    o->proj_rows = 0;
    o->vote_kernel = 0;
    o->fused = 1;
    o->vote_waves = 0;
}

mrpt_status mrpt_plan_create(const mrpt_batch* batches, int32_t nbatch, const mrpt_plan_opts* opts,
                             mrpt_plan** out) {
    clear_error();
    if (!out) return fail(MRPT_EINVAL, "out is NULL");
    if (!batches || nbatch < 1) return fail(MRPT_EINVAL, "a plan needs nbatch >= 1 batches");
    mrpt_plan_opts po;
    mrpt_default_plan_opts(&po);
    if (opts) po = *opts;
    if (po.branches < 1 || po.branches > 64) return fail(MRPT_EINVAL, "branches = %d outside [1, 64]", po.branches);
    if (po.proj_rows != 0 && po.proj_rows != 4 && po.proj_rows != 16)
        return fail(MRPT_EINVAL, "proj_rows = %d is not 0, 4 or 16", po.proj_rows);
    if (po.vote_kernel < 0 || po.vote_kernel > 2) return fail(MRPT_EINVAL, "vote_kernel = %d outside [0, 2]", po.vote_kernel);
    if (po.fused != 0 && po.fused != 1) return fail(MRPT_EINVAL, "fused = %d is not 0 or 1", po.fused);
    if (po.vote_waves != 0 && po.vote_waves != 8 && po.vote_waves != 16)
        return fail(MRPT_EINVAL, "vote_waves = %d is not 0, 8 or 16", po.vote_waves);
    LaunchCfg cfg;
    cfg.proj_rows = po.proj_rows;
    cfg.vote_kernel = po.vote_kernel;
    cfg.vote_waves = po.vote_waves;
    mrpt_query_opts o;
    mrpt_default_opts(&o);
    o.precision = (mrpt_precision)po.precision;
    o.rerank_factor = po.rerank_factor;
    o.recheck_rel = po.recheck_rel;
    int dev = 0;
    MRPT_HIP_TRY(hipGetDevice(&dev));

    // every batch checked as a query call would be
    for (int32_t i = 0; i < nbatch; ++i) {
        const mrpt_batch& b = batches[i];
        mrpt_status st = check_query_args(b.index, b.Q, b.nq, b.k, b.v, b.out_idx, b.out_dist);
        if (st == MRPT_OK && b.nq < 1) st = fail(MRPT_EINVAL, "nq = %lld < 1", (long long)b.nq);
        if (st == MRPT_OK) st = check_arm(b.index, b.k, o);
        if (st == MRPT_OK && b.index->device != dev)
            st = fail(MRPT_EINVAL, "index on device %d, current device %d", b.index->device, dev);
        if (st != MRPT_OK) {
            const std::string why = g_error;
            return fail(st, "batch %d: %s", i, why.c_str());
        }
    }

    // batches of one (index, k, v) form a group, searched as one query call:
    // a multi-batch group gathers its queries into a staging array and
    // scatters the results back (every kernel works per query, so the results
    // are the per-batch ones).  Layout of the plan's allocation, per group:
    // workspace | staged queries, results | gather jobs | scatter jobs.
    struct Group {
        const mrpt_index* ix;
        int32_t k, v;
        std::vector<int32_t> members;
        int64_t rows = 0, cap = 0;
        size_t ws_off = 0, q_off = 0, oi_off = 0, od_off = 0, gj_off = 0, sj_off = 0;
        double work = 0.0;
        bool staged() const { return members.size() > 1; }
    };
    std::vector<Group> groups;
    for (int32_t i = 0; i < nbatch; ++i) {
        const mrpt_batch& b = batches[i];
        size_t gi = 0;
        while (gi < groups.size() && !(groups[gi].ix == b.index && groups[gi].k == b.k && groups[gi].v == b.v)) ++gi;
        if (gi == groups.size()) {
            Group g;
            g.ix = b.index;
            g.k = b.k;
            g.v = b.v;
            groups.push_back(g);
        }
        groups[gi].members.push_back(i);
        groups[gi].rows += b.nq;
    }
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t total = 0;
    for (Group& g : groups) {
        g.cap = candidate_cap(g.ix, g.v);
        g.ws_off = total;
        total += align(workspace_layout(g.ix, g.rows, g.cap, nullptr, nullptr));
        if (g.staged()) {
            g.q_off = total;
            total += align((size_t)g.rows * g.ix->d * sizeof(float));
            g.oi_off = total;
            total += align((size_t)g.rows * g.k * sizeof(int32_t));
            g.od_off = total;
            total += align((size_t)g.rows * g.k * sizeof(float));
            g.gj_off = total;
            total += align(g.members.size() * sizeof(CopyJob));
            g.sj_off = total;
            total += align(2 * g.members.size() * sizeof(CopyJob));
        }
        // estimated bytes moved: leaf id lists, and candidate rows (about
        // T * leaf / v of them)
        const double ids = (double)g.ix->T * g.ix->max_leaf;
        g.work = (double)g.rows * (4.0 * ids + 4.0 * g.ix->d * ids / g.v);
    }

    // fused form: the groups of every stage's kernel form, and the device
    // tables their launches read (placed after the groups' memory)
    struct Class {
        int64_t key = 0;
        std::vector<int32_t> members;   // group numbers
        size_t tab_off = 0, row_off = 0;
        int64_t rows = 0;
    };
    std::vector<Class> route_cls, vote_cls, search_cls;
    std::vector<int32_t> route_alone, vote_alone, search_alone;   // groups launched on their own
    size_t gather_off = 0, scatter_off = 0;
    int32_t n_gather = 0, n_scatter = 0;
    const bool fused = po.fused != 0;
    if (fused) {
        auto add = [](std::vector<Class>& cls, int64_t key, int32_t g) {
            for (Class& c : cls)
                if (c.key == key) { c.members.push_back(g); return; }
            Class c;
            c.key = key;
            c.members.push_back(g);
            cls.push_back(c);
        };
        for (int32_t gi = 0; gi < (int32_t)groups.size(); ++gi) {
            const Group& g = groups[gi];
            const int32_t rf = route_form(g.ix);
            if (rf >= 0) add(route_cls, rf, gi);
            else route_alone.push_back(gi);
            const int64_t vf = vote_form(g.ix, g.v, cfg);
            if (vf >= 0) add(vote_cls, vf, gi);
            else vote_alone.push_back(gi);
            // a staged group's queries are 256-byte aligned; a lone batch's are the caller's
            const float* qp = g.staged() ? nullptr : batches[g.members[0]].Q;
            const int32_t sf = search_form(g.ix, o.precision, g.k, qp);
            if (sf >= 0) add(search_cls, ((int64_t)sf << 20) | g.ix->d, gi);
            else search_alone.push_back(gi);
        }
        // vote classes whose queue would not fit LDS go back to one launch per group
        for (size_t c = 0; c < vote_cls.size();) {
            int32_t mw = 0;
            int64_t most = 0;
            for (int32_t gi : vote_cls[c].members) {
                mw = std::max(mw, vote_map_words(groups[gi].ix));
                most = std::max<int64_t>(most, (int64_t)groups[gi].ix->T * groups[gi].ix->max_leaf);
            }
            if (vote_multi_qcap(vote_cls[c].key, mw, most) < 0) {
                for (int32_t gi : vote_cls[c].members) vote_alone.push_back(gi);
                vote_cls.erase(vote_cls.begin() + (long)c);
            } else {
                ++c;
            }
        }
        for (Class& c : route_cls) {
            c.tab_off = total;
            total += align(c.members.size() * sizeof(RouteItem));
        }
        for (Class& c : vote_cls) {
            for (int32_t gi : c.members) c.rows += groups[gi].rows;
            c.tab_off = total;
            total += align(c.members.size() * sizeof(VoteItem));
            c.row_off = total;
            total += align((size_t)c.rows * sizeof(int32_t));
        }
        for (Class& c : search_cls) {
            c.tab_off = total;
            total += align(c.members.size() * sizeof(SearchItem));
        }
        for (const Group& g : groups)
            if (g.staged()) {
                n_gather += (int32_t)g.members.size();
                n_scatter += 2 * (int32_t)g.members.size();
            }
        gather_off = total;
        total += align((size_t)n_gather * sizeof(CopyJob));
        scatter_off = total;
        total += align((size_t)n_scatter * sizeof(CopyJob));
    }

    std::unique_ptr<mrpt_plan> plan;
    try {
        plan.reset(new mrpt_plan());
    } catch (const std::bad_alloc&) {
        return fail(MRPT_ENOMEM, "host allocation of the plan");
    }
    plan->device = dev;
    if (hipMalloc(&plan->ws_base, total) != hipSuccess) {
        (void)hipGetLastError();
        plan->ws_base = nullptr;
        return fail(MRPT_ENOMEM, "plan workspaces of %zu bytes", total);
    }
    plan->ws_bytes = total;
    char* base = (char*)plan->ws_base;

    // gather / scatter job tables of the staged groups
    for (Group& g : groups) {
        if (!g.staged()) continue;
        std::vector<CopyJob> gather, scatter;
        int64_t row = 0;
        const int d = g.ix->d;
        for (int32_t i : g.members) {
            const mrpt_batch& b = batches[i];
            gather.push_back({reinterpret_cast<const int32_t*>(b.Q),
                              reinterpret_cast<int32_t*>(base + g.q_off) + row * d, b.nq * d});
            scatter.push_back({reinterpret_cast<const int32_t*>(base + g.oi_off) + row * g.k, b.out_idx,
                               b.nq * g.k});
            scatter.push_back({reinterpret_cast<const int32_t*>(base + g.od_off) + row * g.k,
                               reinterpret_cast<int32_t*>(b.out_dist), b.nq * g.k});
            row += b.nq;
        }
        MRPT_HIP_TRY(hipMemcpy(base + g.gj_off, gather.data(), gather.size() * sizeof(CopyJob),
                               hipMemcpyHostToDevice));
        MRPT_HIP_TRY(hipMemcpy(base + g.sj_off, scatter.data(), scatter.size() * sizeof(CopyJob),
                               hipMemcpyHostToDevice));
    }

    if (fused) {
        // the call of group g: its queries, workspace and outputs
        auto call_Q = [&](const Group& g) -> const float* {
            return g.staged() ? reinterpret_cast<const float*>(base + g.q_off) : batches[g.members[0]].Q;
        };
        auto call_idx = [&](const Group& g) -> int32_t* {
            return g.staged() ? reinterpret_cast<int32_t*>(base + g.oi_off) : batches[g.members[0]].out_idx;
        };
        auto call_dist = [&](const Group& g) -> float* {
            return g.staged() ? reinterpret_cast<float*>(base + g.od_off) : batches[g.members[0]].out_dist;
        };
        auto call_ws = [&](const Group& g) -> Workspace {
            Workspace ws;
            (void)workspace_layout(g.ix, g.rows, g.cap, base + g.ws_off, &ws);
            return ws;
        };
        // device tables
        struct RouteLaunch { int32_t form, rpw, qpl, max_d; int64_t blocks; };
        std::vector<RouteLaunch> rl;
        for (const Class& c : route_cls) {
            int64_t tiles = 0;
            for (int32_t gi : c.members) {
                const Group& g = groups[gi];
                const RouteGrid r16 = route_grid(g.ix, g.rows, 16, 1);
                tiles += r16.nbx * r16.nby;
            }
            RouteLaunch L{(int32_t)c.key, 0, 0, 0, 0};
            route_shape(L.form, tiles, po.proj_rows, &L.rpw, &L.qpl);
            std::vector<RouteItem> items;
            for (int32_t gi : c.members) {
                const Group& g = groups[gi];
                if (!route_form_holds(L.form, g.ix))
                    return fail(MRPT_EINTERNAL, "routing form %d does not hold group %d", L.form, gi);
                const Workspace ws = call_ws(g);
                const RouteGrid rg = route_grid(g.ix, g.rows, L.rpw, L.qpl);
                RouteItem it;
                it.Q = call_Q(g);
                it.rowptr = g.ix->rowptr;
                it.col = g.ix->col;
                it.val = g.ix->val;
                it.splits = g.ix->splits;
                it.leaf = ws.leaf;
                it.nq = g.rows;
                it.blk0 = L.blocks;
                it.nbx = rg.nbx;
                it.d = g.ix->d;
                it.T = g.ix->T;
                it.depth = g.ix->depth;
                it.nby = (int32_t)rg.nby;
                items.push_back(it);
                L.blocks += rg.nbx * rg.nby;
                L.max_d = std::max(L.max_d, g.ix->d);
            }
            MRPT_HIP_TRY(hipMemcpy(base + c.tab_off, items.data(), items.size() * sizeof(RouteItem),
                                   hipMemcpyHostToDevice));
            rl.push_back(L);
        }
        struct VoteLaunch { int32_t map_words; int64_t qcap; };
        std::vector<VoteLaunch> vl;
        std::vector<std::vector<int32_t>> recount((size_t)vote_cls.size());
        for (size_t ci = 0; ci < vote_cls.size(); ++ci) {
            const Class& c = vote_cls[ci];
            VoteLaunch L{0, 0};
            int64_t most = 0;
            for (int32_t gi : c.members) {
                L.map_words = std::max(L.map_words, vote_map_words(groups[gi].ix));
                most = std::max<int64_t>(most, (int64_t)groups[gi].ix->T * groups[gi].ix->max_leaf);
            }
            L.qcap = vote_multi_qcap(c.key, L.map_words, most);
            std::vector<VoteItem> items;
            std::vector<int32_t> row_item;
            int64_t row0 = 0;
            for (int32_t gi : c.members) {
                const Group& g = groups[gi];
                const Workspace ws = call_ws(g);
                VoteItem it;
                it.leaf = ws.leaf;
                it.perm = g.ix->perm;
                it.off = g.ix->off;
                it.s_ids = ws.s_ids;
                it.s_count = ws.s_count;
                it.cap = g.cap;
                it.ld = g.ix->perm_ld;
                it.row0 = row0;
                it.n = (int32_t)g.ix->n;
                it.v = g.v;
                it.map_words = vote_map_words(g.ix);
                it.pad_ = 0;
                row_item.insert(row_item.end(), (size_t)g.rows, (int32_t)items.size());
                items.push_back(it);
                row0 += g.rows;
                // a group whose queries could overflow the queue is counted again
                if (g.v >= 2 && L.qcap < vote_most_queued(g.ix)) recount[ci].push_back(gi);
            }
            MRPT_HIP_TRY(hipMemcpy(base + c.tab_off, items.data(), items.size() * sizeof(VoteItem),
                                   hipMemcpyHostToDevice));
            MRPT_HIP_TRY(hipMemcpy(base + c.row_off, row_item.data(), row_item.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice));
            vl.push_back(L);
        }
        std::vector<int64_t> sl;   // rows per search class
        for (const Class& c : search_cls) {
            std::vector<SearchItem> items;
            int64_t row0 = 0;
            for (int32_t gi : c.members) {
                const Group& g = groups[gi];
                const Workspace ws = call_ws(g);
                SearchItem it;
                it.X = g.ix->X;
                it.Xq = o.precision == MRPT_FP8_RERANK ? g.ix->X8 : reinterpret_cast<const uint8_t*>(g.ix->Xb);
                it.sn8 = g.ix->sn8;
                it.Q = call_Q(g);
                it.s_ids = ws.s_ids;
                it.s_count = ws.s_count;
                it.out_idx = call_idx(g);
                it.out_dist = call_dist(g);
                it.cap = g.cap;
                it.row0 = row0;
                it.k = g.k;
                it.kp = g.k * o.rerank_factor;
                items.push_back(it);
                row0 += g.rows;
            }
            MRPT_HIP_TRY(hipMemcpy(base + c.tab_off, items.data(), items.size() * sizeof(SearchItem),
                                   hipMemcpyHostToDevice));
            sl.push_back(row0);
        }
        // one gather and one scatter job table for all staged groups
        std::vector<CopyJob> gather, scatter;
        int64_t most_g = 0, most_s = 0;
        for (const Group& g : groups) {
            if (!g.staged()) continue;
            int64_t row = 0;
            const int d = g.ix->d;
            for (int32_t i : g.members) {
                const mrpt_batch& b = batches[i];
                gather.push_back({reinterpret_cast<const int32_t*>(b.Q),
                                  reinterpret_cast<int32_t*>(base + g.q_off) + row * d, b.nq * d});
                scatter.push_back({reinterpret_cast<const int32_t*>(base + g.oi_off) + row * g.k, b.out_idx,
                                   b.nq * g.k});
                scatter.push_back({reinterpret_cast<const int32_t*>(base + g.od_off) + row * g.k,
                                   reinterpret_cast<int32_t*>(b.out_dist), b.nq * g.k});
                most_g = std::max<int64_t>(most_g, b.nq * d);
                most_s = std::max<int64_t>(most_s, b.nq * g.k);
                row += b.nq;
            }
        }
        if (!gather.empty()) {
            MRPT_HIP_TRY(hipMemcpy(base + gather_off, gather.data(), gather.size() * sizeof(CopyJob),
                                   hipMemcpyHostToDevice));
            MRPT_HIP_TRY(hipMemcpy(base + scatter_off, scatter.data(), scatter.size() * sizeof(CopyJob),
                                   hipMemcpyHostToDevice));
        }

        // the launches of each stage as units: classes of a stage run on up
        // to `branches` streams side by side, and a stage starts when the one
        // before it has ended
        using Unit = std::function<hipError_t(hipStream_t)>;
        std::vector<std::vector<Unit>> stages(5);
        if (!gather.empty())
            stages[0].push_back([&](hipStream_t x) {
                return launch_copy_jobs(reinterpret_cast<const CopyJob*>(base + gather_off), n_gather, most_g, x);
            });
        for (size_t ci = 0; ci < route_cls.size(); ++ci)
            stages[1].push_back([&, ci](hipStream_t x) {
                return launch_route_multi(rl[ci].form, rl[ci].rpw, rl[ci].qpl, rl[ci].max_d,
                                          reinterpret_cast<const RouteItem*>(base + route_cls[ci].tab_off),
                                          (int32_t)route_cls[ci].members.size(), rl[ci].blocks, x);
            });
        for (int32_t gi : route_alone)
            stages[1].push_back([&, gi](hipStream_t x) {
                const Group& g = groups[gi];
                const Workspace ws = call_ws(g);
                return launch_route(g.ix, call_Q(g), g.rows, ws.leaf, x, cfg);
            });
        for (size_t ci = 0; ci < vote_cls.size(); ++ci)
            stages[2].push_back([&, ci](hipStream_t x) {
                hipError_t e1 = launch_vote_multi(vote_cls[ci].key, vl[ci].map_words, vl[ci].qcap,
                                                  reinterpret_cast<const VoteItem*>(base + vote_cls[ci].tab_off),
                                                  reinterpret_cast<const int32_t*>(base + vote_cls[ci].row_off),
                                                  vote_cls[ci].rows, x);
                for (int32_t gi : recount[ci]) {
                    if (e1 != hipSuccess) break;
                    const Group& g = groups[gi];
                    const Workspace ws = call_ws(g);
                    e1 = launch_vote_recount(g.ix, ws.leaf, g.rows, g.v, ws.s_ids, g.cap, ws.s_count, x);
                }
                return e1;
            });
        for (int32_t gi : vote_alone)
            stages[2].push_back([&, gi](hipStream_t x) {
                const Group& g = groups[gi];
                const Workspace ws = call_ws(g);
                return launch_vote(g.ix, ws.leaf, g.rows, g.v, ws.s_ids, g.cap, ws.s_count, x, cfg);
            });
        for (size_t ci = 0; ci < search_cls.size(); ++ci)
            stages[3].push_back([&, ci](hipStream_t x) {
                return launch_search_multi((int32_t)(search_cls[ci].key >> 20),
                                           (int32_t)(search_cls[ci].key & 0xFFFFF),
                                           reinterpret_cast<const SearchItem*>(base + search_cls[ci].tab_off),
                                           (int32_t)search_cls[ci].members.size(), sl[ci], o.recheck_rel, x);
            });
        for (int32_t gi : search_alone)
            stages[3].push_back([&, gi](hipStream_t x) {
                const Group& g = groups[gi];
                const Workspace ws = call_ws(g);
                if (o.precision == MRPT_FP32)
                    return launch_dist_fp32(g.ix, call_Q(g), g.rows, ws.s_ids, g.cap, ws.s_count, g.k, call_idx(g),
                                            call_dist(g), x);
                return launch_dist_prefilter(g.ix, o.precision == MRPT_FP8_RERANK ? 1 : 0, call_Q(g), g.rows,
                                             ws.s_ids, g.cap, ws.s_count, g.k, o.rerank_factor, o.recheck_rel,
                                             call_idx(g), call_dist(g), x);
            });
        if (!scatter.empty())
            stages[4].push_back([&](hipStream_t x) {
                return launch_copy_jobs(reinterpret_cast<const CopyJob*>(base + scatter_off), n_scatter, most_s, x);
            });
        size_t widest = 1;
        for (const auto& u : stages) widest = std::max(widest, u.size());
        const int nstr = (int)std::min<size_t>((size_t)po.branches, widest);

        hipStream_t st = nullptr;
        std::vector<hipStream_t> side((size_t)nstr, nullptr);
        std::vector<hipEvent_t> evs;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        for (int i = 0; i < nstr && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        auto new_event = [&](hipEvent_t* ev) {
            hipError_t r = hipEventCreateWithFlags(ev, hipEventDisableTiming);
            if (r == hipSuccess) evs.push_back(*ev);
            return r;
        };
        bool capturing = false;
        if (e == hipSuccess) {
            e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
            capturing = e == hipSuccess;
        }
        for (const auto& units : stages) {
            if (e != hipSuccess || units.empty()) continue;
            if (units.size() == 1 || nstr == 1) {
                for (const Unit& u : units) {
                    if (e == hipSuccess) e = u(st);
                }
                continue;
            }
            // fork from the chain, unit j on side stream j mod nstr, join
            hipEvent_t fork = nullptr;
            e = new_event(&fork);
            if (e == hipSuccess) e = hipEventRecord(fork, st);
            const int used = (int)std::min<size_t>((size_t)nstr, units.size());
            for (int i = 0; i < used && e == hipSuccess; ++i) e = hipStreamWaitEvent(side[i], fork, 0);
            for (size_t j = 0; j < units.size() && e == hipSuccess; ++j) e = units[j](side[j % (size_t)nstr]);
            for (int i = 0; i < used && e == hipSuccess; ++i) {
                hipEvent_t join = nullptr;
                e = new_event(&join);
                if (e == hipSuccess) e = hipEventRecord(join, side[i]);
                if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
            }
        }
        if (capturing) {
            const hipError_t e2 = hipStreamEndCapture(st, &plan->graph);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        for (hipEvent_t x : evs) (void)hipEventDestroy(x);
        for (hipStream_t x : side)
            if (x) (void)hipStreamDestroy(x);
        if (st) (void)hipStreamDestroy(st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MRPT_EDEVICE, "recording the plan: %s", hipGetErrorString(e));
        }
        *out = plan.release();
        return MRPT_OK;
    }

    // groups dealt to branches, largest first, each to the least loaded
    const int ng = (int)groups.size();
    std::vector<int32_t> order((size_t)ng);
    for (int32_t i = 0; i < ng; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return groups[x].work > groups[y].work; });
    const int nbr = std::min<int>(po.branches, ng);
    std::vector<double> load((size_t)nbr, 0.0);
    std::vector<std::vector<int32_t>> chain((size_t)nbr);
    for (int32_t i : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += groups[i].work;
        chain[b].push_back(i);
    }

    // record: fork from an origin stream to one stream per branch, every
    // branch's groups in sequence (gather, search, scatter), join back
    std::vector<hipStream_t> bs((size_t)nbr, nullptr);
    std::vector<hipEvent_t> ev((size_t)nbr + 1, nullptr);
    hipStream_t origin = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&origin, hipStreamNonBlocking);
    for (int b = 0; b < nbr && e == hipSuccess; ++b) e = hipStreamCreateWithFlags(&bs[b], hipStreamNonBlocking);
    for (int b = 0; b <= nbr && e == hipSuccess; ++b) e = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming);
    bool capturing = false;
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
        capturing = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipEventRecord(ev[nbr], origin);
    for (int b = 0; b < nbr && e == hipSuccess; ++b) e = hipStreamWaitEvent(bs[b], ev[nbr], 0);
    for (int b = 0; b < nbr && e == hipSuccess; ++b) {
        for (int32_t gi : chain[b]) {
            const Group& g = groups[gi];
            Workspace ws;
            (void)workspace_layout(g.ix, g.rows, g.cap, base + g.ws_off, &ws);
            if (g.staged()) {
                int64_t most = 0;
                for (int32_t i : g.members) most = std::max<int64_t>(most, batches[i].nq * g.ix->d);
                e = launch_copy_jobs(reinterpret_cast<const CopyJob*>(base + g.gj_off), (int32_t)g.members.size(),
                                     most, bs[b]);
                if (e == hipSuccess)
                    e = enqueue_batch(g.ix, ws, reinterpret_cast<const float*>(base + g.q_off), g.rows, g.k, g.v,
                                      g.cap, o, reinterpret_cast<int32_t*>(base + g.oi_off),
                                      reinterpret_cast<float*>(base + g.od_off), bs[b], false, cfg);
                most = 0;
                for (int32_t i : g.members) most = std::max<int64_t>(most, batches[i].nq * g.k);
                if (e == hipSuccess)
                    e = launch_copy_jobs(reinterpret_cast<const CopyJob*>(base + g.sj_off),
                                         2 * (int32_t)g.members.size(), most, bs[b]);
            } else {
                const mrpt_batch& bt = batches[g.members[0]];
                e = enqueue_batch(g.ix, ws, bt.Q, bt.nq, g.k, g.v, g.cap, o, bt.out_idx, bt.out_dist, bs[b], false,
                                  cfg);
            }
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = hipEventRecord(ev[b], bs[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, ev[b], 0);
    }
    if (capturing) {
        const hipError_t e2 = hipStreamEndCapture(origin, &plan->graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    for (hipStream_t x : bs)
        if (x) (void)hipStreamDestroy(x);
    if (origin) (void)hipStreamDestroy(origin);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MRPT_EDEVICE, "recording the plan: %s", hipGetErrorString(e));
    }
    *out = plan.release();
    return MRPT_OK;
}

mrpt_status mrpt_plan_launch(mrpt_plan* plan, void* stream) {
    clear_error();
    if (!plan || !plan->exec) return fail(MRPT_EINVAL, "plan is NULL");
    MRPT_HIP_TRY(hipSetDevice(plan->device));
    MRPT_HIP_TRY(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return MRPT_OK;
}

int64_t mrpt_plan_device_bytes(const mrpt_plan* plan) { return plan ? (int64_t)plan->ws_bytes : 0; }

void mrpt_plan_free(mrpt_plan* plan) { delete plan; }

}  // extern "C"
