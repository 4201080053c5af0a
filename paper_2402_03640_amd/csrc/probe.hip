// Bandwidth probes (see hipmsat_probe.h): a streaming copy and a random-row
// gather-sum, the ceilings the solve loop's kernels are compared with.
#include <hip/hip_runtime.h>

#include <string>

#include "hipmsat_probe.h"

namespace {

thread_local std::string g_err;

int32_t fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return (int32_t)e;
}

#define PTRY(expr, what)                      \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return fail(e_, what); \
    } while (0)

// One 16-byte load and store per thread, the grid covering the buffers once
// (of the variants timed, strided grids of 4 to 32 workgroups per compute
// unit with 4 or 8 loads in flight per thread, non-temporal or not, and 1 to
// 8 loads per thread over a covering grid, this one moved the most).
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}


template <int V>
struct Vec {
    float v[V];
};

template <int V>
__device__ __forceinline__ Vec<V> ld(const float* p) {
    Vec<V> r;
    if constexpr (V == 1) {
        r.v[0] = *p;
    } else if constexpr (V == 2) {
        const float2 q = *reinterpret_cast<const float2*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
    } else {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
        r.v[2] = q.z;
        r.v[3] = q.w;
    }
    return r;
}

// W / V lanes per output, each owning V consecutive floats of the row; an
// output's D indices load as D / 4 16-byte loads, then its D rows.
template <int V, int D>
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ src, int32_t W,
                                                const uint32_t* __restrict__ idx, int64_t n_out,
                                                float* __restrict__ out) {
    const int lanes = W / V;
    const int64_t gt = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t o = gt / lanes;
    if (o >= n_out) return;
    const int c = (int)(gt % lanes) * V;
    const uint4* ip = reinterpret_cast<const uint4*>(idx + o * D);
    uint32_t id[D];
#pragma unroll
    for (int q = 0; q < D / 4; ++q) {
        const uint4 u = ip[q];
        id[4 * q] = u.x;
        id[4 * q + 1] = u.y;
        id[4 * q + 2] = u.z;
        id[4 * q + 3] = u.w;
    }
    Vec<V> r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) r[k] = ld<V>(src + (size_t)id[k] * W + c);
    Vec<V> s;
#pragma unroll
    for (int j = 0; j < V; ++j) s.v[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int j = 0; j < V; ++j) s.v[j] = s.v[j] + r[k].v[j];
#pragma unroll
    for (int j = 0; j < V; ++j) out[o * W + c + j] = s.v[j];
}

template <int V, int D>
hipError_t launch_gather(const float* src, int32_t W, const uint32_t* idx, int64_t n_out, float* out, int blocks,
                         hipStream_t s) {
    hipLaunchKernelGGL((k_gather<V, D>), dim3(blocks), dim3(256), 0, s, src, W, idx, n_out, out);
    return hipGetLastError();
}

// Grid barrier: `rounds` rounds in which every block adds one to a counter
// and its first thread polls it until every block has arrived (agent-scope
// release and acquire: what a persistent kernel needs between two passes
// whose data cross the XCDs).  Every wait is bounded: after `limit` polls, or
// once any block has given up, a block sets the abort flag and leaves.
__global__ __launch_bounds__(256) void k_barrier(unsigned* cnt, int* flag, int rounds, int limit) {
    __shared__ int give_up;
    for (int r = 0; r < rounds; ++r) {
        __syncthreads();
        if (threadIdx.x == 0) {
            give_up = 0;
            __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)(r + 1) * gridDim.x;
            int k = 0;
            while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++k > limit || __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    give_up = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (give_up) return;
    }
}

// A kernel that does nothing observable (its one load decides nothing).
__global__ __launch_bounds__(256) void k_empty(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && p[0] == 0x2545f491) p[1] = 1;
}

// Times `iters` launches of `launch` on s (after one warm launch).
template <typename F>
int32_t timed(F launch, int32_t iters, hipStream_t s, double* ms) {
    if (iters < 1 || !ms) {
        g_err = "iters >= 1 and an output pointer required";
        return -1;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PTRY(hipEventCreate(&e0), "hipEventCreate");
    struct Free {
        hipEvent_t& a;
        hipEvent_t& b;
        ~Free() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } fr{e0, e1};
    PTRY(hipEventCreate(&e1), "hipEventCreate");
    PTRY(launch(), "warm launch");
    PTRY(hipEventRecord(e0, s), "hipEventRecord");
    for (int32_t i = 0; i < iters; ++i) PTRY(launch(), "launch");
    PTRY(hipEventRecord(e1, s), "hipEventRecord");
    PTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    float t = 0.0f;
    PTRY(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
    *ms = (double)t / iters;
    return 0;
}

}  // namespace

extern "C" {

const char* hmsp_last_error(void) { return g_err.c_str(); }

int32_t hmsp_copy(const void* src, void* dst, int64_t bytes, int32_t iters, void* stream, double* ms) {
    g_err.clear();
    if (!src || !dst || bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0) {
        g_err = "non-null 16-byte aligned buffers and a positive multiple of 16 bytes required";
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n4 = bytes / 16;
    if ((n4 + 255) / 256 > INT32_MAX) {
        g_err = "copy too large for one launch";
        return -1;
    }
    const int blocks = (int)((n4 + 255) / 256);
    auto launch = [&]() {
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, static_cast<const float4*>(src),
                           static_cast<float4*>(dst), n4);
        return hipGetLastError();
    };
    return timed(launch, iters, s, ms);
}

int32_t hmsp_gather(const float* src, int64_t rows, int32_t row_floats, const uint32_t* idx, int64_t n_idx,
                    int32_t deg, int32_t vec, float* out, int32_t iters, void* stream, double* ms) {
    g_err.clear();
    const int W = row_floats;
    if (!src || !idx || !out || rows <= 0 || n_idx <= 0 || (W != 1 && W != 2 && W != 4 && W != 8 && W != 16 &&
                                                             W != 32 && W != 64)) {
        g_err = "non-null buffers, positive sizes and row_floats in {1, 2, 4, 8, 16, 32, 64} required";
        return -1;
    }
    if ((deg != 8 && deg != 16) || n_idx % 16 != 0 || (vec != 1 && vec != 2 && vec != 4) || vec > W) {
        g_err = "deg 8 or 16, n_idx a multiple of 16, vec 1, 2 or 4 and at most row_floats required";
        return -1;
    }
    if ((uintptr_t)idx % 16 != 0 || (uintptr_t)src % 16 != 0) {
        g_err = "src and idx must be 16-byte aligned";
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_out = n_idx / deg;
    const int64_t threads = n_out * (W / vec);
    const int64_t blocks64 = (threads + 255) / 256;
    if (blocks64 > INT32_MAX) {
        g_err = "too many outputs";
        return -1;
    }
    const int blocks = (int)blocks64;
    auto launch = [&]() -> hipError_t {
        const int v = vec * 100 + deg;
        switch (v) {
            case 108: return launch_gather<1, 8>(src, W, idx, n_out, out, blocks, s);
            case 116: return launch_gather<1, 16>(src, W, idx, n_out, out, blocks, s);
            case 208: return launch_gather<2, 8>(src, W, idx, n_out, out, blocks, s);
            case 216: return launch_gather<2, 16>(src, W, idx, n_out, out, blocks, s);
            case 408: return launch_gather<4, 8>(src, W, idx, n_out, out, blocks, s);
            default: return launch_gather<4, 16>(src, W, idx, n_out, out, blocks, s);
        }
    };
    return timed(launch, iters, s, ms);
}

int32_t hmsp_grid_barrier(int32_t blocks, int32_t rounds, void* stream, double* us, int32_t* gave_up) {
    g_err.clear();
    if (blocks < 1 || rounds < 1 || rounds > (1 << 20) || !us || !gave_up) {
        g_err = "blocks >= 1, 1 <= rounds <= 2^20 and output pointers required";
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    PTRY(hipGetDevice(&dev), "hipGetDevice");
    PTRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev), "hipDeviceGetAttribute");
    PTRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    PTRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_barrier, 256, 0), "occupancy");
    if (!coop || blocks > per_cu * cus) {
        g_err = "cooperative launch unsupported, or more blocks than can be resident at once";
        return -1;
    }
    unsigned* cnt = nullptr;
    PTRY(hipMallocAsync((void**)&cnt, 256, s), "hipMallocAsync");
    struct Free {
        unsigned* p;
        hipStream_t s;
        ~Free() {
            (void)hipStreamSynchronize(s);
            (void)hipFreeAsync(p, s);
        }
    } fr{cnt, s};
    int* flag = reinterpret_cast<int*>(cnt + 32);
    PTRY(hipMemsetAsync(cnt, 0, 256, s), "hipMemsetAsync");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PTRY(hipEventCreate(&e0), "hipEventCreate");
    PTRY(hipEventCreate(&e1), "hipEventCreate");
    struct FreeEv {
        hipEvent_t a, b;
        ~FreeEv() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } fe{e0, e1};
    int limit = 1 << 20;
    void* args[] = {&cnt, &flag, &rounds, &limit};
    PTRY(hipEventRecord(e0, s), "hipEventRecord");
    PTRY(hipLaunchCooperativeKernel((const void*)k_barrier, dim3(blocks), dim3(256), args, 0, s), "cooperative launch");
    PTRY(hipEventRecord(e1, s), "hipEventRecord");
    PTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    float t = 0.0f;
    PTRY(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
    int f = 0;
    PTRY(hipMemcpy(&f, flag, 4, hipMemcpyDeviceToHost), "hipMemcpy");
    *us = (double)t * 1e3 / rounds;
    *gave_up = f;
    return 0;
}

int32_t hmsp_launch_gap(int32_t blocks, int32_t kernels, int32_t graph, void* stream, double* us) {
    g_err.clear();
    if (blocks < 1 || kernels < 1 || kernels > 100000 || !us) {
        g_err = "blocks >= 1, 1 <= kernels <= 100000 and an output pointer required";
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    int* p = nullptr;
    PTRY(hipMallocAsync((void**)&p, 64, s), "hipMallocAsync");
    struct Free {
        int* p;
        hipStream_t s;
        ~Free() {
            (void)hipStreamSynchronize(s);
            (void)hipFreeAsync(p, s);
        }
    } fr{p, s};
    PTRY(hipMemsetAsync(p, 0, 64, s), "hipMemsetAsync");
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipStream_t cs = nullptr;
    struct FreeG {
        hipGraph_t& g;
        hipGraphExec_t& x;
        hipStream_t& cs;
        hipStream_t s;
        ~FreeG() {
            (void)hipStreamSynchronize(s);
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
            if (cs) (void)hipStreamDestroy(cs);
        }
    } fg{g, x, cs, s};
    if (graph) {
        PTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        PTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
        hipError_t ce = hipSuccess;
        for (int i = 0; i < kernels && ce == hipSuccess; ++i) {
            hipLaunchKernelGGL(k_empty, dim3(blocks), dim3(256), 0, cs, p);
            ce = hipGetLastError();
        }
        hipError_t ee = hipStreamEndCapture(cs, &g);
        PTRY(ce, "capture");
        PTRY(ee, "end capture");
        PTRY(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    auto launch = [&]() -> hipError_t {
        if (graph) return hipGraphLaunch(x, s);
        for (int i = 0; i < kernels; ++i) {
            hipLaunchKernelGGL(k_empty, dim3(blocks), dim3(256), 0, s, p);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    double ms = 0.0;
    const int32_t rc = timed(launch, 4, s, &ms);
    if (rc) return rc;
    *us = ms * 1e3 / kernels;
    return 0;
}

}  // extern "C"
