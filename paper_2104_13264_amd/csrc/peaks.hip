// Peak probes: one kernel per unit that the sampler and the build lean on,
// each running that unit alone at its highest rate, so that the published
// MI355X peaks can be checked on the chip the kernels run on (the measured
// rate includes the clock the chip holds under that load).
//
//   MFMA f32   v_mfma_f32_16x16x4_f32    (the FP32 sampler's products)
//   MFMA bf16  v_mfma_f32_16x16x32_bf16  (the BF16 sampler's products)
//   MFMA f64   v_mfma_f64_16x16x4_f64    (the FP64 matrix-core sampler)
//   FMA f64    v_fma_f64 on all lanes     (the plain path and the build)
//   HBM read   streaming 16-byte loads of a buffer much larger than the MALL
//   HBM copy   the same, each load stored to a second buffer
//
// Each compute kernel keeps independent accumulation chains (eight; four for
// the 64-cycle FP64 MFMA) per wave and runs four waves per SIMD, enough for
// the units' issue and latency; its
// result is written only if it equals a value it cannot take, which keeps the
// chains live without memory traffic.  The MFMA accumulators stay in the
// accumulation registers: left to itself the register allocator copied them
// between AGPRs and VGPRs on every iteration, and the probe measured the
// copies.  The FP32 probe pins them with an empty asm statement; for the BF16
// and FP64 probes that was not enough, and their MFMAs are issued from asm
// with the accumulator as an in-out operand (AGPRs for BF16, VGPRs for FP64,
// the class the loop kept).  A chain's next MFMA comes at least three MFMAs
// after its last, as in the compiled loops, so the chains need no wait
// states; the accumulators are read only by the liveness check after the
// loop.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tnmh.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;
constexpr int BLOCK = 256;             // four waves
constexpr int COMPUTE_BLOCKS = 1024;   // four per CU: four waves per SIMD
constexpr int MEMORY_BLOCKS = 4096;    // sixteen per CU

__global__ void __launch_bounds__(BLOCK) k_peak_mfma_f32(int iters, float *out) {
    const float a = 1.0f + threadIdx.x * 1e-7f, b = 1.0f - threadIdx.x * 1e-7f;
    floatx4 acc[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < CHAINS; ++k) {
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
            asm volatile("" : "+a"(acc[k]));
        }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (s == -1.0f) out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) k_peak_mfma_bf16(int iters, float *out) {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)(1.0f + j * 0.125f);
        b[j] = (__bf16)(0.5f + (threadIdx.x & 7) * 0.0625f);
    }
    floatx4 acc[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < CHAINS; ++k) {
            asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+a"(acc[k]) : "v"(a), "v"(b));
        }
    // the compiler does not see the MFMAs above: give their results the wait
    // states a vector read of an MFMA result needs, then name the accumulators
    // in asm that follows (volatile asm keeps its order), so that no read of
    // them moves above the wait
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7");
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) asm volatile("" : "+a"(acc[k]));
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (s == -1.0f) out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

// four chains: a 16x16x4 f64 MFMA takes 64 cycles, so a chain's next one
// still comes 192 cycles after its last
constexpr int CHAINS64 = 4;

__global__ void __launch_bounds__(BLOCK) k_peak_mfma_f64(int iters, float *out) {
    const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
    doublex4 acc[CHAINS64];
#pragma unroll
    for (int k = 0; k < CHAINS64; ++k) acc[k] = doublex4{0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < CHAINS64; ++k) {
            asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %2, %0" : "+v"(acc[k]) : "v"(a), "v"(b));
        }
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7");   // as in the BF16 probe
#pragma unroll
    for (int k = 0; k < CHAINS64; ++k) asm volatile("" : "+v"(acc[k]));
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < CHAINS64; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (s == -1.0) out[blockIdx.x * BLOCK + threadIdx.x] = (float)s;
}

// sixteen chains: a v_fma_f64 result is not ready for the next dependent
// instruction of its wave until several issues later
constexpr int CHAINSV = 16;

__global__ void __launch_bounds__(BLOCK) k_peak_fma_f64(int iters, float *out) {
    const double y = 1.0 - 1e-12, z = 1e-13 * threadIdx.x;
    double x[CHAINSV];
#pragma unroll
    for (int k = 0; k < CHAINSV; ++k) x[k] = 1.0 + k * 1e-3;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < CHAINSV; ++k) x[k] = fma(x[k], y, z);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < CHAINSV; ++k) s += x[k];
    if (s == -1.0) out[blockIdx.x * BLOCK + threadIdx.x] = (float)s;
}

// n16: 16-byte words of the buffer; grid-stride with eight loads in flight
constexpr int RD = 8;
__global__ void __launch_bounds__(BLOCK) k_peak_read(const uint4 *__restrict__ p, size_t n16, uint32_t *out) {
    const size_t stride = (size_t)gridDim.x * BLOCK;
    uint32_t acc = 0;
    size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    for (; i + (RD - 1) * stride < n16; i += RD * stride) {
        uint4 v[RD];
#pragma unroll
        for (int u = 0; u < RD; ++u) v[u] = p[i + u * stride];
#pragma unroll
        for (int u = 0; u < RD; ++u) acc ^= (v[u].x ^ v[u].y) ^ (v[u].z ^ v[u].w);
    }
    for (; i < n16; i += stride) {
        const uint4 v = p[i];
        acc ^= (v.x ^ v.y) ^ (v.z ^ v.w);
    }
    if (acc == 0xFFFFFFFFu) out[blockIdx.x * BLOCK + threadIdx.x] = acc;
}

// four loads in flight, then their stores
__global__ void __launch_bounds__(BLOCK) k_peak_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     size_t n16) {
    const size_t stride = (size_t)gridDim.x * BLOCK;
    size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int tn_peak_probe(int kind, long long amount, double *seconds, double *work) {
    (void)hipGetLastError();
    if (!seconds || !work || amount < 1) return TN_EINVAL;
    const bool memory = kind == TN_PEAK_HBM_READ || kind == TN_PEAK_HBM_COPY;
    if (kind < TN_PEAK_MFMA_F32 || kind > TN_PEAK_HBM_COPY) return TN_EINVAL;
    if (!memory && amount > (1LL << 30)) return TN_EINVAL;
    if (memory && (amount % 16 != 0 || amount > (64LL << 30))) return TN_EINVAL;
    const size_t sink_n = (size_t)MEMORY_BLOCKS * BLOCK;   // one slot per thread of the larger grid
    void *sink = nullptr, *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TN_OK;
    auto fail = [&](int code) {
        rc = code;
        return code;
    };
    do {
        if (hipMalloc(&sink, sink_n * sizeof(float)) != hipSuccess) {
            fail(TN_ENOMEM);
            break;
        }
        if (memory) {
            if (hipMalloc(&a, (size_t)amount) != hipSuccess ||
                (kind == TN_PEAK_HBM_COPY && hipMalloc(&b, (size_t)amount) != hipSuccess)) {
                fail(TN_ENOMEM);
                break;
            }
            if (hipMemset(a, 1, (size_t)amount) != hipSuccess) {
                fail(TN_EHIP);
                break;
            }
        }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            fail(TN_EHIP);
            break;
        }
        const int iters = (int)amount;
        const size_t n16 = (size_t)amount / 16;
        auto launch = [&]() {
            switch (kind) {
            case TN_PEAK_MFMA_F32:
                hipLaunchKernelGGL(k_peak_mfma_f32, dim3(COMPUTE_BLOCKS), dim3(BLOCK), 0, 0, iters, (float *)sink);
                break;
            case TN_PEAK_MFMA_BF16:
                hipLaunchKernelGGL(k_peak_mfma_bf16, dim3(COMPUTE_BLOCKS), dim3(BLOCK), 0, 0, iters, (float *)sink);
                break;
            case TN_PEAK_MFMA_F64:
                hipLaunchKernelGGL(k_peak_mfma_f64, dim3(COMPUTE_BLOCKS), dim3(BLOCK), 0, 0, iters, (float *)sink);
                break;
            case TN_PEAK_FMA_F64:
                hipLaunchKernelGGL(k_peak_fma_f64, dim3(COMPUTE_BLOCKS), dim3(BLOCK), 0, 0, iters, (float *)sink);
                break;
            case TN_PEAK_HBM_READ:
                hipLaunchKernelGGL(k_peak_read, dim3(MEMORY_BLOCKS), dim3(BLOCK), 0, 0, (const uint4 *)a, n16,
                                   (uint32_t *)sink);
                break;
            default:
                hipLaunchKernelGGL(k_peak_copy, dim3(MEMORY_BLOCKS), dim3(BLOCK), 0, 0, (const uint4 *)a, (uint4 *)b,
                                   n16);
                break;
            }
        };
        launch();   // warm-up: code object loaded, clocks up
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            fail(TN_EHIP);
            break;
        }
        if (hipEventRecord(e0, 0) != hipSuccess) {
            fail(TN_EHIP);
            break;
        }
        launch();
        float ms = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            fail(TN_EHIP);
            break;
        }
        *seconds = ms * 1e-3;
        const double waves = (double)COMPUTE_BLOCKS * (BLOCK / 64);
        switch (kind) {
        case TN_PEAK_MFMA_F32:   // 16 x 16 x 4 multiply-adds per instruction
            *work = waves * iters * CHAINS * 2.0 * 16 * 16 * 4;
            break;
        case TN_PEAK_MFMA_F64:
            *work = waves * iters * CHAINS64 * 2.0 * 16 * 16 * 4;
            break;
        case TN_PEAK_MFMA_BF16:   // 16 x 16 x 32
            *work = waves * iters * CHAINS * 2.0 * 16 * 16 * 32;
            break;
        case TN_PEAK_FMA_F64:   // one fma per lane and chain
            *work = waves * 64 * (double)iters * CHAINSV * 2.0;
            break;
        case TN_PEAK_HBM_READ:
            *work = (double)n16 * 16;
            break;
        default:   // read and written
            *work = 2.0 * n16 * 16;
            break;
        }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (sink) (void)hipFree(sink);
    return rc;
}
