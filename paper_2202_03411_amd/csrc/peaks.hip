// gfx950 machine-peak probes for the roofline fractions of the contraction kernels:
//
//  peak_mfma_kernel  back-to-back matrix-core work on register operands, four
//                    independent accumulator chains per wave, no memory traffic
//                    but one store per thread at the end (so nothing is elided).
//  copy_kernel       a streaming 16-byte-per-lane copy, grid-stride.
//
// They measure what this device sustains, to set beside the published peaks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "msft_internal.h"

namespace msft {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int PK_THREADS = 256;
constexpr int PK_CHAINS = 4;

template <int PREC>
__global__ __launch_bounds__(PK_THREADS) void peak_mfma_kernel(int iters, float seed, float* sink)
{
    const float a = seed + 1e-3f * (float)threadIdx.x, b = seed - 1e-3f * (float)threadIdx.x;
    f32x16 acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = f32x16{};
    if (PREC == MSFT_FP32) {
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < PK_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
        }
    } else {
        bf16x8 av, bv;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            av[k] = (__bf16)(a + 0.125f * k);
            bv[k] = (__bf16)(b - 0.125f * k);
        }
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < PK_CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[c], 0, 0, 0);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[c][r];
    sink[(size_t)blockIdx.x * PK_THREADS + threadIdx.x] = s;
}

// Each thread moves four pieces per round (four loads in flight, then four stores),
// lanes on consecutive pieces; the ragged end goes one piece at a time.
constexpr int CP_UNROLL = 4;
__global__ __launch_bounds__(256) void copy_kernel(const u32x4* src, u32x4* dst, int64_t n)
{
    const int64_t per_round = (int64_t)gridDim.x * blockDim.x * CP_UNROLL;
    const int64_t full = n / per_round * per_round;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * CP_UNROLL + threadIdx.x;
    for (int64_t r = 0; r < full; r += per_round) {
        u32x4 v[CP_UNROLL];
#pragma unroll
        for (int u = 0; u < CP_UNROLL; ++u) v[u] = src[r + base + u * blockDim.x];
#pragma unroll
        for (int u = 0; u < CP_UNROLL; ++u) dst[r + base + u * blockDim.x] = v[u];
    }
    for (int64_t i = full + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

int launch_peak_mfma(int precision, int iters, int nblocks, float* sink, double* flops, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    // real flops of one MFMA: 2 M N K
    const double per = precision == MSFT_FP32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
    *flops = per * PK_CHAINS * (double)iters * (PK_THREADS / 64) * (double)nblocks;
    if (precision == MSFT_FP32)
        hipLaunchKernelGGL(peak_mfma_kernel<MSFT_FP32>, dim3(nblocks), dim3(PK_THREADS), 0, s, iters, 0.5f, sink);
    else
        hipLaunchKernelGGL(peak_mfma_kernel<MSFT_BF16X3>, dim3(nblocks), dim3(PK_THREADS), 0, s, iters, 0.5f,
                           sink);
    return (int)hipGetLastError();
}

int launch_copy(const void* src, void* dst, int64_t pieces, void* stream)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(pieces, 256 * CP_UNROLL), 8 * CHIP_CUS));
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)src, (u32x4*)dst, pieces);
    return (int)hipGetLastError();
}

}  // namespace msft
