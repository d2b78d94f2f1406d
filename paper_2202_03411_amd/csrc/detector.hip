// gfx950 Ideal detector (Sec. 5.2, second example): the photon statistics of a
// real recording laid over the computed intensity.
//
// Expected photons in pixel p: mu_p = F (k0^2 / 4 pi)^2 I_p dOmega_p, the scalar
// first-Born cross section dsigma/dOmega = |k0^2 A / 4 pi|^2 of the volume sum A
// (Eq. (1)) times the incident fluence F and the pixel's solid angle.  The
// recorded count is one Poisson draw of mean mu_p from a counter-based stream:
// Philox4x64-10 (Salmon et al., SC'11) keyed by (seed, 0), block m of pixel p at
// counter (m, p, 0, 0), each 64-bit word giving one uniform from its top 53 bits.
// Means below 10 are drawn by inversion on one uniform; larger ones by Hormann's
// transformed rejection with squeeze (PTRS, 1993), two uniforms per trial.
//
// One thread per pixel, FP64 throughout; memory traffic is 4 bytes in and 4-8
// out per pixel, a few microseconds for 512^2.
#include <hip/hip_runtime.h>

#include "msft_internal.h"

namespace msft {

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

struct Words4 {
    uint64_t w[4];
};

__device__ __forceinline__ Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Words4{{c0, c1, c2, c3}};
}

// Uniforms of one pixel, in stream order.
struct PixelStream {
    uint64_t seed, pixel, m;
    Words4 block;

    __device__ __forceinline__ double next()
    {
        if ((m & 3) == 0) block = philox4x64_10(m >> 2, pixel, 0, 0, seed, 0);
        const uint64_t x = block.w[m & 3];
        ++m;
        return (double)(x >> 11) * 0x1.0p-53;
    }
};

__device__ double poisson_draw(PixelStream& s, double mu)
{
#pragma clang fp contract(off)
    if (!(mu > 0.0) || !isfinite(mu)) return 0.0;
    if (mu < 10.0) {
        const double u = s.next();
        double k = 0.0, p = exp(-mu), cdf = p;
        while (u > cdf && p > 0.0) {
            k += 1.0;
            p = (p * mu) / k;
            cdf += p;
        }
        return k;
    }
    const double sq = sqrt(mu), lg = log(mu);
    const double b = 0.931 + 2.53 * sq;
    const double a = -0.059 + 0.02483 * b;
    const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    const double v_r = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        const double u = s.next() - 0.5;
        const double v = s.next();
        const double us = 0.5 - fabs(u);
        const double k = floor((2.0 * a / us + b) * u + mu + 0.43);
        if (us >= 0.07 && v <= v_r) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        const double hat = log(v) + log(inv_alpha) - log(a / (us * us) + b);
        if (hat <= -mu + k * lg - lgamma(k + 1.0)) return k;
    }
}

// Solid angle of the screen rectangle [0, u] x [0, v] at unit distance (odd in u, v).
__device__ __forceinline__ double corner_angle(double u, double v)
{
#pragma clang fp contract(off)
    return atan((u * v) / sqrt(1.0 + u * u + v * v));
}

__global__ __launch_bounds__(256) void detect_ideal_kernel(IdealArgs a, const float* intensity,
                                                           float* counts, float* expected)
{
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)a.n * a.n;
    if (p >= npix) return;
    const int i = (int)(p % a.n), j = (int)(p / a.n);
    const double u0 = ((double)(2 * i - a.n) * a.t) / (double)a.n;
    const double u1 = ((double)(2 * i + 2 - a.n) * a.t) / (double)a.n;
    const double v0 = ((double)(2 * j - a.n) * a.t) / (double)a.n;
    const double v1 = ((double)(2 * j + 2 - a.n) * a.t) / (double)a.n;
    const double omega = corner_angle(u1, v1) - corner_angle(u0, v1) - corner_angle(u1, v0) +
                         corner_angle(u0, v0);
    const double mu = (a.scale * (double)intensity[p]) * omega;
    PixelStream s{a.seed, (uint64_t)p, 0, {}};
    counts[p] = (float)poisson_draw(s, mu);
    if (expected) expected[p] = (float)mu;
}

}  // namespace

int launch_detect_ideal(const IdealArgs& a, const float* intensity, float* counts, float* expected,
                        void* stream)
{
    const int64_t npix = (int64_t)a.n * a.n;
    hipLaunchKernelGGL(detect_ideal_kernel, dim3((unsigned)ceil_div(npix, 256)), dim3(256), 0,
                       (hipStream_t)stream, a, intensity, counts, expected);
    return (int)hipGetLastError();
}

}  // namespace msft
