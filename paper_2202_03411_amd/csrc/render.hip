// gfx950 shape renderers (Sec. 5.2): the sample's delta, beta on the centred voxel
// grid, ahead of the column scan, and the gradient of a loss with respect to the
// star body's harmonic coefficients.
//
//  render_sh_kernel        r_s(theta, phi) = r0 (1 + sum c_lm Y_lm), occupancy, delta/beta
//  render_sh_grad_kernel   per-workgroup partial sums of dL/dc_lm (FP64 partials)
//  render_sh_grad_reduce   the partials summed in a fixed order
//  render_ellipsoid_kernel quadric body, hard or soft
//  render_volume_kernel    a voxel map on its own grid, resampled (trilinear)
//
// One thread per voxel; directions, radii and the harmonic sums in FP64 (a few
// hundred flops per voxel, microseconds for 128^3), outputs in FP32.
#include <hip/hip_runtime.h>

#include "msft_internal.h"

namespace msft {

// Voxel v = (a * ny + b) * nz + k -> centre, distance, cos(theta), cos/sin(phi);
// the origin looks along +z.
struct VoxelDir {
    double x, y, z, r, ct, st, cp, sp;
};

__device__ __forceinline__ VoxelDir voxel_dir(const RenderGrid& g, int64_t v)
{
    const int k = (int)(v % g.nz);
    const int64_t ab = v / g.nz;
    const int b = (int)(ab % g.ny), a = (int)(ab / g.ny);
    const double x = ((double)(2 * a + 1 - g.nx) * g.dx) / 2.0;
    const double y = ((double)(2 * b + 1 - g.ny) * g.dy) / 2.0;
    const double z = ((double)(2 * k + 1 - g.nz) * g.dz) / 2.0;
    VoxelDir d;
    d.x = x;
    d.y = y;
    d.z = z;
    const double rxy = sqrt(x * x + y * y);
    d.r = sqrt(x * x + y * y + z * z);
    if (d.r > 0.0) {
        d.ct = z / d.r;
        d.st = rxy / d.r;
    } else {
        d.ct = 1.0;
        d.st = 0.0;
    }
    if (rxy > 0.0) {
        d.cp = x / rxy;
        d.sp = y / rxy;
    } else {
        d.cp = 1.0;
        d.sp = 0.0;
    }
    return d;
}

// Visit every real harmonic Y_lm, l <= L, at a direction: f(index l*l + l + m, value).
// Normalised associated Legendre values Q_lm (no Condon-Shortley sign) by the
// recurrences in m (diagonal) and in l (three-term), cos/sin(m phi) by angle
// addition; the recurrence constants come from the host.  L is a compile-time
// bound, so the loops unroll and every index is a constant.
template <int L, typename F>
__device__ __forceinline__ void for_each_ylm(const ShArgs& s, const VoxelDir& d, F f)
{
    const double rt2 = 1.4142135623730950488;
    double qmm = 0.28209479177387814347;   // Q_00 = 1 / sqrt(4 pi)
    double cm = 1.0, sm = 0.0;             // cos(m phi), sin(m phi)
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            qmm *= s.diag[m] * d.st;
            const double c2 = cm * d.cp - sm * d.sp;
            sm = sm * d.cp + cm * d.sp;
            cm = c2;
        }
        double q2 = 0.0, q1 = qmm;   // Q_{l-2,m}, Q_{l-1,m} as l advances
#pragma unroll
        for (int l = m; l <= L; ++l) {
            double q;
            if (l == m) {
                q = qmm;
            } else if (l == m + 1) {
                q = s.sub[m] * d.ct * qmm;
                q2 = qmm;
                q1 = q;
            } else {
                q = s.ra[l * SH_TABLE + m] * (d.ct * q1 - s.rb[l * SH_TABLE + m] * q2);
                q2 = q1;
                q1 = q;
            }
            if (m == 0) {
                f(l * l + l, q);
            } else {
                f(l * l + l + m, rt2 * q * cm);
                f(l * l + l - m, rt2 * q * sm);
            }
        }
    }
}

__device__ __forceinline__ double occupancy(double rs, double r, double edge)
{
    if (edge <= 0.0) return r <= rs ? 1.0 : 0.0;
    return 1.0 / (1.0 + exp(-(rs - r) / edge));
}

// Coefficients into LDS, zero beyond (lmax + 1)^2 up to (L + 1)^2.
template <int L>
__device__ __forceinline__ void load_coeffs(const ShArgs& s, const float* coeffs, float* c)
{
    const int nc = (s.lmax + 1) * (s.lmax + 1);
    for (int k = threadIdx.x; k < (L + 1) * (L + 1); k += blockDim.x) c[k] = k < nc ? coeffs[k] : 0.0f;
}

template <int L>
__global__ __launch_bounds__(256) void render_sh_kernel(ShArgs s, const float* coeffs, float* delta,
                                                        float* beta)
{
    __shared__ float c[(L + 1) * (L + 1)];
    load_coeffs<L>(s, coeffs, c);
    __syncthreads();
    const int64_t nv = (int64_t)s.g.nx * s.g.ny * s.g.nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const VoxelDir d = voxel_dir(s.g, v);
    double acc = 0.0;
    for_each_ylm<L>(s, d, [&](int idx, double y) { acc += (double)c[idx] * y; });
    const double o = occupancy(s.r0 * (1.0 + acc), d.r, s.g.edge);
    delta[v] = (float)(s.g.delta0 * o);
    beta[v] = (float)(s.g.beta0 * o);
}

// dL/dc_lm = sum_v (gd delta0 + gb beta0) o (1 - o) / edge r0 Y_lm.  Each thread
// sums its voxels (grid stride) in FP32 per coefficient, the wave reduces by
// shuffles, the workgroup's four wave sums go to FP64 partials [block][coeff].
template <int L>
__global__ __launch_bounds__(256) void render_sh_grad_kernel(ShArgs s, const float* coeffs,
                                                             const float* gd, const float* gb,
                                                             double* partial)
{
    constexpr int NC = (L + 1) * (L + 1);
    __shared__ float c[NC];
    __shared__ float wsum[4][NC];
    load_coeffs<L>(s, coeffs, c);
    __syncthreads();
    float acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0f;
    const int64_t nv = (int64_t)s.g.nx * s.g.ny * s.g.nz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
        const VoxelDir d = voxel_dir(s.g, v);
        double rs = 0.0;
        for_each_ylm<L>(s, d, [&](int idx, double y) { rs += (double)c[idx] * y; });
        const double o = occupancy(s.r0 * (1.0 + rs), d.r, s.g.edge);
        const double w = ((double)gd[v] * s.g.delta0 + (double)gb[v] * s.g.beta0) * o * (1.0 - o) /
                         s.g.edge * s.r0;
        // Recompute the harmonics from a voxel index the compiler cannot prove equal
        // to v: reusing the first pass's values keeps all (L+1)^2 of them live in FP64
        // across the radius and the weight, which spills at L = 12 (4x slower there).
        int64_t v2 = v;
        asm volatile("" : "+v"(v2));
        const VoxelDir d2 = voxel_dir(s.g, v2);
        for_each_ylm<L>(s, d2, [&](int idx, double y) { acc[idx] += (float)(w * y); });
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        float v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) wsum[wave][k] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NC; k += blockDim.x)
        partial[(int64_t)blockIdx.x * MAX_SH_COEFFS + k] =
            (((double)wsum[0][k] + (double)wsum[1][k]) + (double)wsum[2][k]) + (double)wsum[3][k];
}

// One workgroup per coefficient: thread t adds the partials b = t, t + 256, ... in
// FP64, then a fixed pairwise tree over the 256 threads.  The order is fixed, so
// repeated calls give the same bits.  (One thread per coefficient walking all the
// partials waited on one load at a time: most of the gradient's time.)
__global__ __launch_bounds__(256) void render_sh_grad_reduce(const double* partial, int nblocks, float* grad)
{
    __shared__ double red[256];
    const int k = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblocks; b += 256) s += partial[(int64_t)b * MAX_SH_COEFFS + k];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) grad[k] = (float)red[0];
}

__global__ __launch_bounds__(256) void render_ellipsoid_kernel(EllArgs e, float* delta, float* beta)
{
    const int64_t nv = (int64_t)e.g.nx * e.g.ny * e.g.nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const VoxelDir d = voxel_dir(e.g, v);
    // the voxel centre and its unit direction (+z at the origin) in body coordinates
    const double ux = d.st * d.cp, uy = d.st * d.sp, uz = d.ct;
    double rho2 = 0.0, e2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double pj = d.x * e.rot[0 * 3 + j] + d.y * e.rot[1 * 3 + j] + d.z * e.rot[2 * 3 + j];
        rho2 += (pj / e.ax[j]) * (pj / e.ax[j]);
        const double uj = ux * e.rot[0 * 3 + j] + uy * e.rot[1 * 3 + j] + uz * e.rot[2 * 3 + j];
        e2 += (uj / e.ax[j]) * (uj / e.ax[j]);
    }
    double o;
    if (e.g.edge <= 0.0) o = rho2 <= 1.0 ? 1.0 : 0.0;
    else o = occupancy(1.0 / sqrt(e2), d.r, e.g.edge);
    delta[v] = (float)(e.g.delta0 * o);
    beta[v] = (float)(e.g.beta0 * o);
}

// Volume map: trilinear interpolation between the centres of a source grid
// (also centred on the origin), zero beyond it; FP64 coordinates and weights.
__global__ __launch_bounds__(256) void render_volume_kernel(VolArgs a, const float* sd,
                                                            const float* sb, float* delta, float* beta)
{
    const int64_t nv = (int64_t)a.g.nx * a.g.ny * a.g.nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const VoxelDir d = voxel_dir(a.g, v);
    const double fx = d.x / a.sdx + (a.sx - 1) / 2.0;
    const double fy = d.y / a.sdy + (a.sy - 1) / 2.0;
    const double fz = d.z / a.sdz + (a.sz - 1) / 2.0;
    const double ax = floor(fx), ay = floor(fy), az = floor(fz);
    const double wx = fx - ax, wy = fy - ay, wz = fz - az;
    double vd = 0.0, vb = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t x = (int64_t)ax + i, y = (int64_t)ay + j, z = (int64_t)az + k;
                if (x < 0 || x >= a.sx || y < 0 || y >= a.sy || z < 0 || z >= a.sz) continue;
                const double w = (i ? wx : 1.0 - wx) * (j ? wy : 1.0 - wy) * (k ? wz : 1.0 - wz);
                const int64_t s = (x * a.sy + y) * a.sz + z;
                vd += w * (double)sd[s];
                vb += w * (double)sb[s];
            }
    delta[v] = (float)vd;
    beta[v] = (float)vb;
}

int launch_render_volume(const VolArgs& a, const float* sd, const float* sb, float* delta,
                         float* beta, void* stream)
{
    const int64_t nv = (int64_t)a.g.nx * a.g.ny * a.g.nz;
    hipLaunchKernelGGL(render_volume_kernel, dim3((unsigned)ceil_div(nv, 256)), dim3(256), 0,
                       (hipStream_t)stream, a, sd, sb, delta, beta);
    return (int)hipGetLastError();
}

int launch_render_sh(const ShArgs& s, const float* coeffs, float* delta, float* beta, void* stream)
{
    const int64_t nv = (int64_t)s.g.nx * s.g.ny * s.g.nz;
    const dim3 grid((unsigned)ceil_div(nv, 256));
    hipStream_t st = (hipStream_t)stream;
    if (s.lmax <= 8)
        hipLaunchKernelGGL(render_sh_kernel<8>, grid, dim3(256), 0, st, s, coeffs, delta, beta);
    else
        hipLaunchKernelGGL(render_sh_kernel<MAX_SH_L>, grid, dim3(256), 0, st, s, coeffs, delta, beta);
    return (int)hipGetLastError();
}

int launch_render_sh_grad(const ShArgs& s, const float* coeffs, const float* gd, const float* gb,
                          float* grad, double* partial, int nblocks, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (s.lmax <= 8)
        hipLaunchKernelGGL(render_sh_grad_kernel<8>, dim3((unsigned)nblocks), dim3(256), 0, st, s,
                           coeffs, gd, gb, partial);
    else
        hipLaunchKernelGGL(render_sh_grad_kernel<MAX_SH_L>, dim3((unsigned)nblocks), dim3(256), 0, st,
                           s, coeffs, gd, gb, partial);
    const int nc = (s.lmax + 1) * (s.lmax + 1);
    hipLaunchKernelGGL(render_sh_grad_reduce, dim3((unsigned)nc), dim3(256), 0, st, (const double*)partial,
                       nblocks, grad);
    return (int)hipGetLastError();
}

int launch_render_ellipsoid(const EllArgs& e, float* delta, float* beta, void* stream)
{
    const int64_t nv = (int64_t)e.g.nx * e.g.ny * e.g.nz;
    hipLaunchKernelGGL(render_ellipsoid_kernel, dim3((unsigned)ceil_div(nv, 256)), dim3(256), 0,
                       (hipStream_t)stream, e, delta, beta);
    return (int)hipGetLastError();
}

}  // namespace msft
