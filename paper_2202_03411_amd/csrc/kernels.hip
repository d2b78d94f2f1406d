// gfx950 kernels of the MSFT forward model.
//
//  twiddle_*     FP64 phase arguments -> FP32 (or BF16 hi/lo) tables, once per plan.
//  scan_kernel   column scan of the incident field along z and the effective
//                strength w = dV (n^2 - 1) T (Eqs. (6)-(9)), written in the
//                contraction's LDS tile layout.
//  fwd_pair_*    the x-sum as a real-ified complex MFMA contraction (BF16
//                precisions) with the y/z phase-weighted reduction and |A|^2
//                fused behind it.
//  sep_*         the two stages of the separable (uniform-q) detector and its
//                adjoint.
#include <hip/hip_runtime.h>

#include "lds_dma.h"
#include "msft_internal.h"

namespace msft {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pixel of wave tile wt held by lane half h, slot m (0..7) of the MFMA output:
// accumulator rows 8j + 4h + u, u = 0..3, are (pixel 4j + 2h + u/2, re|im).
__device__ __forceinline__ int64_t slot_pixel(int64_t wt, int h, int m)
{
    return wt * WAVE_PIX + 4 * (m >> 1) + 2 * h + (m & 1);
}

// Byte offset of 16-byte slot `slot` of row (h, z) in a W tile; the slot index
// is XOR-swizzled with z so that the 32 lanes reading one slot index from 32
// different rows hit distinct LDS banks.
__device__ __forceinline__ int tile_slot_offset(int h, int z, int slot)
{
    return (h * ZB + z) * ROW_BYTES + ((slot ^ (z & 15)) << 4);
}

// ---------------------------------------------------------------------------
// Twiddle tables (plan time).  T = exp(i phi), phi = -q . r, phases in FP64.
// ---------------------------------------------------------------------------

// FP32 A operand, per (wt, xc): [g 16][lane 64][e 4] floats; step s = 4g + e.
// Lane (h, i): row i = (pixel i/2, c = i&1).  Values: h=0,c=0: Re T; h=0,c=1: Im T;
// h=1,c=0: -Im T; h=1,c=1: Re T, so that row (p, re) . [Wr; Wi] = Re(T W) and
// row (p, im) . [Wr; Wi] = Im(T W).
__global__ void twiddle_txa_f32(float* txa, int64_t total, int64_t npix, int nx, int nxc,
                                const double* q, const double* xs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int e = (int)(idx & 3);
    const int lane = (int)((idx >> 2) & 63);
    const int g = (int)((idx >> 8) & 15);
    const int64_t tile = idx >> 12;
    const int xc = (int)(tile % nxc);
    const int64_t wt = tile / nxc;
    const int h = lane >> 5, i = lane & 31, c = i & 1;
    const int64_t pix = wt * WAVE_PIX + (i >> 1);
    const int x = xc * XC + 4 * g + e;
    float v = 0.0f;
    if (pix < npix && x < nx) {
        double sn, cs;
        sincos(-(q[3 * pix] * xs[x]), &sn, &cs);
        if (h == 0) v = (float)(c == 0 ? cs : sn);
        else v = (float)(c == 0 ? -sn : cs);
    }
    txa[idx] = v;
}

// BF16X3 A operand, per (wt, xc): [s 8][hl 2][lane 64][e 8] bf16; x = 8s + e.
__global__ void twiddle_txa_bf16(__bf16* txa, int64_t total, int64_t npix, int nx, int nxc,
                                 const double* q, const double* xs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one (s, lane, e)
    if (idx >= total) return;
    const int e = (int)(idx & 7);
    const int lane = (int)((idx >> 3) & 63);
    const int s = (int)((idx >> 9) & 7);
    const int64_t tile = idx >> 12;
    const int xc = (int)(tile % nxc);
    const int64_t wt = tile / nxc;
    const int h = lane >> 5, i = lane & 31, c = i & 1;
    const int64_t pix = wt * WAVE_PIX + (i >> 1);
    const int x = xc * XC + 8 * s + e;
    float v = 0.0f;
    if (pix < npix && x < nx) {
        double sn, cs;
        sincos(-(q[3 * pix] * xs[x]), &sn, &cs);
        if (h == 0) v = (float)(c == 0 ? cs : sn);
        else v = (float)(c == 0 ? -sn : cs);
    }
    const __bf16 hi = (__bf16)v;
    const __bf16 lo = (__bf16)(v - (float)hi);
    __bf16* base = txa + tile * (TILE_BYTES / 2) + (int64_t)s * 1024;
    base[lane * 8 + e] = hi;
    base[512 + lane * 8 + e] = lo;
}

// Ty: [wt][y][h][m] complex, exp(-i q_y y) of the pixel in lane half h, slot m.
__global__ void twiddle_ty(float2* ty, int64_t total, int64_t npix, int ny, const double* q,
                           const double* ys)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int m = (int)(idx & 7);
    const int h = (int)((idx >> 3) & 1);
    const int64_t rest = idx >> 4;
    const int y = (int)(rest % ny);
    const int64_t wt = rest / ny;
    const int64_t pix = slot_pixel(wt, h, m);
    float2 v = make_float2(0.0f, 0.0f);
    if (pix < npix) {
        double sn, cs;
        sincos(-(q[3 * pix + 1] * ys[y]), &sn, &cs);
        v = make_float2((float)cs, (float)sn);
    }
    ty[idx] = v;
}

// Tz: [wt][zb][h][z 32][m] complex, exp(-i q_z z) (zero beyond nz, and for a
// pixel whose q_z is not finite: no propagating wave reaches it).
__global__ void twiddle_tz(float2* tz, int64_t total, int64_t npix, int nz, int nzb,
                           const double* q, const double* zs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int m = (int)(idx & 7);
    const int zl = (int)((idx >> 3) & 31);
    const int h = (int)((idx >> 8) & 1);
    const int64_t rest = idx >> 9;
    const int zb = (int)(rest % nzb);
    const int64_t wt = rest / nzb;
    const int64_t pix = slot_pixel(wt, h, m);
    const int z = zb * ZB + zl;
    float2 v = make_float2(0.0f, 0.0f);
    if (pix < npix && z < nz && isfinite(q[3 * pix + 2])) {
        double sn, cs;
        sincos(-(q[3 * pix + 2] * zs[z]), &sn, &cs);
        v = make_float2((float)cs, (float)sn);
    }
    tz[idx] = v;
}

static int grid_for(int64_t total, int block) { return (int)ceil_div(total, block); }

int launch_twiddles(int precision, const Dims& d, const double* q_dev, const double* xs_dev,
                    const double* ys_dev, const double* zs_dev, uint8_t* txa, float* ty,
                    float* tz, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int B = 256;
    const int64_t ttiles = d.nwt * d.nxc;
    if (precision == MSFT_FP32) {
        const int64_t total = ttiles * (TILE_BYTES / 4);
        hipLaunchKernelGGL(twiddle_txa_f32, dim3(grid_for(total, B)), dim3(B), 0, s,
                           (float*)txa, total, d.npix, d.nx, d.nxc, q_dev, xs_dev);
    } else {
        const int64_t total = ttiles * (TILE_BYTES / 4);  // (s, lane, e) triples per tile
        hipLaunchKernelGGL(twiddle_txa_bf16, dim3(grid_for(total, B)), dim3(B), 0, s,
                           (__bf16*)txa, total, d.npix, d.nx, d.nxc, q_dev, xs_dev);
    }
    const int64_t nty = d.nwt * d.ny * WAVE_PIX;
    hipLaunchKernelGGL(twiddle_ty, dim3(grid_for(nty, B)), dim3(B), 0, s, (float2*)ty, nty,
                       d.npix, d.ny, q_dev, ys_dev);
    const int64_t ntz = d.nwt * d.nzb * 2 * ZB * 8;
    hipLaunchKernelGGL(twiddle_tz, dim3(grid_for(ntz, B)), dim3(B), 0, s, (float2*)tz, ntz,
                       d.npix, d.nz, d.nzb, q_dev, zs_dev);
    return (int)hipGetLastError();
}

static void launch_txa(int precision, uint8_t* txa, int64_t nwt, int64_t npix, int nx, int nxc,
                       const double* q, const double* xs, hipStream_t s)
{
    const int B = 256;
    const int64_t total = nwt * nxc * (TILE_BYTES / 4);
    if (precision == MSFT_FP32)
        hipLaunchKernelGGL(twiddle_txa_f32, dim3(grid_for(total, B)), dim3(B), 0, s, (float*)txa,
                           total, npix, nx, nxc, q, xs);
    else
        hipLaunchKernelGGL(twiddle_txa_bf16, dim3(grid_for(total, B)), dim3(B), 0, s, (__bf16*)txa,
                           total, npix, nx, nxc, q, xs);
}

// Tables of the separable detector: A operands exp(-i q_x(i) x) of the first
// stage and exp(-i q_y(j) y) of the second (the q arrays hold the one component
// in slot 0), and Tz over the second stage's pixel order (i, j).
int launch_sep_twiddles(int precision, const Dims& d, const SepDims& sd, const double* qcol,
                        const double* qrow, const double* qk, const double* xs, const double* ys,
                        const double* zs, uint8_t* txa1, uint8_t* txa2, float* tz, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int B = 256;
    // (the Gauss form has its own A tables: txa1 and txa2 null)
    if (txa1) launch_txa(precision, txa1, sd.nblk1 * WAVES, sd.n, d.nx, d.nxc, qcol, xs, s);
    if (txa2) launch_txa(precision, txa2, sd.npad / WAVE_PIX, sd.n, d.ny, sd.nyc, qrow, ys, s);
    const int64_t nwt2 = (int64_t)sd.n * (sd.npad / WAVE_PIX);
    const int64_t ntz = nwt2 * d.nzb * 2 * ZB * 8;
    hipLaunchKernelGGL(twiddle_tz, dim3(grid_for(ntz, B)), dim3(B), 0, s, (float2*)tz, ntz,
                       (int64_t)sd.n * sd.npad, d.nz, d.nzb, qk, zs);
    return (int)hipGetLastError();
}

// Four BF16 values as one 8-byte piece, first value lowest.
__device__ __forceinline__ uint2 pack_bf16x4(__bf16 a, __bf16 b, __bf16 c, __bf16 d)
{
    union { __bf16 h[4]; uint2 u; } v;
    v.h[0] = a;
    v.h[1] = b;
    v.h[2] = c;
    v.h[3] = d;
    return v.u;
}

// ---------------------------------------------------------------------------
// Column scan (Eq. (8)) and effective strength (Eqs. (6), (9)).
//
// Workgroup (block of 32 columns x, y), 4 waves, four z blocks of 32 slices per
// round: wave w takes z block zb0 + w of the 32 columns.  Lanes run along z: lane
// (zs, cc) holds slices 4 zs .. 4 zs + 3 of the block for 4 columns, so the 8 lanes
// of a group read one 128-byte line of delta and one of beta per column.  The
// exclusive prefix S = sum_{s'<s} (beta + i delta) of a slice is the carry of the
// earlier rounds, plus the totals of the earlier z blocks of the round (through
// LDS), plus an inclusive shuffle scan over the 8 lanes of the group, plus the
// lane's own earlier slices.  Then
//   T = exp(-k0 dz (S_beta + i S_delta)),   w = dV chi T,
//   chi = n^2 - 1 = delta (delta - 2) - beta^2 + 2 i beta (1 - delta)
// (chi written without the cancelling "+1 -1").  The lane's 4 columns are the 4 x
// of one 16-byte slot of the W tile layout (x = 8 g + 2 e + h in the Gauss layout,
// 4 consecutive x otherwise), so it writes w straight to the workspace: per slice,
// one 16-byte slot per plane (Gauss, FP32) or per re/im row (FP32), two 8-byte
// pieces per row (BF16 hi, lo).  Workgroups are small and need no staging, so
// several share a CU and their loads, arithmetic and stores overlap.
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ZROUND = 4;   // z blocks per round, one wave each
constexpr int SCAN_XB = 32;      // columns per workgroup

// One step of the 8-lane inclusive scans: lane l takes lane l - OFF of its 16-lane row
// (a DPP row shift, no LDS traffic) and adds it when that lane is in its group.
template <int OFF>
__device__ __forceinline__ void scan8_step(float& b, float& d, int zs)
{
    const float tb = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(b), 0x110 + OFF, 0xF, 0xF, false));
    const float td = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), 0x110 + OFF, 0xF, 0xF, false));
    if (zs >= OFF) {
        b += tb;
        d += td;
    }
}

template <int PREC, bool G3>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(ScanArgs a)
{
    __shared__ float tot[2][SCAN_ZROUND][SCAN_XB];   // block totals of beta and delta per column
    const int xb = blockIdx.x, y = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, zr = tid >> 6;
    const int zs = lane & 7, cc = lane >> 3;
    // the lane's columns within the block: one tile slot
    auto col_of = [&](int e) { return G3 ? 8 * (cc >> 1) + 2 * e + (cc & 1) : 4 * cc + e; };
    const bool vec = (a.nz & 3) == 0;
    float carry_b[4], carry_d[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) carry_b[e] = carry_d[e] = 0.0f;

    for (int zb0 = 0; zb0 < a.nzb; zb0 += SCAN_ZROUND) {
        const int zb = zb0 + zr;
        const bool active = zb < a.nzb;
        const int z0 = zb * ZB + 4 * zs;
        float d[4][4], b[4][4], sb[4], sd[4], ib[4], id[4];
        // A wave whose 32 x 32 block lies inside the grid issues its 8 loads at once
        // under one branch (a guard per column would wait for each column in turn).
        if (active && vec && (xb + 1) * SCAN_XB <= a.nx && (zb + 1) * ZB <= a.nz) {
            float4 dv[4], bv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const size_t col = ((size_t)(xb * SCAN_XB + col_of(e)) * a.ny + y) * a.nz + z0;
                dv[e] = *(const float4*)(a.delta + col);
                bv[e] = *(const float4*)(a.beta + col);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                d[e][0] = dv[e].x; d[e][1] = dv[e].y; d[e][2] = dv[e].z; d[e][3] = dv[e].w;
                b[e][0] = bv[e].x; b[e][1] = bv[e].y; b[e][2] = bv[e].z; b[e][3] = bv[e].w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = xb * SCAN_XB + col_of(e);
                const size_t col = ((size_t)x * a.ny + y) * a.nz;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool in = active && x < a.nx && z0 + k < a.nz;
                    d[e][k] = in ? a.delta[col + z0 + k] : 0.0f;
                    b[e][k] = in ? a.beta[col + z0 + k] : 0.0f;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sb[e] = (b[e][0] + b[e][1]) + (b[e][2] + b[e][3]);
            sd[e] = (d[e][0] + d[e][1]) + (d[e][2] + d[e][3]);
            // inclusive scan over the 8 lanes (z segments) of the column's group: DPP
            // shifts inside the 16-lane row; a lane adds only when the source lies in
            // its own group (zs >= off)
            ib[e] = sb[e];
            id[e] = sd[e];
            scan8_step<1>(ib[e], id[e], zs);
            scan8_step<2>(ib[e], id[e], zs);
            scan8_step<4>(ib[e], id[e], zs);
            if (zs == 7) {
                tot[0][zr][col_of(e)] = ib[e];
                tot[1][zr][col_of(e)] = id[e];
            }
        }
        __syncthreads();
        float pb[4], pd[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int xl = col_of(e);
            float eb = carry_b[e], ed = carry_d[e];
            for (int k = 0; k < zr; ++k) {
                eb += tot[0][k][xl];
                ed += tot[1][k][xl];
            }
            pb[e] = eb + (ib[e] - sb[e]);
            pd[e] = ed + (id[e] - sd[e]);
            for (int k = zr; k < SCAN_ZROUND && zb0 + k < a.nzb; ++k) {
                eb += tot[0][k][xl];
                ed += tot[1][k][xl];
            }
            carry_b[e] = eb;
            carry_d[e] = ed;
        }
        // the next round rewrites tot only after every wave has read it
        __syncthreads();
        if (!active) continue;
        float wr[4][4], wi[4][4];   // [slice k][column e]
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float Sb = pb[e], Sd = pd[e];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (a.strength == MSFT_STRENGTH_DENSITY) {
                    wr[k][e] = a.dV * d[e][k];
                    wi[k][e] = a.dV * b[e][k];
                } else {
                    const float chr = d[e][k] * (d[e][k] - 2.0f) - b[e][k] * b[e][k];
                    const float chi = 2.0f * b[e][k] * (1.0f - d[e][k]);
                    float tr = 1.0f, ti = 0.0f;
                    if (a.strength == MSFT_STRENGTH_MSFT) {
                        const float mag = expf(-a.k0dz * Sb);
                        float sn, cs;
                        sincosf(-a.k0dz * Sd, &sn, &cs);
                        tr = mag * cs;
                        ti = mag * sn;
                    }
                    wr[k][e] = a.dV * (chr * tr - chi * ti);
                    wi[k][e] = a.dV * (chr * ti + chi * tr);
                }
                Sb += b[e][k];
                Sd += d[e][k];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int zl = 4 * zs + k;
            if (G3) {
                // Gauss tile (xb, zb, y): rows (plane, h, z) of 4 slots, slot g ^ g3_swizzle(z)
                uint8_t* row = a.wtiles + ((size_t)(xb * a.nzb + zb) * a.ny + y) * G3_TILE_BYTES +
                               ((cc & 1) * ZB + zl) * G3_ROW_BYTES + (((cc >> 1) ^ g3_swizzle(zl)) << 4);
                *(f32x4*)row = f32x4{wr[k][0], wr[k][1], wr[k][2], wr[k][3]};
                *(f32x4*)(row + 2 * ZB * G3_ROW_BYTES) = f32x4{wi[k][0], wi[k][1], wi[k][2], wi[k][3]};
                *(f32x4*)(row + 4 * ZB * G3_ROW_BYTES) = f32x4{wr[k][0] + wi[k][0], wr[k][1] + wi[k][1],
                                                              wr[k][2] + wi[k][2], wr[k][3] + wi[k][3]};
            } else {
                // W tile (xb / 2, zb, y): x = 32 (xb % 2) + 4 cc + e of its 64
                uint8_t* tile = a.wtiles + ((size_t)((xb >> 1) * a.nzb + zb) * a.ny + y) * TILE_BYTES;
                const int xl = 32 * (xb & 1) + 4 * cc;
                if (PREC == MSFT_FP32) {
                    *(f32x4*)(tile + tile_slot_offset(0, zl, xl >> 2)) = f32x4{wr[k][0], wr[k][1], wr[k][2], wr[k][3]};
                    *(f32x4*)(tile + tile_slot_offset(1, zl, xl >> 2)) = f32x4{wi[k][0], wi[k][1], wi[k][2], wi[k][3]};
                } else {
                    __bf16 rh[4], rl[4], ih[4], il[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        rh[e] = (__bf16)wr[k][e];
                        rl[e] = (__bf16)(wr[k][e] - (float)rh[e]);
                        ih[e] = (__bf16)wi[k][e];
                        il[e] = (__bf16)(wi[k][e] - (float)ih[e]);
                    }
                    const int sub = (xl & 7) * 2;
                    *(uint2*)(tile + tile_slot_offset(0, zl, xl >> 3) + sub) = pack_bf16x4(rh[0], rh[1], rh[2], rh[3]);
                    *(uint2*)(tile + tile_slot_offset(0, zl, 8 + (xl >> 3)) + sub) = pack_bf16x4(rl[0], rl[1], rl[2], rl[3]);
                    *(uint2*)(tile + tile_slot_offset(1, zl, xl >> 3) + sub) = pack_bf16x4(ih[0], ih[1], ih[2], ih[3]);
                    *(uint2*)(tile + tile_slot_offset(1, zl, 8 + (xl >> 3)) + sub) = pack_bf16x4(il[0], il[1], il[2], il[3]);
                }
            }
        }
    }
}

int launch_scan(int precision, const ScanArgs& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)ceil_div(a.nx, SCAN_XB), a.ny);
    if (precision == MSFT_FP32 && a.g3)
        hipLaunchKernelGGL((scan_kernel<MSFT_FP32, true>), grid, dim3(SCAN_THREADS), 0, s, a);
    else if (precision == MSFT_FP32)
        hipLaunchKernelGGL((scan_kernel<MSFT_FP32, false>), grid, dim3(SCAN_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((scan_kernel<MSFT_BF16X3, false>), grid, dim3(SCAN_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward contraction for one pixel block (BLOCK_PIX pixels, one workgroup).
//
//   for each x chunk xc:     A operand (Tx of a wave tile's 16 pixels) -> registers
//     for each z block zb:   G = 0
//       for each y:          C = A . W(xc, zb, y)           (MFMA, K = 2 * 64)
//                            G += exp(-i q_y y) C           (per pixel, lane = z)
//       acc += exp(-i q_z z) G
//   A_p = sum over the 32 z lanes of acc;  I_p = |A_p|^2
//
// W tiles stream through a double-buffered LDS ring shared by the workgroup's
// waves.  The order of every sum depends only on the plan, never on the launch.
// ---------------------------------------------------------------------------
// C += A . B for one W tile: the wave's A operand (registers) times the tile's
// column `col` of lane half h (LDS row `row`), over the first `nx` x values.
// FP32: 4 x values per 16-byte LDS slot, one v_mfma_f32_32x32x2_f32 per x.
// BF16X3: 8 x values per slot, hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16;
// BF16 (plain): hi*hi only, from the same tables.
template <int PREC, int NX>
__device__ __forceinline__ f32x16 tile_mfma(f32x16 C, const uint8_t* row, int col, const f32x4* Af,
                                            const bf16x8* Ahi, const bf16x8* Alo)
{
    const int sw = col & 15;
    if (PREC == MSFT_FP32) {
#pragma unroll
        for (int g = 0; g < NX / 4; ++g) {
            const f32x4 b = *(const f32x4*)(row + ((g ^ sw) << 4));
            C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][0], b[0], C, 0, 0, 0);
            C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][1], b[1], C, 0, 0, 0);
            C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][2], b[2], C, 0, 0, 0);
            C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][3], b[3], C, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < NX / 8; ++s) {
            const bf16x8 bh = *(const bf16x8*)(row + ((s ^ sw) << 4));
            C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi[s], bh, C, 0, 0, 0);
            if (PREC == MSFT_BF16X3) {
                const bf16x8 bl = *(const bf16x8*)(row + (((8 + s) ^ sw) << 4));
                C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi[s], bl, C, 0, 0, 0);
                C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Alo[s], bh, C, 0, 0, 0);
            }
        }
    }
    return C;
}

// The last, partial x chunk: the same products in steps of 8 x values.
template <int PREC>
__device__ __forceinline__ f32x16 tile_mfma_partial(f32x16 C, const uint8_t* row, int col, int nx,
                                                 const f32x4* Af, const bf16x8* Ahi,
                                                 const bf16x8* Alo)
{
    const int sw = col & 15;
#pragma unroll
    for (int s = 0; s < XC / 8; ++s) {
        if (8 * s < nx) {
            if (PREC == MSFT_FP32) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int g = 2 * s + u;
                    const f32x4 b = *(const f32x4*)(row + ((g ^ sw) << 4));
                    C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][0], b[0], C, 0, 0, 0);
                    C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][1], b[1], C, 0, 0, 0);
                    C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][2], b[2], C, 0, 0, 0);
                    C = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][3], b[3], C, 0, 0, 0);
                }
            } else {
                const bf16x8 bh = *(const bf16x8*)(row + ((s ^ sw) << 4));
                C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi[s], bh, C, 0, 0, 0);
                if (PREC == MSFT_BF16X3) {
                    const bf16x8 bl = *(const bf16x8*)(row + (((8 + s) ^ sw) << 4));
                    C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi[s], bl, C, 0, 0, 0);
                    C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Alo[s], bh, C, 0, 0, 0);
                }
            }
        }
    }
    return C;
}

// The wave's A operand for one x chunk (one A tile of the table) into registers.
template <int PREC>
__device__ __forceinline__ void load_a(const uint8_t* ta, int lane, f32x4* Af, bf16x8* Ahi,
                                       bf16x8* Alo)
{
    if (PREC == MSFT_FP32) {
#pragma unroll
        for (int g = 0; g < 16; ++g) Af[g] = ((const f32x4*)ta)[g * 64 + lane];
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            Ahi[s] = ((const bf16x8*)ta)[s * 128 + lane];
            if (PREC == MSFT_BF16X3) Alo[s] = ((const bf16x8*)ta)[s * 128 + 64 + lane];
        }
    }
}

// C = A . B of one tile: FULL when the chunk is known to hold XC x values,
// otherwise chosen per tile from xlen.
template <int PREC, bool FULL>
__device__ __forceinline__ f32x16 tile_product(const uint8_t* row, int col, int xlen, const f32x4* Af,
                                               const bf16x8* Ahi, const bf16x8* Alo)
{
    const f32x16 zero = {};
    if (FULL || xlen == XC) return tile_mfma<PREC, XC>(zero, row, col, Af, Ahi, Alo);
    return tile_mfma_partial<PREC>(zero, row, col, xlen, Af, Ahi, Alo);
}

// G[m] += Ty[m] * C[m] for the 8 complex slots m = 2j + u of a lane: C rows
// 4j + 2u (re) and 4j + 2u + 1 (im) of the MFMA result; ty: 4 x f32x4 of Ty.
// Each component takes two chained FMAs into G.
__device__ __forceinline__ void rotate_add(float* G, const f32x16& C, const f32x4* ty)
{
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int r = 4 * (m >> 1) + 2 * (m & 1);
        const float tr = ty[m >> 1][2 * (m & 1)], ti = ty[m >> 1][2 * (m & 1) + 1];
        G[2 * m] = __builtin_fmaf(-ti, C[r + 1], __builtin_fmaf(tr, C[r], G[2 * m]));
        G[2 * m + 1] = __builtin_fmaf(ti, C[r], __builtin_fmaf(tr, C[r + 1], G[2 * m + 1]));
    }
}

// ---------------------------------------------------------------------------
// The flat detector's BF16 contraction, two wave tiles per wave.  A workgroup of
// PW_WAVES waves takes one pixel block; wave v owns the wave tiles wt0 = 8 block +
// 2 v and wt0 + 1 (32 pixels, two MFMA row tiles) and keeps both A operands of an
// x chunk in registers, so each B fragment read from LDS feeds six MFMAs instead of
// three.  Two workgroups share a CU (256 registers per lane), so that one
// workgroup's barrier and Ty rotation run under the other's matrix work.  Each slot
// of a two-slot LDS ring holds one W tile (rows padded, below) and the Ty rows of
// the block's 8 wave tiles at that tile's y; the next slot is filled by direct global -> LDS loads
// issued at the start of each stage, under the stage's MFMA chain.  The per-lane
// sums over z blocks live in LDS.  Measured against one workgroup of 8 waves with
// one wave tile each (128³ / 512², BF16 split): 7.33 ms against 8.29; a third
// ring slot with the z-lane sums taken per z block measured 7.66 ms.
// ---------------------------------------------------------------------------
constexpr int PW_WAVES = 4;
constexpr int PW_THREADS = 64 * PW_WAVES;
// In LDS a W tile row is padded by one 16-byte piece (272 bytes): the 16 lanes of a
// ds_read_b128 group (16 consecutive rows) then start 4 banks apart and meet all 64
// banks, and a lane reads every slot of its row at an immediate offset from one row
// address.  The pad pieces are filled with a copy of the row's first piece.
constexpr int PW_ROW = ROW_BYTES + 16;                     // 272
constexpr int PW_ROWS = 2 * ZB;                            // 64 rows (h, z)
constexpr int PW_PIECES = PW_ROWS * (PW_ROW / 16);         // 1088 pieces of 16 bytes
constexpr int PW_TILE = PW_ROWS * PW_ROW;                  // 17408 bytes
constexpr int PW_COPY = PW_PIECES / PW_THREADS;            // 4 whole passes (wave 0: a fifth)
constexpr int PW_TY_BYTES = WAVES * WAVE_PIX * 8;          // Ty of a block's wave tiles at one y
constexpr int PW_SLOT = PW_TILE + PW_TY_BYTES;
static_assert(PW_PIECES == PW_COPY * PW_THREADS + 64, "four passes plus one wave's pieces");
static_assert(2 * PW_WAVES == WAVES && PW_TY_BYTES == 64 * 16, "one wave gathers the Ty rows");
static_assert(ROW_BYTES == 256 && TILE_BYTES == PW_ROWS * ROW_BYTES, "a W tile is 64 rows of 16 slots");
// Byte offset in the tile of the global piece for LDS piece p: row p / 17, slot
// p % 17 (the pad slot 16 takes the row's slot 0); a row's logical slot k sits at
// global slot k ^ (row % 16).
__device__ __forceinline__ uint32_t pw_src_bytes(int p)
{
    const int row = p / (PW_ROW / 16), k = p % (PW_ROW / 16);
    return 16u * (uint32_t)(row * 16 + (k < 16 ? (k ^ (row & 15)) : (row & 15)));
}
// Slot contents for tile tn (whose y is yn): the padded W tile (waves 0-3 four
// passes, wave 0 the last 64 pieces) and, from wave 1, the block's Ty rows at yn.
// src: the lane's byte offsets in the tile for passes 0-4, and (last) its byte offset
// in the block's Ty rows at one y.  Bases are wave-uniform, offsets 32-bit.
__device__ __forceinline__ void pw_fill(const FwdArgs& a, int64_t wtb, int tn, int yn, const u32x4* gw,
                                        uint8_t* slot, const uint32_t (&src)[PW_COPY + 2])
{
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const u32x4* tile = gw + (size_t)tn * (TILE_BYTES / 16);
#pragma unroll
    for (int c = 0; c < PW_COPY; ++c) lds_dma16_s(tile, src[c], slot + (c * PW_THREADS + wave * 64) * 16);
    if (wave == 0) lds_dma16_s(tile, src[PW_COPY], slot + PW_COPY * PW_THREADS * 16);
    if (wave == 1) lds_dma16_s(a.ty + 2 * (wtb * a.ny + yn) * WAVE_PIX, src[PW_COPY + 1], slot + PW_TILE);
}

// C0, C1 = the wave's two row tiles against one W tile; each B fragment read once.
// row: the lane's padded row in the current slot; slot s of the tile's logical order
// is at row + 16 s.  A fixed instruction order (LDS reads: mask 0x100, MFMA: 0x008)
// issues the reads of steps 0 and 1 first and then, after each step's products, the
// reads of step s + 2, so each read lands under a whole step of matrix work.
template <int PREC, bool FULL>
__device__ __forceinline__ void tile_product2(const uint8_t* row, int xlen, const bf16x8* Ah0,
                                              const bf16x8* Al0, const bf16x8* Ah1, const bf16x8* Al1,
                                              f32x16& C0, f32x16& C1)
{
    auto rd = [&](int slot) { return *(const bf16x8*)(row + 16 * slot); };
    C0 = f32x16{};
    C1 = f32x16{};
    bf16x8 bh = rd(0), bl = PREC == MSFT_BF16X3 ? rd(8) : bh;
#pragma unroll
    for (int s = 0; s < XC / 8; ++s) {
        bf16x8 nh = bh, nl = bl;
        if (s + 1 < XC / 8 && (FULL || 8 * (s + 1) < xlen)) {
            nh = rd(s + 1);
            if (PREC == MSFT_BF16X3) nl = rd(8 + s + 1);
        }
        if (FULL || 8 * s < xlen) {
            C0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah0[s], bh, C0, 0, 0, 0);
            C1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah1[s], bh, C1, 0, 0, 0);
            if (PREC == MSFT_BF16X3) {
                C0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah0[s], bl, C0, 0, 0, 0);
                C1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah1[s], bl, C1, 0, 0, 0);
                C0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al0[s], bh, C0, 0, 0, 0);
                C1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al1[s], bh, C1, 0, 0, 0);
            }
        }
        bh = nh;
        bl = nl;
    }
    if (FULL && PREC == MSFT_BF16X3) {
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int s = 0; s < XC / 8; ++s) {
            __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
            if (s + 2 < XC / 8) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        }
    } else if (FULL) {
        // plain BF16: one read and 2 products per step, in the same order
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int s = 0; s < XC / 8; ++s) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            if (s + 2 < XC / 8) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
    }
}

// All z blocks of one x chunk; tile t sits in slot t & 1.  accl: the lane's 32 sums
// in LDS, stride 64 floats ([row tile][16]).
template <int PREC, bool FULL>
__device__ __forceinline__ void chunk_pair(const FwdArgs& a, int64_t wt0, int ntiles, const u32x4* gw,
                                           uint8_t* lds, int xlen, const bf16x8* Ah0, const bf16x8* Al0,
                                           const bf16x8* Ah1, const bf16x8* Al1, int& t, float* accl,
                                           const uint32_t (&src)[PW_COPY + 2])
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t wtb = wt0 - 2 * wave;
    for (int zb = 0; zb < a.nzb; ++zb) {
        float G0[16], G1[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) G0[q] = G1[q] = 0.0f;
        for (int y = 0; y < a.ny; ++y, ++t) {
            // the next slot (the last tile again at the very end, with y = 0: a slot
            // nobody reads again); tiles run y fastest
            pw_fill(a, wtb, min(t + 1, ntiles - 1), y + 1 == a.ny ? 0 : y + 1, gw,
                    lds + (size_t)((t + 1) & 1) * PW_SLOT, src);
            const uint8_t* cur = lds + (size_t)(t & 1) * PW_SLOT;
            f32x16 C0, C1;
            // matrix work at raised priority: a SIMD's other wave (of the other
            // workgroup) fills the gaps with its rotation and barrier
            __builtin_amdgcn_s_setprio(1);
            tile_product2<PREC, FULL>(cur + (h * ZB + col) * PW_ROW, xlen, Ah0, Al0, Ah1, Al1, C0, C1);
            __builtin_amdgcn_s_setprio(0);
            const f32x4* ty0 = (const f32x4*)(cur + PW_TILE + (2 * wave) * 128 + h * 64);
            const f32x4 t0[4] = {ty0[0], ty0[1], ty0[2], ty0[3]};
            rotate_add(G0, C0, t0);
            const f32x4* ty1 = (const f32x4*)(cur + PW_TILE + (2 * wave + 1) * 128 + h * 64);
            const f32x4 t1[4] = {ty1[0], ty1[1], ty1[2], ty1[3]};
            rotate_add(G1, C1, t1);
            // the next slot's loads have landed (the compiler does not track them)
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            __syncthreads();
        }
        // acc[r][m] += Tz[m] * G_r[m] for the two wave tiles
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const f32x4* tzp = (const f32x4*)(a.tz + 2 * (((((wt0 + r) * a.nzb + zb) * 2 + h) * ZB + col) * 8));
            const float* G = r == 0 ? G0 : G1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 v = tzp[q];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int m = 2 * q + u;
                    const float tr = v[2 * u], ti = v[2 * u + 1];
                    accl[(16 * r + 2 * m) * 64] += tr * G[2 * m] - ti * G[2 * m + 1];
                    accl[(16 * r + 2 * m + 1) * 64] += tr * G[2 * m + 1] + ti * G[2 * m];
                }
            }
        }
    }
}

template <int PREC>
__device__ __forceinline__ void fwd_pair_block(const FwdArgs& a, int64_t block, uint8_t* lds, float* accs)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t wtb = block * WAVES;
    const int64_t wt0 = wtb + 2 * wave;
    const int ntiles = a.nxc * a.nzb * a.ny;   // tiles of W (at most a few million)
    const u32x4* gw = (const u32x4*)a.wtiles;

    // the lane's byte offsets for the five tile passes (the fifth only on wave 0) and
    // for the Ty rows (wave 1): wave tile wtb + lane / 8, piece lane % 8, at one y
    uint32_t src[PW_COPY + 2];
#pragma unroll
    for (int c = 0; c < PW_COPY; ++c) src[c] = pw_src_bytes(c * PW_THREADS + tid);
    src[PW_COPY] = pw_src_bytes(PW_COPY * PW_THREADS + lane);
    src[PW_COPY + 1] = (uint32_t)(((lane >> 3) * a.ny * 2 * WAVE_PIX + (lane & 7) * 4) * sizeof(float));
    pw_fill(a, wtb, 0, 0, gw, lds, src);
    float* accl = accs + wave * 32 * 64 + lane;
#pragma unroll
    for (int q = 0; q < 32; ++q) accl[q * 64] = 0.0f;
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __syncthreads();

    int t = 0;
    for (int xc = 0; xc < a.nxc; ++xc) {
        const int xlen = min(XC, a.x_pad - xc * XC);
        f32x4 Af[16];
        bf16x8 Ah0[8], Al0[8], Ah1[8], Al1[8];
        load_a<PREC>(a.txa + (size_t)(wt0 * a.nxc + xc) * TILE_BYTES, lane, Af, Ah0, Al0);
        load_a<PREC>(a.txa + (size_t)((wt0 + 1) * a.nxc + xc) * TILE_BYTES, lane, Af, Ah1, Al1);
        // one wait for the A operands per chunk (the memory counter is in order)
        __builtin_amdgcn_s_waitcnt(0);
        if (xlen == XC)
            chunk_pair<PREC, true>(a, wt0, ntiles, gw, lds, xlen, Ah0, Al0, Ah1, Al1, t, accl, src);
        else
            chunk_pair<PREC, false>(a, wt0, ntiles, gw, lds, xlen, Ah0, Al0, Ah1, Al1, t, accl, src);
    }
    const int h = lane >> 5, col = lane & 31;
    // sum over the 32 z lanes of each half (fixed butterfly order)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float v = accl[(16 * r + q) * 64];
            v += __shfl_xor(v, 16, 32);
            v += __shfl_xor(v, 8, 32);
            v += __shfl_xor(v, 4, 32);
            v += __shfl_xor(v, 2, 32);
            v += __shfl_xor(v, 1, 32);
            acc[q] = v;
        }
        if (col == 0) {
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int64_t pix = slot_pixel(wt0 + r, h, m);
                if (pix < a.npix) {
                    const float re = acc[2 * m], im = acc[2 * m + 1];
                    a.intensity[pix] = re * re + im * im;
                    if (a.amplitude) ((float2*)a.amplitude)[pix] = make_float2(re, im);
                }
            }
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(PW_THREADS, 2) void fwd_pair_kernel(FwdArgs a, int64_t block_begin)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * PW_SLOT];
    __shared__ float accs[PW_WAVES * 32 * 64];
    fwd_pair_block<PREC>(a, block_begin + blockIdx.x, lds, accs);
}

// Batched form: one workgroup per (request, pixel block) item, in the host's order.
template <int PREC>
__global__ __launch_bounds__(PW_THREADS, 2) void fwd_pair_batch_kernel(BatchArgs b)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * PW_SLOT];
    __shared__ float accs[PW_WAVES * 32 * 64];
    const int32_t it = blockIdx.x;
    int r = 0;
    while (r + 1 < b.nreq && b.item_begin[r + 1] <= it) ++r;
    fwd_pair_block<PREC>(b.req[r], (int64_t)b.block_begin[r] + (it - b.item_begin[r]), lds, accs);
}

int launch_forward(int precision, const FwdArgs& a, int64_t block_begin, int64_t nblocks, void* stream)
{
    if (nblocks <= 0) return 0;
    if (precision == MSFT_FP32) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)nblocks);
    if (precision == MSFT_BF16X3)
        hipLaunchKernelGGL(fwd_pair_kernel<MSFT_BF16X3>, grid, dim3(PW_THREADS), 0, s, a, block_begin);
    else
        hipLaunchKernelGGL(fwd_pair_kernel<MSFT_BF16>, grid, dim3(PW_THREADS), 0, s, a, block_begin);
    return (int)hipGetLastError();
}

int launch_forward_batch(int precision, const BatchArgs& b, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int32_t items = b.nreq > 0 ? b.item_begin[b.nreq] : 0;
    if (items <= 0) return 0;
    if (precision == MSFT_FP32) return (int)hipErrorInvalidValue;   // three-product kernel
    if (precision == MSFT_BF16X3)
        hipLaunchKernelGGL(fwd_pair_batch_kernel<MSFT_BF16X3>, dim3(items), dim3(PW_THREADS), 0, s, b);
    else
        hipLaunchKernelGGL(fwd_pair_batch_kernel<MSFT_BF16>, dim3(items), dim3(PW_THREADS), 0, s, b);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// First stage of the separable detector (Sec. 3, Blocks 6-7 with q_x a function
// of the column i alone):  H[i][y][z] = sum_x exp(-i q_x(i) x) w(x, y, z).
// Workgroup (block of 128 columns i, S1_Y consecutive y, z block): the wave
// loads its A operand once per x chunk and multiplies the S1_Y tiles of that
// chunk (double-buffered in LDS) into S1_Y accumulators, so the x chunks are
// summed in the MFMA accumulators.  Each lane then holds, for its 8 columns,
// S1_Y consecutive y of one z: one 16-byte slot (FP32) or two 8-byte runs (BF16
// hi, lo) of an H tile row, written with vector stores into the tile group of
// column i (the W tile layout with y in place of x).  Workgroups beyond ny store
// the zero padding rows.
// ---------------------------------------------------------------------------
constexpr int S1_Y = 4;


// Row (h, zl) of an H tile, y = yl .. yl + 3 (yl a multiple of 4).
template <int PREC>
__device__ __forceinline__ void store_h4(uint8_t* tile, int h, int zl, int yl, const float* v)
{
    if (PREC == MSFT_FP32) {
        *(float4*)(tile + tile_slot_offset(h, zl, yl >> 2)) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        __bf16 hi[4], lo[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            hi[u] = (__bf16)v[u];
            lo[u] = (__bf16)(v[u] - (float)hi[u]);
        }
        const int sub = (yl & 7) * 2;
        *(uint2*)(tile + tile_slot_offset(h, zl, yl >> 3) + sub) = pack_bf16x4(hi[0], hi[1], hi[2], hi[3]);
        *(uint2*)(tile + tile_slot_offset(h, zl, 8 + (yl >> 3)) + sub) = pack_bf16x4(lo[0], lo[1], lo[2], lo[3]);
    }
}

// NY y per workgroup: S1_Y for the H tiles (one 16-byte slot per lane); the plain
// output of the adjoint takes any NY, and with NY = 1 two workgroups share a CU.
template <int PREC, bool PLAIN, int NY>
__global__ __launch_bounds__(512, NY == 1 ? 4 : 2) void sep_stage1_kernel(Stage1Args a)
{
    static_assert(PLAIN || NY == S1_Y, "H tiles are written S1_Y consecutive y at a time");
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int y0 = blockIdx.y * NY, zb = blockIdx.z;
    const int64_t wt = (int64_t)blockIdx.x * WAVES + wave;
    const int nyh = max(0, min(NY, a.ny - y0));   // y of this workgroup inside the grid
    const uint4* wbase = (const uint4*)a.wtiles;
    // tile (xc, y0 + u) of this z block, in uint4 units
    auto tile_at = [&](int xc, int u) {
        return wbase + ((size_t)(xc * a.nzb + zb) * a.ny + y0 + u) * (TILE_BYTES / 16);
    };
    f32x16 C[NY];
#pragma unroll
    for (int u = 0; u < NY; ++u) C[u] = f32x16{};
    if (nyh > 0) {
        {
            const uint4* g0 = tile_at(0, 0);
            const uint4 r0 = g0[tid], r1 = g0[tid + 512];
            ((uint4*)lds)[tid] = r0;
            ((uint4*)lds)[tid + 512] = r1;
        }
        __syncthreads();
        int k = 0;   // tiles consumed so far; tile k sits in LDS buffer k & 1
        for (int xc = 0; xc < a.nxc; ++xc) {
            f32x4 Af[16];
            bf16x8 Ahi[8], Alo[8];
            load_a<PREC>(a.txa + (size_t)(wt * a.nxc + xc) * TILE_BYTES, lane, Af, Ahi, Alo);
            __builtin_amdgcn_s_waitcnt(0);
            const int xlen = min(XC, a.x_pad - xc * XC);
#pragma unroll
            for (int u = 0; u < NY; ++u) {
                if (u < nyh) {
                    // next tile: (xc, u + 1) or (xc + 1, 0)
                    const int nxc_ = (u + 1 < nyh) ? xc : xc + 1;
                    const int nu = (u + 1 < nyh) ? u + 1 : 0;
                    const bool has_next = nxc_ < a.nxc;
                    uint4 n0, n1;
                    if (has_next) {
                        const uint4* g = tile_at(nxc_, nu);
                        n0 = g[tid];
                        n1 = g[tid + 512];
                    }
                    const uint8_t* row = lds + (k & 1) * TILE_BYTES + (h * ZB + col) * ROW_BYTES;
                    C[u] = (xlen == XC) ? tile_mfma<PREC, XC>(C[u], row, col, Af, Ahi, Alo)
                                        : tile_mfma_partial<PREC>(C[u], row, col, xlen, Af, Ahi, Alo);
                    if (has_next) {
                        uint4* nb = (uint4*)(lds + ((k + 1) & 1) * TILE_BYTES);
                        nb[tid] = n0;
                        nb[tid + 512] = n1;
                    }
                    __syncthreads();
                    ++k;
                }
            }
        }
    }
    const int yc = y0 / XC, yl = y0 - yc * XC;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int64_t i = slot_pixel(wt, h, m);
        if (i < a.n) {
            const int r = 4 * (m >> 1) + 2 * (m & 1);
            if (PLAIN) {
                // rows of the adjoint's R: 32 lanes write 32 consecutive z
#pragma unroll
                for (int u = 0; u < NY; ++u)
                    if (u < nyh)
                        ((float2*)a.rplain)[((size_t)i * a.ny + y0 + u) * a.nz2 + zb * ZB + col] =
                            make_float2(C[u][r], C[u][r + 1]);
            } else {
                float re[NY], im[NY];
#pragma unroll
                for (int u = 0; u < NY; ++u) {
                    re[u] = C[u][r];
                    im[u] = C[u][r + 1];
                }
                uint8_t* tile = a.htiles + ((size_t)(i * a.nyc + yc) * a.nzb + zb) * TILE_BYTES;
                store_h4<PREC>(tile, 0, col, yl, re);
                store_h4<PREC>(tile, 1, col, yl, im);
            }
        }
    }
}

// Four-wave workgroups of the BF16 separable stages: 64 rows (columns i in stage 1,
// rows j in stage 2), pipeline stages of two W or H tiles.  SR_YC: chunks whose A
// operands a wave keeps resident.
constexpr int SR_YC = 2;
constexpr int SP_WAVES = 4;
constexpr int SP_THREADS = 64 * SP_WAVES;
constexpr int SP_ROWS = SP_WAVES * WAVE_PIX;                  // 64 rows j per workgroup
constexpr int SP_STAGE = 2 * TILE_BYTES;                      // both y chunks
constexpr int SP_COPY = SP_STAGE / 16 / SP_THREADS;           // 8 pieces per thread, 4 per tile
constexpr int SP_TZ_READ = 4;                                 // stage 2: Tz table read every 4 z blocks
static_assert(SP_COPY * SP_THREADS * 16 == SP_STAGE && (TILE_BYTES / 16) % 64 == 0, "whole wave pieces");

// ---------------------------------------------------------------------------
// First stage for the BF16 precisions: workgroups of 4 waves (64 columns i) walk
// SP1_PASSES passes of SP1_Y = 8 consecutive y; per pass and x chunk the wave loads
// its A operand and four pipeline stages follow, each with the W tiles of two y
// (direct global -> LDS loads into a two-slot ring, 48 MFMAs per wave and
// barrier).  Each lane then holds 8 consecutive y of its columns at one z: one whole
// 16-byte slot of an H row per (column, re|im, hi|lo).  Two workgroups share a CU.
// ---------------------------------------------------------------------------
constexpr int SP1_Y = 8;
constexpr int SP1_PASSES = 1;

// The stage (x chunk xc, y and y + 1): two W tiles of z block zb (the first again
// past ny, so every stage issues SP_COPY pieces).
__device__ __forceinline__ void sp1_fill(const Stage1Args& a, int xc, int zb, int y, int wave, uint8_t* slot)
{
    const int lane = threadIdx.x & 63;
    const uint8_t* t0 = a.wtiles + ((size_t)(xc * a.nzb + zb) * a.ny + y) * TILE_BYTES;
    const uint8_t* t1 = y + 1 < a.ny ? t0 + TILE_BYTES : t0;
    constexpr int PER = SP_COPY / 2;
#pragma unroll
    for (int p = 0; p < SP_COPY; ++p) {
        const int q = (p % PER) * SP_THREADS + wave * 64;   // piece of the wave's lane 0 in its tile
        lds_dma16((const u32x4*)(p < PER ? t0 : t1) + q + lane, slot + (p < PER ? 0 : TILE_BYTES) + q * 16);
    }
}

// Eight values as the BF16 hi and lo slots of one 16-byte piece each (value e in
// bits 16 (e % 2) of word e / 2).
__device__ __forceinline__ void split_bf16x8(const float* v, u32x4& hi, u32x4& lo)
{
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const __bf16 h0 = (__bf16)v[2 * w], h1 = (__bf16)v[2 * w + 1];
        const __bf16 l0 = (__bf16)(v[2 * w] - (float)h0), l1 = (__bf16)(v[2 * w + 1] - (float)h1);
        hi[w] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        lo[w] = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
    }
}

// Grid (column blocks of 64, groups of SP1_PASSES passes over nyc * 64, z blocks);
// rows y >= ny of the H tiles are written as zeros.
template <int PREC>
__global__ __launch_bounds__(SP_THREADS, 2) void sep_stage1p_kernel(Stage1Args a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * SP_STAGE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, col = lane & 31;
    const int64_t wt = (int64_t)blockIdx.x * SP_WAVES + wave;   // 16 columns
    const int zb = blockIdx.z;
    const int ybase = SP1_Y * SP1_PASSES * blockIdx.y;
    const int yend = min(a.ny, ybase + SP1_Y * SP1_PASSES);
    // stages (pass, xc, y pair); the one after (pass from y0, xc, pair v)
    auto next_stage = [&](int y0, int xc, int v, int& xn, int& yn) {
        if (y0 + 2 * v + 2 < min(yend, y0 + SP1_Y)) {
            xn = xc;
            yn = y0 + 2 * v + 2;
        } else if (xc + 1 < a.nxc) {
            xn = xc + 1;
            yn = y0;
        } else {
            xn = 0;
            yn = y0 + SP1_Y;
        }
    };
    if (ybase < yend) {
        sp1_fill(a, 0, zb, ybase, wave, lds);
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        __syncthreads();
    }
    int k = 0;   // stages consumed; stage k sits in slot k & 1
#pragma unroll 1
    for (int ps = 0; ps < SP1_PASSES; ++ps) {
        const int y0 = ybase + SP1_Y * ps;
        const int nyp = max(0, min(SP1_Y, a.ny - y0));
        f32x16 C[SP1_Y];
#pragma unroll
        for (int u = 0; u < SP1_Y; ++u) C[u] = f32x16{};
        for (int xc = 0; xc < a.nxc && nyp > 0; ++xc) {
            f32x4 Af[16];
            bf16x8 Ahi[8], Alo[8];
            load_a<PREC>(a.txa + (size_t)(wt * a.nxc + xc) * TILE_BYTES, lane, Af, Ahi, Alo);
            const int xlen = min(XC, a.x_pad - xc * XC);
#pragma unroll
            for (int v = 0; v < SP1_Y / 2; ++v) {
                if (2 * v < nyp) {
                    int xn, yn;
                    next_stage(y0, xc, v, xn, yn);
                    if (yn < yend) sp1_fill(a, xn, zb, yn, wave, lds + ((k + 1) & 1) * SP_STAGE);
                    const uint8_t* cur = lds + (k & 1) * SP_STAGE + (h * ZB + col) * ROW_BYTES;
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        if (xlen == XC)
                            C[2 * v + t] = tile_mfma<PREC, XC>(C[2 * v + t], cur + t * TILE_BYTES, col, Af, Ahi, Alo);
                        else
                            C[2 * v + t] = tile_mfma_partial<PREC>(C[2 * v + t], cur + t * TILE_BYTES, col, xlen, Af,
                                                                   Ahi, Alo);
                    }
                    // the next slot's loads have landed (the compiler does not track them)
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                    __syncthreads();
                    ++k;
                }
            }
        }
        // H slots: row (re|im, z) of tile (i, y0 / 64, zb), hi slot (y0 % 64) / 8, lo slot 8 + that
        const int yc = y0 / XC, ys = (y0 - yc * XC) >> 3;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int64_t i = slot_pixel(wt, h, m);
            if (i < a.n) {
                const int r = 4 * (m >> 1) + 2 * (m & 1);
                float re[SP1_Y], im[SP1_Y];
#pragma unroll
                for (int u = 0; u < SP1_Y; ++u) {
                    // (a y beyond ny summed a repeated tile: its row is zero)
                    re[u] = u < nyp ? C[u][r] : 0.0f;
                    im[u] = u < nyp ? C[u][r + 1] : 0.0f;
                }
                uint8_t* tile = a.htiles + ((size_t)(i * a.nyc + yc) * a.nzb + zb) * TILE_BYTES;
                u32x4 hi, lo;
                split_bf16x8(re, hi, lo);
                *(u32x4*)(tile + tile_slot_offset(0, col, ys)) = hi;
                *(u32x4*)(tile + tile_slot_offset(0, col, 8 + ys)) = lo;
                split_bf16x8(im, hi, lo);
                *(u32x4*)(tile + tile_slot_offset(1, col, ys)) = hi;
                *(u32x4*)(tile + tile_slot_offset(1, col, 8 + ys)) = lo;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Second stage of the separable detector: A(i, j) = sum_z Tz(i, j, z) sum_y
// exp(-i q_y(j) y) H(i, y, z).  The A operand, exp(-i q_y(j) y) for the 16 rows j
// of a wave, does not depend on the column i, so a workgroup (one block of 128
// rows j, CPW consecutive columns i) loads it once per y chunk and multiplies the
// tiles of all its columns with it: per y chunk, for each column, one tile per z
// block (double-buffered in LDS), rotated by Tz into the column's own per-lane
// sums.  The per-workgroup costs (first tile, the wait for the A operand, the
// z-lane butterfly) are paid once per CPW columns.
// ---------------------------------------------------------------------------
template <int PREC, int CPW>
__global__ __launch_bounds__(512) void sep_stage2_kernel(FwdArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t cg = blockIdx.x / a.group_blocks, rb = blockIdx.x - cg * a.group_blocks;
    const int64_t i0 = cg * CPW;
    const int ncol = (int)min((int64_t)CPW, (int64_t)a.out_n - i0);   // >= 1, uniform
    const int64_t wa = rb * WAVES + wave;                                // A operand row
    const int nzb = a.nzb;
    // tile (xc, zb) of column i0 + c, in uint4 units
    auto tile_at = [&](int xc, int c, int zb) {
        return (const uint4*)(a.wtiles + ((size_t)(i0 + c) * a.group_tiles + (size_t)xc * nzb + zb) * TILE_BYTES);
    };
    {
        const uint4* g0 = tile_at(0, 0, 0);
        const uint4 r0 = g0[tid], r1 = g0[tid + 512];
        ((uint4*)lds)[tid] = r0;
        ((uint4*)lds)[tid + 512] = r1;
    }
    __syncthreads();

    float acc[CPW][16];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[c][q] = 0.0f;

    int k = 0;   // tiles consumed; tile k sits in LDS buffer k & 1
    for (int xc = 0; xc < a.nxc; ++xc) {
        const int xlen = min(XC, a.x_pad - xc * XC);
        f32x4 Af[16];
        bf16x8 Ahi[8], Alo[8];
        load_a<PREC>(a.txa + (size_t)(wa * a.nxc + xc) * TILE_BYTES, lane, Af, Ahi, Alo);
        __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (c < ncol) {
                const int64_t wt = ((i0 + c) * a.group_blocks + rb) * WAVES + wave;
                for (int zb = 0; zb < nzb; ++zb) {
                    const f32x4* tzp = (const f32x4*)(a.tz + 2 * ((((wt * nzb + zb) * 2 + h) * ZB + col) * 8));
                    f32x4 tzv[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) tzv[q] = tzp[q];
                    // next tile: (xc, c, zb + 1), (xc, c + 1, 0) or (xc + 1, 0, 0)
                    int nx_ = xc, nc = c, nz_ = zb + 1;
                    if (nz_ == nzb) {
                        nz_ = 0;
                        if (++nc == ncol) {
                            nc = 0;
                            ++nx_;
                        }
                    }
                    const bool has_next = nx_ < a.nxc;
                    uint4 n0, n1;
                    if (has_next) {
                        const uint4* g = tile_at(nx_, nc, nz_);
                        n0 = g[tid];
                        n1 = g[tid + 512];
                    }
                    const uint8_t* row = lds + (k & 1) * TILE_BYTES + (h * ZB + col) * ROW_BYTES;
                    const f32x16 C = tile_product<PREC, false>(row, col, xlen, Af, Ahi, Alo);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int m = 2 * q + u;
                            const int r = 4 * (m >> 1) + 2 * (m & 1);
                            const float tr = tzv[q][2 * u], ti = tzv[q][2 * u + 1];
                            acc[c][2 * m] += tr * C[r] - ti * C[r + 1];
                            acc[c][2 * m + 1] += tr * C[r + 1] + ti * C[r];
                        }
                    }
                    if (has_next) {
                        uint4* nb = (uint4*)(lds + ((k + 1) & 1) * TILE_BYTES);
                        nb[tid] = n0;
                        nb[tid + 512] = n1;
                    }
                    __syncthreads();
                    ++k;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        if (c < ncol) {
            // sum over the 32 z lanes of each half (fixed butterfly order)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                float v = acc[c][q];
                v += __shfl_xor(v, 16, 32);
                v += __shfl_xor(v, 8, 32);
                v += __shfl_xor(v, 4, 32);
                v += __shfl_xor(v, 2, 32);
                v += __shfl_xor(v, 1, 32);
                acc[c][q] = v;
            }
            if (col == 0) {
                const int64_t i = i0 + c;
                const int64_t wt = (i * a.group_blocks + rb) * WAVES + wave;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int64_t j = slot_pixel(wt, h, m) - i * a.out_npad;
                    if (j < a.out_n) {
                        const int64_t out = j * a.out_n + i;
                        const float re = acc[c][2 * m], im = acc[c][2 * m + 1];
                        a.intensity[out] = re * re + im * im;
                        if (a.amplitude) ((float2*)a.amplitude)[out] = make_float2(re, im);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Second stage for the BF16 precisions with at most two y chunks: workgroups of 4
// waves (64 rows j, CPW columns i) with both chunks' A operands resident; each
// pipeline stage is one (column, z block) with the H tiles of both chunks, filled
// by direct global -> LDS loads into a two-slot ring, so one barrier covers 48
// MFMAs per wave; two workgroups share a CU, and the row blocks of a column group
// run on one XCD (workgroup b runs on XCD b % 8) so that each H tile comes from HBM
// about once.  Per (column, z block) the y chunks accumulate in one MFMA
// accumulator, then Tz rotates the result into the column's per-lane sums.
// ---------------------------------------------------------------------------

// The stage of column i, z block zb: tiles (y chunk 0, 1) of the column's group into
// an LDS slot (with one chunk, its tile twice, so every stage issues SP_COPY pieces).
__device__ __forceinline__ void sp_fill(const FwdArgs& a, int64_t i, int zb, int wave, uint8_t* slot)
{
    const int lane = threadIdx.x & 63;
    const uint8_t* t0 = a.wtiles + ((size_t)i * a.group_tiles + zb) * TILE_BYTES;
    const uint8_t* t1 = a.nxc > 1 ? t0 + (size_t)a.nzb * TILE_BYTES : t0;
    constexpr int PER = SP_COPY / 2;
#pragma unroll
    for (int p = 0; p < SP_COPY; ++p) {
        const int q = (p % PER) * SP_THREADS + wave * 64;   // piece of the wave's lane 0 in its tile
        lds_dma16((const u32x4*)(p < PER ? t0 : t1) + q + lane, slot + (p < PER ? 0 : TILE_BYTES) + q * 16);
    }
}

template <int PREC, int CPW>
__global__ __launch_bounds__(SP_THREADS, 2) void sep_stage2p_kernel(FwdArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * SP_STAGE];
    __shared__ f32x4 rzs[SP_THREADS * 4];   // per thread: exp(-i q_z 32 dz) of its 8 rows
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, col = lane & 31;
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int nrb = a.out_npad / SP_ROWS;
    const int64_t cg = L / nrb;
    const int rb = (int)(L - cg * nrb);
    const int64_t i0 = cg * CPW;
    const int ncol = (int)min((int64_t)CPW, (int64_t)a.out_n - i0);   // >= 1, uniform
    const int64_t jt = (int64_t)rb * SP_WAVES + wave;                  // 16-row tile in the column
    const int nzb = a.nzb, nyc = a.nxc;
    const int ylast = a.x_pad - (nyc - 1) * XC;   // y values in the last chunk
    f32x4 Af[SR_YC][16];
    bf16x8 Ahi[SR_YC][8], Alo[SR_YC][8];
#pragma unroll
    for (int yc = 0; yc < SR_YC; ++yc)
        if (yc < nyc) load_a<PREC>(a.txa + (size_t)(jt * nyc + yc) * TILE_BYTES, lane, Af[yc], Ahi[yc], Alo[yc]);
    sp_fill(a, i0, 0, wave, lds);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __syncthreads();
    int s = 0;   // stages consumed; stage s sits in slot s & 1
    for (int c = 0; c < ncol; ++c) {
        const int64_t i = i0 + c;
        const int64_t wt = i * (a.out_npad / WAVE_PIX) + jt;
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
        // Tz of the lane's 8 rows at its z: read from the plan's table every SP_TZ_READ z
        // blocks and rotated by rz = exp(-i q_z 32 dz) = Tz(block 1) conj(Tz(block 0))
        // in between (a quarter of the table's traffic; at most SP_TZ_READ - 1 FP32
        // rotations from a table value)
        const float* tzc = a.tz + 2 * (((wt * nzb * 2 + h) * ZB + col) * 8);
        const int64_t tz_block = 2 * 2 * ZB * 8;   // floats per z block
        // (the thread's rz lives in its own LDS slot: registers are full)
        f32x4* rzt = rzs + tid * 4;
        if (nzb > 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 t0 = ((const f32x4*)tzc)[q], t1 = ((const f32x4*)(tzc + tz_block))[q];
                f32x4 r;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    r[2 * u] = t1[2 * u] * t0[2 * u] + t1[2 * u + 1] * t0[2 * u + 1];
                    r[2 * u + 1] = t1[2 * u + 1] * t0[2 * u] - t1[2 * u] * t0[2 * u + 1];
                }
                rzt[q] = r;
            }
        }
        f32x4 tzv[4];
        for (int zb = 0; zb < nzb; ++zb) {
            if (zb % SP_TZ_READ == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) tzv[q] = ((const f32x4*)(tzc + zb * tz_block))[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 r = rzt[q];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const float tr = tzv[q][2 * u], ti = tzv[q][2 * u + 1];
                        tzv[q][2 * u] = tr * r[2 * u] - ti * r[2 * u + 1];
                        tzv[q][2 * u + 1] = tr * r[2 * u + 1] + ti * r[2 * u];
                    }
                }
            }
            if (zb + 1 < nzb) sp_fill(a, i, zb + 1, wave, lds + ((s + 1) & 1) * SP_STAGE);
            else if (c + 1 < ncol) sp_fill(a, i + 1, 0, wave, lds + ((s + 1) & 1) * SP_STAGE);
            const uint8_t* cur = lds + (s & 1) * SP_STAGE + (h * ZB + col) * ROW_BYTES;
            f32x16 C = {};
#pragma unroll
            for (int yc = 0; yc < SR_YC; ++yc) {
                if (yc < nyc) {
                    if (yc + 1 < nyc || ylast == XC)
                        C = tile_mfma<PREC, XC>(C, cur + yc * TILE_BYTES, col, Af[yc], Ahi[yc], Alo[yc]);
                    else
                        C = tile_mfma_partial<PREC>(C, cur + yc * TILE_BYTES, col, ylast, Af[yc], Ahi[yc], Alo[yc]);
                }
            }
            // the next slot's loads have landed (the compiler does not track them)
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            __syncthreads();
            ++s;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int m = 2 * q + u;
                    const int r = 4 * (m >> 1) + 2 * (m & 1);
                    const float tr = tzv[q][2 * u], ti = tzv[q][2 * u + 1];
                    acc[2 * m] += tr * C[r] - ti * C[r + 1];
                    acc[2 * m + 1] += tr * C[r + 1] + ti * C[r];
                }
            }
        }
        // sum over the 32 z lanes of each half (fixed butterfly order)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float v = acc[q];
            v += __shfl_xor(v, 16, 32);
            v += __shfl_xor(v, 8, 32);
            v += __shfl_xor(v, 4, 32);
            v += __shfl_xor(v, 2, 32);
            v += __shfl_xor(v, 1, 32);
            acc[q] = v;
        }
        if (col == 0) {
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int64_t j = slot_pixel(wt, h, m) - i * a.out_npad;
                if (j < a.out_n) {
                    const int64_t out = j * a.out_n + i;
                    const float re = acc[2 * m], im = acc[2 * m + 1];
                    a.intensity[out] = re * re + im * im;
                    if (a.amplitude) ((float2*)a.amplitude)[out] = make_float2(re, im);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the separable detector.  With h = g conj(A) the strength gradient
// needs R(x, y, z) = sum_{i,j} h(i, j) exp(-i (q_x(i) x + q_y(j) y + q_z(i, j) z)),
// the transposed two-stage sum:
//   K(i, y, z) = sum_j exp(-i q_y(j) y) [h(i, j) exp(-i q_z(i, j) z)]   (this kernel)
//   R(x, y, z) = sum_i exp(-i q_x(i) x) K(i, y, z)          (sep_stage1_kernel, PLAIN)
// Workgroup (128 rows y, S1_Y consecutive columns i, z block).  Per chunk of 64
// detector rows j the wave loads its A operand (one table shared by every column)
// and multiplies the chunk's S1_Y B tiles h Tz into S1_Y accumulators; the B
// tiles (W tile layout, j in place of x) sit in a double-buffered LDS ring, and
// the workgroup forms the next chunk's tiles right behind the MFMA chain, from
// Tz values loaded one chunk ahead, so one barrier per chunk remains.  K is stored in tiles (i chunk, z block, y) with i in place of x
// (columns beyond N store zeros), ready to be the B operand of the second sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void sepadj_rows_kernel(SepAdjArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * S1_Y * TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t wt = (int64_t)blockIdx.x * WAVES + wave;   // 16 rows y
    const int i0 = blockIdx.y * S1_Y, zb = blockIdx.z;
    const int nih = max(0, min(S1_Y, a.n - i0));               // columns inside the detector
    // this thread's 4 consecutive entries of one Tz block (16 pixels x 32 z of a z block)
    const int w4 = tid >> 7, e0 = (tid & 127) * 4;
    const int hh = e0 >> 8, z = (e0 >> 3) & 31, m0 = e0 & 7;
    // the thread's Tz entries of chunk jc, column i0 + u
    auto load_tz = [&](int jc, f32x4 (&t)[S1_Y][2]) {
#pragma unroll
        for (int u = 0; u < S1_Y; ++u) {
            if (u < nih) {
                const int64_t wt2 = (int64_t)(i0 + u) * (a.npad / WAVE_PIX) + jc * (XC / WAVE_PIX) + w4;
                const f32x4* tzp = (const f32x4*)(a.tz + 2 * ((wt2 * a.nzb + zb) * (2 * ZB * 8) + e0));
                t[u][0] = tzp[0];
                t[u][1] = tzp[1];
            }
        }
    };
    // B tiles h Tz of chunk jc (rows j in place of x) into the S1_Y tiles at buf
    auto form_tiles = [&](int jc, uint8_t* buf, const f32x4 (&t)[S1_Y][2]) {
#pragma unroll
        for (int u = 0; u < S1_Y; ++u) {
            if (u < nih) {
                const int64_t i = i0 + u;
                const float tz[8] = {t[u][0][0], t[u][0][1], t[u][0][2], t[u][0][3],
                                     t[u][1][0], t[u][1][1], t[u][1][2], t[u][1][3]};
                uint8_t* tile = buf + u * TILE_BYTES;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = m0 + v;
                    const int jl = w4 * WAVE_PIX + 4 * (m >> 1) + 2 * hh + (m & 1);
                    const int64_t j = (int64_t)jc * XC + jl;
                    float2 hv = make_float2(0.0f, 0.0f);
                    if (j < a.n) hv = ((const float2*)a.h)[j * a.n + i];
                    const float tr = tz[2 * v], ti = tz[2 * v + 1];
                    *(float*)(tile + tile_slot_offset(0, z, jl >> 2) + (jl & 3) * 4) = hv.x * tr - hv.y * ti;
                    *(float*)(tile + tile_slot_offset(1, z, jl >> 2) + (jl & 3) * 4) = hv.x * ti + hv.y * tr;
                }
            }
        }
    };
    f32x16 C[S1_Y];
#pragma unroll
    for (int u = 0; u < S1_Y; ++u) C[u] = f32x16{};
    if (nih > 0) {
        f32x4 tzn[S1_Y][2];
        load_tz(0, tzn);
        form_tiles(0, lds, tzn);
        if (a.njc > 1) load_tz(1, tzn);
        __syncthreads();
        for (int jc = 0; jc < a.njc; ++jc) {
            f32x4 Af[16];
            bf16x8 Ahi[8], Alo[8];
            load_a<MSFT_FP32>(a.tyT + (size_t)(wt * a.njc + jc) * TILE_BYTES, lane, Af, Ahi, Alo);
            const uint8_t* cur = lds + (jc & 1) * S1_Y * TILE_BYTES;
#pragma unroll
            for (int u = 0; u < S1_Y; ++u)
                if (u < nih)
                    C[u] = tile_mfma<MSFT_FP32, XC>(C[u], cur + u * TILE_BYTES + (h * ZB + col) * ROW_BYTES,
                                                    col, Af, Ahi, Alo);
            // the next chunk's tiles go to the other buffer, which every wave finished
            // reading before the last barrier; its Tz values arrived during this chunk
            if (jc + 1 < a.njc) {
                form_tiles(jc + 1, lds + ((jc + 1) & 1) * S1_Y * TILE_BYTES, tzn);
                if (jc + 2 < a.njc) load_tz(jc + 2, tzn);
            }
            __syncthreads();
        }
    }
    const int ic = i0 / XC, il = i0 - ic * XC;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int64_t y = slot_pixel(wt, h, m);
        if (y < a.ny) {
            const int r = 4 * (m >> 1) + 2 * (m & 1);
            float re[S1_Y], im[S1_Y];
#pragma unroll
            for (int u = 0; u < S1_Y; ++u) {
                re[u] = C[u][r];
                im[u] = C[u][r + 1];
            }
            uint8_t* tile = a.ktiles + ((size_t)(ic * a.nzb + zb) * a.ny + y) * TILE_BYTES;
            store_h4<MSFT_FP32>(tile, 0, col, il, re);
            store_h4<MSFT_FP32>(tile, 1, col, il, im);
        }
    }
}

// Both contractions of the separable adjoint; R goes to ra.rplain.
int launch_sep_adjoint(const SepAdjArgs& ka, const Stage1Args& ra, int64_t nblk_rows, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int nic = (int)ceil_div(ka.n, XC);
    const dim3 g1((unsigned)ceil_div(ka.ny, BLOCK_PIX), (unsigned)(nic * XC / S1_Y), (unsigned)ka.nzb);
    hipLaunchKernelGGL(sepadj_rows_kernel, g1, dim3(512), 0, s, ka);
    // as many y per workgroup as keep two workgroups per CU in the grid
    const int ny_wg = nblk_rows * ceil_div(ra.ny, 4) * ra.nzb >= 2 * CHIP_CUS   ? 4
                      : nblk_rows * ceil_div(ra.ny, 2) * ra.nzb >= 2 * CHIP_CUS ? 2
                                                                                  : 1;
    const dim3 g2((unsigned)nblk_rows, (unsigned)ceil_div(ra.ny, ny_wg), (unsigned)ra.nzb);
    if (ny_wg == 4)
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_FP32, true, 4>), g2, dim3(512), 0, s, ra);
    else if (ny_wg == 2)
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_FP32, true, 2>), g2, dim3(512), 0, s, ra);
    else
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_FP32, true, 1>), g2, dim3(512), 0, s, ra);
    return (int)hipGetLastError();
}

// A tables of the adjoint (FP32): rows y against rows j, rows x against columns i;
// xq3 / yq3 hold the voxel coordinates in slot 0 of [n][3] arrays.
int launch_sep_adj_tables(const SepDims& sd, int nx, int ny, const double* xq3, const double* qx,
                          const double* yq3, const double* qy, uint8_t* txT, uint8_t* tyT,
                          void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    launch_txa(MSFT_FP32, tyT, ceil_div(ny, BLOCK_PIX) * WAVES, ny, sd.n, sd.njc, yq3, qy, s);
    launch_txa(MSFT_FP32, txT, ceil_div(nx, BLOCK_PIX) * WAVES, nx, sd.n, sd.nic, xq3, qx, s);
    return (int)hipGetLastError();
}

template <int CPW>
static void launch_stage2_cpw(int precision, const FwdArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)(ceil_div(a.out_n, CPW) * a.group_blocks));
    if (precision == MSFT_FP32)
        hipLaunchKernelGGL((sep_stage2_kernel<MSFT_FP32, CPW>), grid, dim3(512), 0, s, a);
    else if (precision == MSFT_BF16X3)
        hipLaunchKernelGGL((sep_stage2_kernel<MSFT_BF16X3, CPW>), grid, dim3(512), 0, s, a);
    else
        hipLaunchKernelGGL((sep_stage2_kernel<MSFT_BF16, CPW>), grid, dim3(512), 0, s, a);
}

// General second stage: two columns per workgroup when that still leaves
// STAGE2_MIN_WG workgroups (two per CU), else one.  Four measured no faster in FP32
// and slower in BF16.
constexpr int64_t STAGE2_MIN_WG = 2 * CHIP_CUS;


template <int CPW>
static void launch_stage2p_cpw(int precision, const FwdArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)(ceil_div(a.out_n, CPW) * (a.out_npad / SP_ROWS)));
    if (precision == MSFT_BF16X3)
        hipLaunchKernelGGL((sep_stage2p_kernel<MSFT_BF16X3, CPW>), grid, dim3(SP_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((sep_stage2p_kernel<MSFT_BF16, CPW>), grid, dim3(SP_THREADS), 0, s, a);
}

// Second stage: for BF16 with at most SR_YC y chunks the four-wave kernel with
// the A operand resident, as many columns per workgroup as still leave two
// workgroups per CU; otherwise the general kernel, two columns per workgroup when
// that still leaves STAGE2_MIN_WG workgroups, else one.
int launch_sep_stage2(int precision, const FwdArgs& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.out_n <= 0 || a.group_blocks <= 0) return (int)hipErrorInvalidValue;
    const int64_t gb = a.group_blocks;
    if (precision != MSFT_FP32 && a.nxc <= SR_YC) {
        // BF16: four-wave workgroups, as many columns each as leave two per CU
        const int64_t nrb = a.out_npad / SP_ROWS;
        if (ceil_div(a.out_n, 8) * nrb >= 2 * CHIP_CUS) launch_stage2p_cpw<8>(precision, a, s);
        else if (ceil_div(a.out_n, 4) * nrb >= 2 * CHIP_CUS) launch_stage2p_cpw<4>(precision, a, s);
        else if (ceil_div(a.out_n, 2) * nrb >= 2 * CHIP_CUS) launch_stage2p_cpw<2>(precision, a, s);
        else launch_stage2p_cpw<1>(precision, a, s);
        return (int)hipGetLastError();
    }
    if (ceil_div(a.out_n, 2) * gb >= STAGE2_MIN_WG) launch_stage2_cpw<2>(precision, a, s);
    else launch_stage2_cpw<1>(precision, a, s);
    return (int)hipGetLastError();
}

int launch_sep_stage1(int precision, const Stage1Args& a, int64_t nblk, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (precision != MSFT_FP32) {
        const dim3 g((unsigned)ceil_div(a.n, SP_ROWS), (unsigned)(a.nyc * XC / (SP1_Y * SP1_PASSES)), (unsigned)a.nzb);
        if (precision == MSFT_BF16X3)
            hipLaunchKernelGGL(sep_stage1p_kernel<MSFT_BF16X3>, g, dim3(SP_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL(sep_stage1p_kernel<MSFT_BF16>, g, dim3(SP_THREADS), 0, s, a);
        return (int)hipGetLastError();
    }
    const dim3 grid((unsigned)nblk, (unsigned)(a.nyc * XC / S1_Y), (unsigned)a.nzb);
    if (precision == MSFT_FP32)
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_FP32, false, S1_Y>), grid, dim3(512), 0, s, a);
    else if (precision == MSFT_BF16X3)
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_BF16X3, false, S1_Y>), grid, dim3(512), 0, s, a);
    else
        hipLaunchKernelGGL((sep_stage1_kernel<MSFT_BF16, false, S1_Y>), grid, dim3(512), 0, s, a);
    return (int)hipGetLastError();
}

}  // namespace msft
