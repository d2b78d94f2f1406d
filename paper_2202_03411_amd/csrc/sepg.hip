// gfx950 Gauss (3M) form of the uniform transverse-q detector's two contractions
// in FP32 (Sec. 3's separable sum: q_x depends on the detector column i alone, q_y
// on the row j alone):
//
//   stage 1:  H(i, y, z) = sum_x exp(-i q_x(i) x) w(x, y, z)
//   stage 2:  A(i, j)    = sum_z exp(-i q_z(i, j) z) sum_y exp(-i q_y(j) y) H(i, y, z)
//             I(i, j)    = |A(i, j)|^2
//
// Every complex sum runs as three real MFMA products P1 = Tr.Br, P2 = Ti.Bi,
// P3 = (Tr + Ti).(Br + Bi), then Re = P1 - P2 and Im = P3 - P1 - P2, with the three
// planes of each operand made ahead: the A operands at plan time (phases in FP64),
// the W tiles by the column scan, H by stage 1.
//
// Stage 1 (v_mfma_f32_32x32x2_f32): rows are a wave's 32 columns i, columns the 32 z
// of a W tile, K two x values (x parity = lane half), as in the flat detector's
// Gauss kernel; a workgroup of 4 waves takes 128 columns, two consecutive y and one
// z block, and the sums over the x chunks stay in the MFMA accumulators.
//
// Stage 2 (v_mfma_f32_16x16x4_f32): rows are a wave's 16 rows j, columns 16 z, K
// four y values.  The wave keeps its A operand for every y (at most 128: 96
// registers) resident, so a column's H tiles stream through LDS once per z block
// with the sums over y in the MFMA accumulators; the z phase and the sum over the z
// lanes follow.  A workgroup of 4 waves takes 64 rows j and a group of columns;
// the workgroups of one column group run on one XCD, so its H tiles come from HBM
// about once.
//
// H tile (i, y chunk yc of 32, z block): [plane 3][kk 4][g 2][z 32][e 4] floats
// holding y = 32 yc + 8 kk + 4 g + e, planes Hr, Hi, Hr + Hi.  Sums run in an order
// fixed by the plan alone.
#include <hip/hip_runtime.h>

#include "lds_dma.h"
#include "msft_internal.h"

namespace msft {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int SG_WAVES = 4;
constexpr int SG_THREADS = 64 * SG_WAVES;
constexpr int SG_PLANE_BYTES = G3_TILE_BYTES / 3;            // 4 KiB
constexpr int SG_TILE_F4 = G3_TILE_BYTES / 16;               // 768 pieces of 16 bytes
constexpr int SG1_COPY = SG_TILE_F4 / SG_THREADS;            // 3 per thread
constexpr int SG2_STAGE = 2 * G3_TILE_BYTES;                 // two y chunks of one (column, z block)
constexpr int SG2_COPY = 2 * SG_TILE_F4 / SG_THREADS;        // 6 per thread
constexpr int SG2_ROWS = 16;                                 // rows j per stage-2 wave
constexpr int SG2_WG_ROWS = SG2_ROWS * SG_WAVES;             // 64
static_assert(SG1_COPY * SG_THREADS == SG_TILE_F4 && SG_TILE_F4 % 64 == 0,
              "a tile is copied in whole wave pieces");
static_assert(SG2_A_BYTES == 6 * 64 * 16, "stage 2 A: six 16-byte pieces per lane and y chunk");
static_assert(SG2_ROWS == WAVE_PIX, "stage 2 rows match the 16-row Tz tiles");

// ---------------------------------------------------------------------------
// Plan-time A tables.  T = exp(i phi), phi = -q . r in FP64; planes Re T, Im T,
// Re T + Im T (the sum formed in FP64).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float plane_value(double phi, int plane)
{
    double sn, cs;
    sincos(phi, &sn, &cs);
    return (float)(plane == 0 ? cs : plane == 1 ? sn : cs + sn);
}

// Stage 1: [wt][xc][plane 3][g 4][lane 64][e 4]; lane (h, c) holds column
// i = 32 wt + c at x = 32 xc + 8 g + 2 e + h for MFMA step 4 g + e.
__global__ void sg_twiddle_a1(float* t, int64_t total, int n, int nx, int nxc3, const double* qx,
                              const double* xs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int e = (int)(idx & 3), lane = (int)((idx >> 2) & 63);
    const int64_t rest = idx >> 8;
    const int q = (int)(rest % 12);
    const int64_t tile = rest / 12;
    const int plane = q >> 2, g = q & 3;
    const int xc = (int)(tile % nxc3);
    const int64_t wt = tile / nxc3;
    const int64_t i = wt * G3_WAVE_PIX + (lane & 31);
    const int x = xc * G3_XC + 8 * g + 2 * e + (lane >> 5);
    t[idx] = (i < n && x < nx) ? plane_value(-(qx[i] * xs[x]), plane) : 0.0f;
}

// Stage 2: [jt][yc][plane 3][g 2][lane 64][e 4]; lane (kk, m) holds row
// j = 16 jt + m at y = 32 yc + 8 kk + 4 g + e for MFMA step 4 g + e of chunk yc.
__global__ void sg_twiddle_a2(float* t, int64_t total, int n, int ny, int nyc2, const double* qy,
                              const double* ys)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int e = (int)(idx & 3), lane = (int)((idx >> 2) & 63);
    const int64_t rest = idx >> 8;
    const int q = (int)(rest % 6);
    const int64_t tile = rest / 6;
    const int plane = q >> 1, g = q & 1;
    const int yc = (int)(tile % nyc2);
    const int64_t jt = tile / nyc2;
    const int64_t j = jt * SG2_ROWS + (lane & 15);
    const int y = yc * 32 + 8 * (lane >> 4) + 4 * g + e;
    t[idx] = (j < n && y < ny) ? plane_value(-(qy[j] * ys[y]), plane) : 0.0f;
}

// ---------------------------------------------------------------------------
// Stage 1.
// ---------------------------------------------------------------------------

// W tile (xc, zb, y) into an LDS slot: three 16-byte pieces per thread (wave:
// the wave index as a wave-uniform value, so the addresses stay scalar).
__device__ __forceinline__ void sg1_fill(const SepG3Args& a, int xc, int zb, int y, int wave, uint8_t* slot)
{
    const int lane = threadIdx.x & 63;
    const u32x4* src = (const u32x4*)(a.wtiles + ((size_t)(xc * a.nzb + zb) * a.ny + y) * G3_TILE_BYTES);
#pragma unroll
    for (int c = 0; c < SG1_COPY; ++c) {
        const int q = c * SG_THREADS + wave * 64;   // piece of the wave's lane 0
        lds_dma16(src + q + lane, slot + q * 16);
    }
}

// P += the three products of one W tile (all 32 x; the tables are zero beyond nx).
// The next step group's B fragments are read from LDS before the current group's
// MFMAs are issued.
__device__ __forceinline__ void sg1_tile(const uint8_t* row, int col, const f32x4* Af, f32x16 (&P)[3])
{
    const int sw = (col >> 1) & 3;
    f32x4 b[2][3];
#pragma unroll
    for (int p = 0; p < 3; ++p) b[0][p] = *(const f32x4*)(row + p * SG_PLANE_BYTES + ((0 ^ sw) << 4));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (g + 1 < 4) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
                b[(g + 1) & 1][p] = *(const f32x4*)(row + p * SG_PLANE_BYTES + (((g + 1) ^ sw) << 4));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            P[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][e], b[g & 1][0][e], P[0], 0, 0, 0);
            P[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[4 + g][e], b[g & 1][1][e], P[1], 0, 0, 0);
            P[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[8 + g][e], b[g & 1][2][e], P[2], 0, 0, 0);
        }
    }
}

// Grid (column blocks of 128, groups of SG1_PAIRS y pairs over nyc2 * 32, z
// blocks): the workgroup walks its y pairs one after the other with the tile ring
// running on across them.  Rows y >= ny of the H tiles are written as zeros;
// columns i >= N are not stored.
constexpr int SG1_PAIRS = 2;

__global__ __launch_bounds__(SG_THREADS, 2) void sepg_stage1_kernel(SepG3Args a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * G3_TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, col = lane & 31;
    const int64_t wt = (int64_t)blockIdx.x * SG_WAVES + wave;
    const int zb = blockIdx.z;
    const int ybase = 2 * SG1_PAIRS * blockIdx.y;
    // y rows of the pairs inside the grid: tiles (xc, y) in the order (pair, xc, y)
    const int nyw = max(0, min(2 * SG1_PAIRS, a.ny - ybase));
    // the stage after (pair p, xc, u): its W tile
    auto next_tile = [&](int p, int xc, int u, int& xn, int& yn) {
        const int y = ybase + 2 * p + u;
        const int nyh = min(2, a.ny - (ybase + 2 * p));
        if (u + 1 < nyh) {
            xn = xc;
            yn = y + 1;
        } else if (xc + 1 < a.nxc3) {
            xn = xc + 1;
            yn = ybase + 2 * p;
        } else {
            xn = 0;
            yn = ybase + 2 * p + 2;
        }
    };
    if (nyw > 0) {
        sg1_fill(a, 0, zb, ybase, wave, lds);
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        __syncthreads();
    }
    int k = 0;   // tiles consumed so far; tile k sits in slot k & 1
#pragma unroll 1
    for (int p = 0; p < SG1_PAIRS; ++p) {
        const int y0 = ybase + 2 * p;
        const int nyh = max(0, min(2, a.ny - y0));   // y of this pair inside the grid
        f32x16 P[2][3];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) P[u][q] = f32x16{};
        for (int xc = 0; xc < a.nxc3 && nyh > 0; ++xc) {
            f32x4 Af[12];
            const f32x4* ta = (const f32x4*)(a.txa1 + (size_t)(wt * a.nxc3 + xc) * G3_TILE_BYTES);
#pragma unroll
            for (int q = 0; q < 12; ++q) Af[q] = ta[q * 64 + lane];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u < nyh) {
                    int xn, yn;
                    next_tile(p, xc, u, xn, yn);
                    if (yn < min(a.ny, ybase + 2 * SG1_PAIRS))
                        sg1_fill(a, xn, zb, yn, wave, lds + ((k + 1) & 1) * G3_TILE_BYTES);
                    sg1_tile(lds + (k & 1) * G3_TILE_BYTES + (h * ZB + col) * G3_ROW_BYTES, col, Af, P[u]);
                    // the next slot's loads have landed (the compiler does not track them)
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                    __syncthreads();
                    ++k;
                }
            }
        }
        // H = (P1 - P2) + i (P3 - P1 - P2) and Hr + Hi at y0, y0 + 1: 8 bytes per plane
        const int yc = y0 >> 5, yl = y0 & 31;
        const int off = (((yl >> 3) * 2 + ((yl >> 2) & 1)) * 32 + col) * 16 + 4 * (yl & 3);
        uint8_t* hcol = a.htiles + ((size_t)yc * a.nzb + zb) * G3_TILE_BYTES + off;
        const size_t col_stride = (size_t)a.nyc2 * a.nzb * G3_TILE_BYTES;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = wt * G3_WAVE_PIX + 8 * (r >> 2) + 4 * h + (r & 3);
            if (i < a.n) {
                float hr[2], hi[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    hr[u] = P[u][0][r] - P[u][1][r];
                    hi[u] = (P[u][2][r] - P[u][0][r]) - P[u][1][r];
                }
                uint8_t* tile = hcol + i * col_stride;
                *(float2*)tile = make_float2(hr[0], hr[1]);
                *(float2*)(tile + SG_PLANE_BYTES) = make_float2(hi[0], hi[1]);
                *(float2*)(tile + 2 * SG_PLANE_BYTES) = make_float2(hr[0] + hi[0], hr[1] + hi[1]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 2.
// ---------------------------------------------------------------------------

// The stage of column i, z block zb and y chunks 2 half, 2 half + 1 (those below
// nyc2) into an LDS slot of two tiles: six pieces per thread (wave: the wave index
// as a wave-uniform value, so the addresses stay scalar).
__device__ __forceinline__ void sg2_fill(const SepG3Args& a, int64_t i, int zb, int half, int wave,
                                         uint8_t* slot)
{
    static_assert(SG2_COPY == 2 * SG1_COPY, "pieces 0-2 of a thread fill the first tile, 3-5 the second");
    const int lane = threadIdx.x & 63;
    const size_t chunk = (size_t)a.nzb * G3_TILE_BYTES;
    const u32x4* t0 = (const u32x4*)(a.htiles + ((size_t)i * a.nyc2 + 2 * half) * chunk + (size_t)zb * G3_TILE_BYTES);
    const bool two = 2 * half + 1 < a.nyc2;
#pragma unroll
    for (int p = 0; p < SG2_COPY; ++p) {
        const int q = (p % SG1_COPY) * SG_THREADS + wave * 64;   // piece of the wave's lane 0 in its tile
        if (p < SG1_COPY)
            lds_dma16(t0 + q + lane, slot + q * 16);
        else if (two)
            lds_dma16((const u32x4*)((const uint8_t*)t0 + chunk) + q + lane, slot + G3_TILE_BYTES + q * 16);
    }
}

// P[plane][n tile] += the products of NT y chunks (2 HALF, 2 HALF + 1) of one
// stage.  Groups (chunk t, step group g, plane p) of eight MFMAs; the B fragments of
// the next group are read from LDS before the current group's MFMAs are issued.
// Every chain P[p][nt] runs over (t, g, e) in the same order whatever NT.
template <int HALF, int NT>
__device__ __forceinline__ void sg2_chunks(const uint8_t* slot, int kk, int n16,
                                           const f32x4 (&Af)[SG2_MAXYC][6], f32x4 (&P)[3][2])
{
    constexpr int NG = NT * 6;
    // B fragment of lane (kk, n16): y = 8 kk + 4 g + e, z = 16 nt + n16 of chunk t, plane p
    const uint8_t* base = slot + kk * 1024 + n16 * 16;
    auto group = [&](int k) { return base + (k / 6) * G3_TILE_BYTES + (k % 3) * SG_PLANE_BYTES + ((k / 3) % 2) * 512; };
    f32x4 b[2][2];
    b[0][0] = *(const f32x4*)group(0);
    b[0][1] = *(const f32x4*)(group(0) + 256);
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        if (k + 1 < NG) {
            b[(k + 1) & 1][0] = *(const f32x4*)group(k + 1);
            b[(k + 1) & 1][1] = *(const f32x4*)(group(k + 1) + 256);
        }
        const int t = k / 6, g = (k / 3) % 2, p = k % 3;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                P[p][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[2 * HALF + t][2 * p + g][e], b[k & 1][nt][e],
                                                                P[p][nt], 0, 0, 0);
    }
}

template <int HALF>
__device__ __forceinline__ void sg2_stage(const uint8_t* slot, int nyc, int kk, int n16,
                                          const f32x4 (&Af)[SG2_MAXYC][6], f32x4 (&P)[3][2])
{
    if (2 * HALF + 1 < nyc) sg2_chunks<HALF, 2>(slot, kk, n16, Af, P);
    else sg2_chunks<HALF, 1>(slot, kk, n16, Af, P);
}

// Grid: column groups of CPW x row blocks of 64 j.  Lane (kk, n16) holds output
// rows j = 16 jt + 4 kk + r (r = 0..3) at z = 16 nt + n16 of each z block.
template <int CPW>
__global__ __launch_bounds__(SG_THREADS, 2) void sepg_stage2_kernel(SepG3Args a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * SG2_STAGE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kk = lane >> 4, n16 = lane & 15;
    // workgroup b runs on XCD b % 8: consecutive L share an XCD
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int nrb = a.npad / SG2_WG_ROWS;
    const int64_t cg = L / nrb;
    const int rb = (int)(L - cg * nrb);
    const int64_t i0 = cg * CPW;
    const int ncol = (int)min((int64_t)CPW, (int64_t)a.n - i0);   // >= 1, uniform
    const int64_t jt = (int64_t)rb * SG_WAVES + wave;              // row tile of 16 j
    const int nyc = a.nyc2, nyh = (nyc + 1) >> 1, nzb = a.nzb;

    f32x4 Af[SG2_MAXYC][6];
    const f32x4* ta = (const f32x4*)(a.txa2 + (size_t)jt * nyc * SG2_A_BYTES);
#pragma unroll
    for (int yc = 0; yc < SG2_MAXYC; ++yc)
#pragma unroll
        for (int q = 0; q < 6; ++q) Af[yc][q] = yc < nyc ? ta[(yc * 6 + q) * 64 + lane] : f32x4{};

    sg2_fill(a, i0, 0, 0, wave, lds);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __syncthreads();

    int s = 0;   // stages consumed so far; stage s sits in slot s & 1
    for (int c = 0; c < ncol; ++c) {
        const int64_t i = i0 + c;
        const int64_t w16 = i * (a.npad / SG2_ROWS) + jt;
        float acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        for (int zb = 0; zb < nzb; ++zb) {
            // Tz of the lane's outputs: entries (w16, zb, hp, z, m = 2 kk + (r & 1)),
            // row r = 2 hp + (r & 1) of the 16-row tile
            f32x4 tz[2][2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int hp = 0; hp < 2; ++hp)
                    tz[nt][hp] = *(const f32x4*)(a.tz + 2 * ((((w16 * nzb + zb) * 2 + hp) * ZB + 16 * nt + n16) * 8 +
                                                             2 * kk));
            f32x4 P[3][2];
#pragma unroll
            for (int p = 0; p < 3; ++p) P[p][0] = P[p][1] = f32x4{};
            // the stage after this z block's last: the next z block, else the next column
            const bool last_zb = zb + 1 == nzb;
            const int64_t in = last_zb ? i + 1 : i;
            const int zbn = last_zb ? 0 : zb + 1;
            const bool more = !last_zb || c + 1 < ncol;
            // the stage after half 0: half 1, else the one after the z block
            if (nyh > 1) sg2_fill(a, i, zb, 1, wave, lds + ((s + 1) & 1) * SG2_STAGE);
            else if (more) sg2_fill(a, in, zbn, 0, wave, lds + ((s + 1) & 1) * SG2_STAGE);
            sg2_stage<0>(lds + (s & 1) * SG2_STAGE, nyc, kk, n16, Af, P);
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            __syncthreads();
            ++s;
            if (nyh > 1) {
                if (more) sg2_fill(a, in, zbn, 0, wave, lds + ((s + 1) & 1) * SG2_STAGE);
                sg2_stage<1>(lds + (s & 1) * SG2_STAGE, nyc, kk, n16, Af, P);
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                __syncthreads();
                ++s;
            }
            // acc[r] += Tz (P1 - P2 + i (P3 - P1 - P2)) over both n tiles
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float cr = P[0][nt][r] - P[1][nt][r];
                    const float ci = (P[2][nt][r] - P[0][nt][r]) - P[1][nt][r];
                    const float tr = tz[nt][r >> 1][2 * (r & 1)], ti = tz[nt][r >> 1][2 * (r & 1) + 1];
                    acc[2 * r] = __builtin_fmaf(-ti, ci, __builtin_fmaf(tr, cr, acc[2 * r]));
                    acc[2 * r + 1] = __builtin_fmaf(ti, cr, __builtin_fmaf(tr, ci, acc[2 * r + 1]));
                }
            }
        }
        // sum over the 16 z lanes (fixed butterfly order)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float v = acc[q];
            v += __shfl_xor(v, 8, 16);
            v += __shfl_xor(v, 4, 16);
            v += __shfl_xor(v, 2, 16);
            v += __shfl_xor(v, 1, 16);
            acc[q] = v;
        }
        if (n16 == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = jt * SG2_ROWS + 4 * kk + r;
                if (j < a.n) {
                    const int64_t out = j * a.n + i;
                    const float re = acc[2 * r], im = acc[2 * r + 1];
                    a.intensity[out] = re * re + im * im;
                    if (a.amplitude) ((float2*)a.amplitude)[out] = make_float2(re, im);
                }
            }
        }
    }
}

int grid_for(int64_t total, int block) { return (int)ceil_div(total, block); }

template <int CPW>
void launch_stage2(const SepG3Args& a, hipStream_t s)
{
    const int64_t nrb = a.npad / SG2_WG_ROWS;
    const dim3 grid((unsigned)(ceil_div(a.n, CPW) * nrb));
    hipLaunchKernelGGL((sepg_stage2_kernel<CPW>), grid, dim3(SG_THREADS), 0, s, a);
}

}  // namespace

int launch_sepg_twiddles(const SepDims& sd, int nx, int ny, int nxc3, const double* qx,
                         const double* qy, const double* xs, const double* ys, uint8_t* txa1,
                         uint8_t* txa2, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int B = 256;
    const int64_t n1 = (int64_t)sd.txa1g_bytes(nxc3) / 4;
    hipLaunchKernelGGL(sg_twiddle_a1, dim3(grid_for(n1, B)), dim3(B), 0, s, (float*)txa1, n1, sd.n, nx,
                       nxc3, qx, xs);
    const int64_t n2 = (int64_t)sd.txa2g_bytes() / 4;
    hipLaunchKernelGGL(sg_twiddle_a2, dim3(grid_for(n2, B)), dim3(B), 0, s, (float*)txa2, n2, sd.n, ny,
                       sd.nyc2, qy, ys);
    return (int)hipGetLastError();
}

// Both stages.  Stage 2 takes as many columns per workgroup as still leave two
// workgroups per CU.
int launch_sepg(const SepG3Args& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.n <= 0 || a.nyc2 <= 0 || a.nyc2 > SG2_MAXYC || a.npad % SG2_WG_ROWS) return (int)hipErrorInvalidValue;
    const dim3 g1((unsigned)a.nblk1, (unsigned)(a.nyc2 * 16 / SG1_PAIRS), (unsigned)a.nzb);
    hipLaunchKernelGGL(sepg_stage1_kernel, g1, dim3(SG_THREADS), 0, s, a);
    const int64_t nrb = a.npad / SG2_WG_ROWS;
    if (ceil_div(a.n, 8) * nrb >= 2 * CHIP_CUS) launch_stage2<8>(a, s);
    else if (ceil_div(a.n, 4) * nrb >= 2 * CHIP_CUS) launch_stage2<4>(a, s);
    else if (ceil_div(a.n, 2) * nrb >= 2 * CHIP_CUS) launch_stage2<2>(a, s);
    else launch_stage2<1>(a, s);
    return (int)hipGetLastError();
}

}  // namespace msft
