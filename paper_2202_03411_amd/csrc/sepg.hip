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
// Stage 1 (v_mfma_f32_16x16x4_f32): rows are a wave's 16 columns i, columns 16 z of
// a W tile, K four x values; a workgroup of 4 waves takes 64 columns, one z block and
// two quads of 4 consecutive y in turn, the sums over the x chunks stay in the MFMA
// accumulators, and each lane ends a quad with 4 consecutive y of its columns at 2 z:
// whole 16-byte slots of the H tiles.  The column blocks that read the same W tiles
// run on one XCD.
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

// 16x16x4 A operand [jt][chunk kc][plane 3][g 2][lane 64][e 4]: lane (kk, m) holds row
// r = 16 jt + m at K index k = 32 kc + 8 kk + 4 g + e (the H tile order; stage 2, and
// the adjoint's first pass) or, with wlay, k = 32 kc + 8 (2 g + kk / 2) + 2 e + kk % 2
// (the Gauss W tile order; stage 1), for MFMA step 4 g + e of chunk kc.  Value: the
// plane of exp(-i qy[r] ys[k]).
__global__ void sg_twiddle_a2(float* t, int64_t total, int n, int ny, int nyc2, const double* qy,
                              const double* ys, int wlay)
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
    const int kk = lane >> 4;
    const int y = yc * 32 + (wlay ? 8 * (2 * g + (kk >> 1)) + 2 * e + (kk & 1) : 8 * kk + 4 * g + e);
    t[idx] = (j < n && y < ny) ? plane_value(-(qy[j] * ys[y]), plane) : 0.0f;
}

// ---------------------------------------------------------------------------
// Stage 1.
// ---------------------------------------------------------------------------

// P += the three products of one W tile (all 32 x; the tables are zero beyond nx).
// The next step group's B fragments are read from LDS before the current group's
// MFMAs are issued.
__device__ __forceinline__ void sg1_tile(const uint8_t* row, int col, const f32x4* Af, f32x16 (&P)[3])
{
    const int sw = g3_swizzle(col);
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

// Stage 1, H(i, y, z) = sum_x Tx(i, x) W(x, y, z), on v_mfma_f32_16x16x4_f32: rows
// are a wave's 16 columns i, columns 16 z, K four x (lane (kk, n16) reads row (plane,
// x parity kk % 2, z) of the Gauss W tile, slot 2 g + kk / 2: x = 8 (2 g + kk / 2) +
// 2 e + kk % 2).  A workgroup of 4 waves takes 64 columns, one z block and SG1_QUADS
// quads of 4 consecutive y in turn; per quad the x chunks run through the two-slot
// LDS ring two tiles (two y) per stage, the sums over x stay in the accumulators,
// and each lane then holds, for its 4 columns and 2 z, the quad's 4 y: one 16-byte
// slot of an H tile per plane, 16 lanes writing 256 consecutive bytes.
constexpr int SG1_QUADS = 2;

// The stage (x chunk xc, y pair y, y + 1 of the quad) into an LDS slot of two W
// tiles: six pieces per thread (the second tile is the first again past ny).
__device__ __forceinline__ void sg1_fill(const SepG3Args& a, int xc, int zb, int y, int wave, uint8_t* slot)
{
    const int lane = threadIdx.x & 63;
    const uint8_t* t0 = a.wtiles + ((size_t)(xc * a.nzb + zb) * a.ny + y) * G3_TILE_BYTES;
    const uint8_t* t1 = y + 1 < a.ny ? t0 + G3_TILE_BYTES : t0;
#pragma unroll
    for (int p = 0; p < SG2_COPY; ++p) {
        const int q = (p % SG1_COPY) * SG_THREADS + wave * 64;   // piece of the wave's lane 0 in its tile
        const u32x4* src = (const u32x4*)(p < SG1_COPY ? t0 : t1);
        lds_dma16(src + q + lane, slot + (p < SG1_COPY ? 0 : G3_TILE_BYTES) + q * 16);
    }
}

// P[u][plane][n tile] += the products of the two W tiles of a stage (y of the quad
// u0, u0 + 1) with the wave's A operand for that x chunk: Af[2 plane + g], step 4 g + e.
__device__ __forceinline__ void sg1_stage(const uint8_t* slot, int kk, int n16, const f32x4 (&Af)[6],
                                          f32x4 (&P0)[3][2], f32x4 (&P1)[3][2])
{
    // B fragment of lane (kk, n16) for tile t, plane p, g, n tile nt: row (p, kk % 2, z)
    auto frag = [&](int t, int p, int g, int nt) {
        const int z = 16 * nt + n16;
        return *(const f32x4*)(slot + t * G3_TILE_BYTES + p * SG_PLANE_BYTES + ((kk & 1) * ZB + z) * G3_ROW_BYTES +
                               (((2 * g + (kk >> 1)) ^ g3_swizzle(z)) << 4));
    };
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 (&P)[3][2] = t == 0 ? P0 : P1;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const f32x4 b0 = frag(t, p, g, 0), b1 = frag(t, p, g, 1);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    P[p][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[2 * p + g][e], b0[e], P[p][0], 0, 0, 0);
                    P[p][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[2 * p + g][e], b1[e], P[p][1], 0, 0, 0);
                }
            }
        }
    }
}

// Grid (column blocks of 64, groups of SG1_QUADS y quads over nyc2 * 32, z blocks).
// Rows y >= ny of the H tiles are written as zeros; columns i >= N are not stored.
__global__ __launch_bounds__(SG_THREADS, 2) void sepg_stage1_kernel(SepG3Args a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * SG2_STAGE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kk = lane >> 4, n16 = lane & 15;
    // workgroup b runs on XCD b % 8: consecutive L (the column blocks of one y group
    // and z block, which read the same W tiles) share an XCD and its L2
    const int gx = gridDim.x, gy = gridDim.y;
    const int G = gx * gy * gridDim.z;
    const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int cb = L % gx, yg = (L / gx) % gy, zb = L / (gx * gy);
    const int64_t wt = (int64_t)cb * SG_WAVES + wave;   // 16 columns
    const int ybase = 4 * SG1_QUADS * yg;
    const int yend = min(a.ny, ybase + 4 * SG1_QUADS);   // rows y of this workgroup: [ybase, yend)
    const f32x4* ta = (const f32x4*)a.txa1 + (size_t)wt * a.nxc3 * 6 * 64 + lane;
    // stages (quad, xc, y pair) in that order; the one after (quad q, xc, pair v)
    auto next_stage = [&](int y0, int xc, int v, int& xn, int& yn) {
        if (v == 0 && y0 + 2 < min(yend, y0 + 4)) {
            xn = xc;
            yn = y0 + 2;
        } else if (xc + 1 < a.nxc3) {
            xn = xc + 1;
            yn = y0;
        } else {
            xn = 0;
            yn = y0 + 4;
        }
    };
    if (ybase < yend) {
        sg1_fill(a, 0, zb, ybase, wave, lds);
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        __syncthreads();
    }
    int k = 0;   // stages consumed so far; stage k sits in slot k & 1
#pragma unroll 1
    for (int qd = 0; qd < SG1_QUADS; ++qd) {
        const int y0 = ybase + 4 * qd;
        const int nyq = max(0, min(4, a.ny - y0));   // y of this quad inside the grid
        f32x4 P[4][3][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int p = 0; p < 3; ++p) P[u][p][0] = P[u][p][1] = f32x4{};
        for (int xc = 0; xc < a.nxc3 && nyq > 0; ++xc) {
            f32x4 Af[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) Af[q] = ta[(xc * 6 + q) * 64];
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                if (2 * v < nyq) {
                    int xn, yn;
                    next_stage(y0, xc, v, xn, yn);
                    if (yn < yend) sg1_fill(a, xn, zb, yn, wave, lds + ((k + 1) & 1) * SG2_STAGE);
                    sg1_stage(lds + (k & 1) * SG2_STAGE, kk, n16, Af, P[2 * v], P[2 * v + 1]);
                    // the next slot's loads have landed (the compiler does not track them)
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                    __syncthreads();
                    ++k;
                }
            }
        }
        // H = (P1 - P2) + i (P3 - P1 - P2) and Hr + Hi at y0 .. y0 + 3 of column i, z:
        // the 16-byte slot (kk', g') = ((y0 % 32) / 8, (y0 % 8) / 4) of row z
        const int yc = y0 >> 5, yl = y0 & 31;
        const size_t col_stride = (size_t)a.nyc2 * a.nzb * G3_TILE_BYTES;
        uint8_t* hbase = a.htiles + ((size_t)yc * a.nzb + zb) * G3_TILE_BYTES + (((yl >> 3) * 2 + ((yl >> 2) & 1)) * 32 + n16) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = wt * SG2_ROWS + 4 * kk + r;
            if (i < a.n) {
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    f32x4 hr, hi, hs;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        // (a y beyond ny summed a repeated tile: its row is zero)
                        const bool in = u < nyq;
                        hr[u] = in ? P[u][0][nt][r] - P[u][1][nt][r] : 0.0f;
                        hi[u] = in ? (P[u][2][nt][r] - P[u][0][nt][r]) - P[u][1][nt][r] : 0.0f;
                        hs[u] = hr[u] + hi[u];
                    }
                    uint8_t* t = hbase + i * col_stride + nt * 256;
                    *(f32x4*)t = hr;
                    *(f32x4*)(t + SG_PLANE_BYTES) = hi;
                    *(f32x4*)(t + 2 * SG_PLANE_BYTES) = hs;
                }
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

// ---------------------------------------------------------------------------
// Adjoint.  With h = g conj(A) the strength gradient needs
//   R(x, y, z) = sum_{i,j} h(i, j) exp(-i (q_x(i) x + q_y(j) y + q_z(i, j) z)),
// the transposed two-stage sum:
//   K(i, y, z) = sum_j exp(-i q_y(j) y) [h(i, j) exp(-i q_z(i, j) z)]   (pass 1)
//   R(x, y, z) = sum_i exp(-i q_x(i) x) K(i, y, z)                      (pass 2)
// Pass 1 (v_mfma_f32_16x16x4_f32): rows are a wave's 16 y, columns 16 z, K four
// rows j; a workgroup takes 64 y, SGA_COLS columns i and one z block.  Each thread
// loads its own Tz and h for the chunk after next into registers, and forms the
// next chunk's B tiles h Tz (three planes) into the other LDS buffer between the
// current chunk's MFMAs, one barrier per chunk; K goes out as two planes Kr, Ki of
// [i][y][z] floats (16 lanes store 16 consecutive z).  Pass 2 (sepg_adj_cols_kernel)
// has the shape of stage 1 with rows x and K over the columns i, split in two
// halves whose partial sums the column walk adds.
// ---------------------------------------------------------------------------
constexpr int SGA_COLS = 2;

// P[c] += the three products of the B tiles of 32 j of NC columns (the H tile
// layout, j in place of y; column c at tiles + c G3_TILE_BYTES) with the wave's A
// operand for that chunk: Af[2 plane + g], step 4 g + e.  Groups (column, g, plane)
// of eight MFMAs; the next group's B fragments are read from LDS before the current
// group's MFMAs are issued.  form(c) (the next chunk's B tiles of column c, into the
// other LDS buffer: VALU work and three LDS stores) is spread between the MFMAs of
// the groups FORM0 and FORM1 - 1.
template <int NC, bool FORM, class Form>
__device__ __forceinline__ void sga_tiles(const uint8_t* tiles, int kk, int n16, const f32x4 (&Af)[6],
                                          f32x4 (&P)[SGA_COLS][3][2], Form&& form)
{
    constexpr int NG = NC * 6;
    constexpr int FORM0 = 2, FORM1 = 8;
    static_assert(NG > FORM1, "two groups to hide the forming under");
    const uint8_t* base = tiles + kk * 1024 + n16 * 16;
    // group k: column k / 6, g = (k / 3) % 2, plane k % 3
    auto frag = [&](int k, int nt) {
        return *(const f32x4*)(base + (k / 6) * G3_TILE_BYTES + (k % 3) * SG_PLANE_BYTES + ((k / 3) % 2) * 512 +
                               nt * 256);
    };
    f32x4 b[2][2];
    b[0][0] = frag(0, 0);
    b[0][1] = frag(0, 1);
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        if (k + 1 < NG) {
            b[(k + 1) & 1][0] = frag(k + 1, 0);
            b[(k + 1) & 1][1] = frag(k + 1, 1);
        }
        if (FORM && (k == FORM0 || k == FORM1)) {
            // this region holds group k - 1's MFMAs, group k + 1's reads and one
            // column's forming: reads first, then one MFMA per three VALU operations,
            // the stores last
            form(k == FORM0 ? 0 : 1);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x200, 3, 0);
        }
        // keep the next group's reads ahead of this group's MFMAs
        __builtin_amdgcn_sched_barrier(0);
        const int c = k / 6, g = (k / 3) % 2, p = k % 3;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                P[c][p][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[2 * p + g][e], b[k & 1][nt][e], P[c][p][nt], 0,
                                                                   0, 0);
    }
}

// Grid: (blocks of 64 y) x (column groups over nic3 * 32) x (z blocks), blocks of y
// fastest; the y blocks of one column group run on one XCD, so their Tz comes from
// HBM about once.  Columns i >= N (up to nic3 * 32) store zeros; rows y >= ny are
// not stored.
__global__ __launch_bounds__(SG_THREADS, 2) void sepg_adj_rows_kernel(SepG3AdjArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * SGA_COLS * G3_TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kk = lane >> 4, n16 = lane & 15;
    // workgroup b runs on XCD b % 8: consecutive L share an XCD
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int nyb = (a.ny + SG2_WG_ROWS - 1) / SG2_WG_ROWS, ncg = a.nic3 * 32 / SGA_COLS;
    const int64_t yt = (L % nyb) * SG_WAVES + wave;   // row tile of 16 y
    const int i0 = (int)(SGA_COLS * ((L / nyb) % ncg)), zb = (int)(L / ((int64_t)nyb * ncg));
    const int ncol = max(0, min(SGA_COLS, a.n - i0));           // columns inside the detector
    // the thread's slot of each B tile: rows j = 8 fk + 4 fg + e (e = 0..3) at z = fz
    const int fk = tid >> 6, fg = (tid >> 5) & 1, fz = tid & 31;
    f32x4 P[SGA_COLS][3][2];
#pragma unroll
    for (int c = 0; c < SGA_COLS; ++c)
#pragma unroll
        for (int p = 0; p < 3; ++p) P[c][p][0] = P[c][p][1] = f32x4{};
    if (ncol > 0) {
        // the thread's Tz of chunk jc, straight into registers: per column c the
        // 16-row tile w16 = i (npad / 16) + 2 jc + fk / 2 is a contiguous block
        // (hp, z, m) of 4 KiB holding row 4 (m / 2) + 2 hp + m % 2 at z, so rows
        // 8 fk + 4 fg + e sit at hp = e / 2, m = 4 (fk % 2) + 2 fg + e % 2: one 16-byte
        // piece per hp (a column beyond the detector loads the last one; its h is
        // taken as zero)
        auto load_tz = [&](int jc, f32x4 (&tz)[SGA_COLS][2]) {
#pragma unroll
            for (int c = 0; c < SGA_COLS; ++c) {
                const int64_t w16 = (int64_t)min(i0 + c, a.n - 1) * (a.npad / SG2_ROWS) + 2 * jc + (fk >> 1);
                const float* blk = a.tz + (w16 * a.nzb + zb) * (2 * 2 * ZB * 8);
#pragma unroll
                for (int hp = 0; hp < 2; ++hp)
                    tz[c][hp] = *(const f32x4*)(blk + ((hp * ZB + fz) * 8 + 4 * (fk & 1) + 2 * fg) * 2);
            }
        };
        // h of the thread's rows j = 32 jc + 8 fk + 4 fg + e for the columns i0, i0 + 1,
        // one 16-byte piece per row (the row clamped into the detector; form_b zeroes
        // the rows and columns beyond it)
        auto load_h = [&](int jc, u32x4 (&hv)[4]) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                hv[e] = *(const u32x4*)((const float2*)a.h + (int64_t)min(32 * jc + 8 * fk + 4 * fg + e, a.n - 1) * a.n + i0);
        };
        // column c of B = h Tz for chunk jc in three planes, rows j = 8 fk + 4 fg + e of
        // the tile at z = fz
        auto form_b = [&](int jc, int c, const f32x4 (&tz)[SGA_COLS][2], const u32x4 (&hv)[4], uint8_t* slot) {
            f32x4 br, bi, bs;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool in = 32 * jc + 8 * fk + 4 * fg + e < a.n && c < ncol;
                const float hr = in ? __uint_as_float(hv[e][2 * c]) : 0.0f;
                const float hi = in ? __uint_as_float(hv[e][2 * c + 1]) : 0.0f;
                const float tr = tz[c][e >> 1][2 * (e & 1)], ti = tz[c][e >> 1][2 * (e & 1) + 1];
                br[e] = hr * tr - hi * ti;
                bi[e] = hr * ti + hi * tr;
                bs[e] = br[e] + bi[e];
            }
            uint8_t* q = slot + c * G3_TILE_BYTES + ((fk * 2 + fg) * 32 + fz) * 16;
            *(f32x4*)q = br;
            *(f32x4*)(q + SG_PLANE_BYTES) = bi;
            *(f32x4*)(q + 2 * SG_PLANE_BYTES) = bs;
        };
        auto buf = [&](int jc) { return lds + (jc & 1) * SGA_COLS * G3_TILE_BYTES; };
        const f32x4* ta = (const f32x4*)a.tyT + (size_t)yt * a.njc2 * 6 * 64 + lane;
        // two register sets, taking turns: A operand of the chunk in flight, and Tz
        // and h of the chunk after it
        f32x4 AcA[6], AcB[6], tzA[SGA_COLS][2], tzB[SGA_COLS][2];
        u32x4 hA[4], hB[4];
#pragma unroll
        for (int q = 0; q < 6; ++q) AcA[q] = ta[q * 64];
        load_tz(0, tzA);
        load_h(0, hA);
#pragma unroll
        for (int c = 0; c < SGA_COLS; ++c) form_b(0, c, tzA, hA, buf(0));
        load_tz(min(1, a.njc2 - 1), tzA);
        load_h(min(1, a.njc2 - 1), hA);
        __syncthreads();
        // chunk jc's MFMAs (A operand Acur), chunk jc + 1's tiles formed under them from
        // tzc, hc into the other buffer (last read before the previous barrier); the
        // loads for the next step go out first: chunk jc + 1's A operand into Anext,
        // chunk jc + 2's Tz and h (clamped to the last chunk, so every path issues the
        // same loads) into tzn, hn
        auto step = [&](int jc, const f32x4 (&Acur)[6], f32x4 (&Anext)[6], const f32x4 (&tzc)[SGA_COLS][2],
                        const u32x4 (&hc)[4], f32x4 (&tzn)[SGA_COLS][2], u32x4 (&hn)[4]) {
#pragma unroll
            for (int q = 0; q < 6; ++q) Anext[q] = ta[((jc + 1) * 6 + q) * 64];
            const int jn = min(jc + 2, a.njc2 - 1);
            load_tz(jn, tzn);
            load_h(jn, hn);
            sga_tiles<SGA_COLS, true>(buf(jc), kk, n16, Acur, P,
                                      [&](int c) { form_b(jc + 1, c, tzc, hc, buf(jc + 1)); });
            __syncthreads();
        };
        int jc = 0;
        for (; jc + 2 < a.njc2; jc += 2) {
            step(jc, AcA, AcB, tzA, hA, tzB, hB);
            step(jc + 1, AcB, AcA, tzB, hB, tzA, hA);
        }
        if (jc + 1 < a.njc2) {
            step(jc, AcA, AcB, tzA, hA, tzB, hB);
            sga_tiles<SGA_COLS, false>(buf(jc + 1), kk, n16, AcB, P, [&](int) {});
        } else {
            sga_tiles<SGA_COLS, false>(buf(jc), kk, n16, AcA, P, [&](int) {});
        }
    }
    // K = (P1 - P2) + i (P3 - P1 - P2), planes Kr, Ki of [i][y][z2] floats (pass 2
    // forms Kr + Ki from them): 16 lanes write 16 consecutive z
    const size_t plane = (size_t)a.nic3 * 32 * a.ny * a.nz2;
#pragma unroll
    for (int c = 0; c < SGA_COLS; ++c) {
        const int i = i0 + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t y = yt * SG2_ROWS + 4 * kk + r;
            if (y < a.ny) {
                float* k = a.kplain + ((size_t)i * a.ny + y) * a.nz2 + zb * ZB + n16;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const float kr = P[c][0][nt][r] - P[c][1][nt][r];
                    const float ki = (P[c][2][nt][r] - P[c][0][nt][r]) - P[c][1][nt][r];
                    k[16 * nt] = kr;
                    k[plane + 16 * nt] = ki;
                }
            }
        }
    }
}

// Pass 2: R(x, y, z) = sum_i exp(-i q_x(i) x) K(i, y, z), on the 32x32x2 Gauss block (rows x of 32
// per wave, 128 per workgroup, one y pair, one z block, one half of the i chunks)
// with the B tiles built in LDS from the plain K planes: a thread gathers, for one
// row (plane, i parity h, z) of a tile, the four i of one 16-byte slot (coalesced
// over z across the lanes) and writes the slot with one LDS store.  The next tile's
// values are loaded during the current tile's MFMAs.
__global__ __launch_bounds__(SG_THREADS, 2) void sepg_adj_cols_kernel(SepG3AdjArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * G3_TILE_BYTES];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, col = lane & 31;
    const int64_t wt = (int64_t)blockIdx.x * SG_WAVES + wave;
    const int zb = (int)(blockIdx.z % a.nzb), split = (int)(blockIdx.z / a.nzb);
    const int per = (a.nic3 + SEPG_ADJ_SPLIT - 1) / SEPG_ADJ_SPLIT;
    const int kc0 = split * per, kc1 = min(a.nic3, kc0 + per);
    const int y0 = 2 * blockIdx.y;
    const int nyh = min(2, a.ny - y0);   // >= 1
    const size_t plane = (size_t)a.nic3 * 32 * a.ny * a.nz2;
    // the thread's slots: (plane q, h, z = col, g = wave); i = 32 kc + 8 g + 2 e + h;
    // planes Kr, Ki are loaded, Kr + Ki formed here (the same FP32 sum pass 1 would store)
    auto load_tile = [&](int kc, int y, float (&v)[2][4]) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[q][e] = a.kplain[q * plane + ((size_t)(32 * kc + 8 * wave + 2 * e + h) * a.ny + y) * a.nz2 +
                                   zb * ZB + col];
    };
    auto store_tile = [&](uint8_t* slot, const float (&v)[2][4]) {
        uint8_t* q0 = slot + (h * ZB + col) * G3_ROW_BYTES + ((wave ^ g3_swizzle(col)) << 4);
        *(f32x4*)q0 = f32x4{v[0][0], v[0][1], v[0][2], v[0][3]};
        *(f32x4*)(q0 + SG_PLANE_BYTES) = f32x4{v[1][0], v[1][1], v[1][2], v[1][3]};
        *(f32x4*)(q0 + 2 * SG_PLANE_BYTES) =
            f32x4{v[0][0] + v[1][0], v[0][1] + v[1][1], v[0][2] + v[1][2], v[0][3] + v[1][3]};
    };
    f32x16 P[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 3; ++q) P[u][q] = f32x16{};
    if (kc0 < kc1) {
        float v[2][4];
        load_tile(kc0, y0, v);
        store_tile(lds, v);
        __syncthreads();
        int k = 0;   // tiles consumed so far, in the order (kc, y); tile k sits in slot k & 1
        for (int kc = kc0; kc < kc1; ++kc) {
            f32x4 Af[12];
            const f32x4* ta = (const f32x4*)(a.txT + (size_t)(wt * a.nic3 + kc) * G3_TILE_BYTES);
#pragma unroll
            for (int q = 0; q < 12; ++q) Af[q] = ta[q * 64 + lane];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u < nyh) {
                    const bool same = u + 1 < nyh;
                    const bool more = same || kc + 1 < kc1;
                    if (more) load_tile(same ? kc : kc + 1, same ? y0 + u + 1 : y0, v);
                    sg1_tile(lds + (k & 1) * G3_TILE_BYTES + (h * ZB + col) * G3_ROW_BYTES, col, Af, P[u]);
                    // the other slot was last read before the previous barrier
                    if (more) store_tile(lds + ((k + 1) & 1) * G3_TILE_BYTES, v);
                    __syncthreads();
                    ++k;
                }
            }
        }
    }
    // R = (P1 - P2) + i (P3 - P1 - P2): 32 lanes write 32 consecutive z
    float2* out = (float2*)a.rpart + (size_t)split * a.rows_pad * a.ny * a.nz2 + zb * ZB + col;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t x = wt * G3_WAVE_PIX + 8 * (r >> 2) + 4 * h + (r & 3);
        if (x < a.nx) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (u < nyh)
                    out[((size_t)x * a.ny + y0 + u) * a.nz2] =
                        make_float2(P[u][0][r] - P[u][1][r], (P[u][2][r] - P[u][0][r]) - P[u][1][r]);
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
    hipLaunchKernelGGL(sg_twiddle_a2, dim3(grid_for(n1, B)), dim3(B), 0, s, (float*)txa1, n1, sd.n, nx,
                       nxc3, qx, xs, 1);
    const int64_t n2 = (int64_t)sd.txa2g_bytes() / 4;
    hipLaunchKernelGGL(sg_twiddle_a2, dim3(grid_for(n2, B)), dim3(B), 0, s, (float*)txa2, n2, sd.n, ny,
                       sd.nyc2, qy, ys, 0);
    return (int)hipGetLastError();
}

// Both stages.  Stage 1 walks two y quads per workgroup; stage 2 takes as many
// columns per workgroup as still leave two workgroups per CU.
int launch_sepg(const SepG3Args& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.n <= 0 || a.nyc2 <= 0 || a.nyc2 > SG2_MAXYC || a.npad % SG2_WG_ROWS) return (int)hipErrorInvalidValue;
    const dim3 g1((unsigned)ceil_div(a.n, SG_WAVES * SG2_ROWS), (unsigned)(a.nyc2 * 32 / (4 * SG1_QUADS)),
                  (unsigned)a.nzb);
    hipLaunchKernelGGL(sepg_stage1_kernel, g1, dim3(SG_THREADS), 0, s, a);
    const int64_t nrb = a.npad / SG2_WG_ROWS;
    if (ceil_div(a.n, 8) * nrb >= 2 * CHIP_CUS) launch_stage2<8>(a, s);
    else if (ceil_div(a.n, 4) * nrb >= 2 * CHIP_CUS) launch_stage2<4>(a, s);
    else if (ceil_div(a.n, 2) * nrb >= 2 * CHIP_CUS) launch_stage2<2>(a, s);
    else launch_stage2<1>(a, s);
    return (int)hipGetLastError();
}

// The adjoint's tables: pass 1 A [16 rows y][j chunk] exp(-i q_y(j) y), pass 2 A
// [32 rows x][i chunk] exp(-i q_x(i) x); ys, xs the voxel coordinates, qy, qx the
// per-row and per-column components.
int launch_sepg_adj_tables(const SepDims& sd, int nx, int ny, const double* xs, const double* qx,
                           const double* ys, const double* qy, uint8_t* txT, uint8_t* tyT, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int B = 256;
    const int64_t n1 = (int64_t)sd.tyTg_bytes(ny) / 4;
    hipLaunchKernelGGL(sg_twiddle_a2, dim3(grid_for(n1, B)), dim3(B), 0, s, (float*)tyT, n1, ny, sd.n, sd.nic3,
                       ys, qy, 0);
    const int64_t n2 = (int64_t)sd.txTg_bytes(nx) / 4;
    hipLaunchKernelGGL(sg_twiddle_a1, dim3(grid_for(n2, B)), dim3(B), 0, s, (float*)txT, n2, nx, sd.n, sd.nic3,
                       xs, qx);
    return (int)hipGetLastError();
}

// Both passes of the adjoint; R goes to a.rpart as two partial sums.
int launch_sepg_adjoint(const SepG3AdjArgs& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.n <= 0 || a.njc2 <= 0 || a.nic3 <= 0) return (int)hipErrorInvalidValue;
    const dim3 g1((unsigned)(ceil_div(a.ny, SG2_WG_ROWS) * (a.nic3 * 32 / SGA_COLS) * a.nzb));
    hipLaunchKernelGGL(sepg_adj_rows_kernel, g1, dim3(SG_THREADS), 0, s, a);
    const dim3 g2((unsigned)ceil_div(a.nx, SG_WAVES * G3_WAVE_PIX), (unsigned)ceil_div(a.ny, 2),
                  (unsigned)(a.nzb * SEPG_ADJ_SPLIT));
    hipLaunchKernelGGL(sepg_adj_cols_kernel, g2, dim3(SG_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

}  // namespace msft
