// gfx950 Gauss (3M) form of the FP32 forward contraction (flat detector and q
// lists): the x-sum of T W with three real MFMA products per complex
// multiply-add, followed by the same fused y/z phase reduction and |A|^2.
//
//   for each x chunk xc:     A operands Tr, Ti, Tr + Ti of the wave's 32 pixels
//     for each z block zb:   G = 0
//       for each y:          P1 = Tr.Wr, P2 = Ti.Wi, P3 = (Tr+Ti).(Wr+Wi)  (MFMA)
//                            C = (P1 - P2) + i (P3 - P1 - P2)
//                            G += exp(-i q_y y) C        (per pixel row, lane = z)
//       acc += exp(-i q_z z) G
//   A_p = sum over the 32 z lanes of acc;  I_p = |A_p|^2
//
// v_mfma_f32_32x32x2_f32: rows are the wave's 32 pixels, columns the 32 z of a
// tile, K two x values (x parity = lane half).  Lane l holds output rows
// 8j + 4h + u (j, u = 0..3, h = l / 32) at z = l % 32.  Four waves make a pixel
// block and two blocks share a CU (256 registers per lane), so each SIMD runs two
// waves whose barriers are independent.  W tiles stream through a double-buffered
// LDS ring.  Sums run in an order fixed by the plan alone.
#include <hip/hip_runtime.h>

#include "msft_internal.h"

namespace msft {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int G3_THREADS = 64 * G3_WAVES;
constexpr int G3_PLANE_BYTES = 2 * ZB * G3_ROW_BYTES;     // 4 KB
constexpr int G3_TILE_F4 = G3_TILE_BYTES / 16;            // 768
constexpr int G3_COPY = G3_TILE_F4 / G3_THREADS;          // 16-byte pieces per thread per tile
constexpr int G3_STEPS = G3_XC / 8;                       // f32x4 A values per plane
static_assert(G3_COPY * G3_THREADS == G3_TILE_F4, "a tile is copied in whole pieces");

// Pixel of Gauss wave wt at lane half h, output row r (0..15) of the lane.
__device__ __forceinline__ int64_t g3_pixel(int64_t wt, int h, int r)
{
    return wt * G3_WAVE_PIX + 8 * (r >> 2) + 4 * h + (r & 3);
}

// ---------------------------------------------------------------------------
// Plan-time tables.  T = exp(i phi), phi = -q . r, phases in FP64.
// ---------------------------------------------------------------------------

// A tiles [wt][xc][plane 3][g 4][lane 64][e 4] floats: lane (h, i) holds, for MFMA
// step 4g + e, pixel wt*32 + i at x = xc*32 + 8g + 2e + h; planes Re T, Im T,
// Re T + Im T (the sum formed in FP64).
__global__ void twiddle_txa_g3(float* txa, int64_t total, int64_t npix, int nx, int nxc,
                               const double* q, const double* xs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int f = (int)(idx % (G3_TILE_BYTES / 4));
    const int64_t tile = idx / (G3_TILE_BYTES / 4);
    const int plane = f / (G3_PLANE_BYTES / 4), rem = f % (G3_PLANE_BYTES / 4);
    const int g = rem >> 8, lane = (rem >> 2) & 63, e = rem & 3;
    const int xc = (int)(tile % nxc);
    const int64_t wt = tile / nxc;
    const int64_t pix = wt * G3_WAVE_PIX + (lane & 31);
    const int x = xc * G3_XC + 8 * g + 2 * e + (lane >> 5);
    float v = 0.0f;
    if (pix < npix && x < nx) {
        double sn, cs;
        sincos(-(q[3 * pix] * xs[x]), &sn, &cs);
        v = (float)(plane == 0 ? cs : plane == 1 ? sn : cs + sn);
    }
    txa[idx] = v;
}

// Ty [wt][y][h][r 16] complex: exp(-i q_y y) of the pixel of lane half h, row r.
__global__ void twiddle_ty_g3(float2* ty, int64_t total, int64_t npix, int ny, const double* q,
                              const double* ys)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int r = (int)(idx & 15);
    const int h = (int)((idx >> 4) & 1);
    const int64_t rest = idx >> 5;
    const int y = (int)(rest % ny);
    const int64_t wt = rest / ny;
    const int64_t pix = g3_pixel(wt, h, r);
    float2 v = make_float2(0.0f, 0.0f);
    if (pix < npix) {
        double sn, cs;
        sincos(-(q[3 * pix + 1] * ys[y]), &sn, &cs);
        v = make_float2((float)cs, (float)sn);
    }
    ty[idx] = v;
}

// Tz [wt][zb][h][z 32][r 16] complex: exp(-i q_z z), zero beyond nz and for a
// pixel whose q_z is not finite.
__global__ void twiddle_tz_g3(float2* tz, int64_t total, int64_t npix, int nz, int nzb,
                              const double* q, const double* zs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int r = (int)(idx & 15);
    const int zl = (int)((idx >> 4) & 31);
    const int h = (int)((idx >> 9) & 1);
    const int64_t rest = idx >> 10;
    const int zb = (int)(rest % nzb);
    const int64_t wt = rest / nzb;
    const int64_t pix = g3_pixel(wt, h, r);
    const int z = zb * ZB + zl;
    float2 v = make_float2(0.0f, 0.0f);
    if (pix < npix && z < nz && isfinite(q[3 * pix + 2])) {
        double sn, cs;
        sincos(-(q[3 * pix + 2] * zs[z]), &sn, &cs);
        v = make_float2((float)cs, (float)sn);
    }
    tz[idx] = v;
}

// ---------------------------------------------------------------------------
// Contraction.
// ---------------------------------------------------------------------------

// The wave's A operand for one x chunk: Af[plane * G3_STEPS + g].
__device__ __forceinline__ void load_a_g3(const uint8_t* ta, int lane, f32x4* Af)
{
#pragma unroll
    for (int k = 0; k < 3 * G3_STEPS; ++k) Af[k] = ((const f32x4*)ta)[k * 64 + lane];
}

// The three products of one W tile over its first xlen x (all G3_XC when FULL).
// row: the lane's row (plane 0, h, z = col) of the tile in LDS; the planes follow
// at G3_PLANE_BYTES.
template <bool FULL>
__device__ __forceinline__ void tile_g3(const uint8_t* row, int col, int xlen, const f32x4* Af,
                                        f32x16& P1, f32x16& P2, f32x16& P3)
{
    const int sw = g3_swizzle(col);
    P1 = f32x16{};
    P2 = f32x16{};
    P3 = f32x16{};
#pragma unroll
    for (int g = 0; g < G3_STEPS; ++g) {
        if (FULL || 8 * g < xlen) {
            const int off = (g ^ sw) << 4;
            const f32x4 b1 = *(const f32x4*)(row + off);
            const f32x4 b2 = *(const f32x4*)(row + G3_PLANE_BYTES + off);
            const f32x4 b3 = *(const f32x4*)(row + 2 * G3_PLANE_BYTES + off);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                P1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[g][e], b1[e], P1, 0, 0, 0);
                P2 = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[G3_STEPS + g][e], b2[e], P2, 0, 0, 0);
                P3 = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[2 * G3_STEPS + g][e], b3[e], P3, 0, 0, 0);
            }
        }
    }
}

// G[r] += Ty[r] * C[r], C = (P1 - P2) + i (P3 - P1 - P2); G interleaved re, im;
// ty: 8 x f32x4 = 16 complex.  Each component takes two chained FMAs into G.
__device__ __forceinline__ void combine_rotate(float* G, const f32x16& P1, const f32x16& P2,
                                               const f32x16& P3, const f32x4* ty)
{
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float cr = P1[r] - P2[r];
        const float ci = (P3[r] - P1[r]) - P2[r];
        const float tr = ty[r >> 1][2 * (r & 1)], ti = ty[r >> 1][2 * (r & 1) + 1];
        G[2 * r] = __builtin_fmaf(-ti, ci, __builtin_fmaf(tr, cr, G[2 * r]));
        G[2 * r + 1] = __builtin_fmaf(ti, cr, __builtin_fmaf(tr, ci, G[2 * r + 1]));
    }
}

// All z blocks of one x chunk, one W tile per pipeline stage; t: next tile.
template <bool FULL>
__device__ __forceinline__ void chunk_g3(const FwdArgs& a, int64_t wt, int64_t ntiles, const u32x4* gw,
                                         uint8_t* lds, int xlen, const f32x4* Af, int64_t& t,
                                         float* acc)
{
    // acc: the lane's 32 running sums in LDS, stride 64 floats (they change once per
    // z block; keeping them out of registers leaves room for two waves per SIMD)
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5, col = lane & 31;
    for (int zb = 0; zb < a.nzb; ++zb) {
        float G[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) G[q] = 0.0f;
        for (int y = 0; y < a.ny; ++y, ++t) {
            const bool has_next = (t + 1) < ntiles;
            u32x4 nx[G3_COPY];
            if (has_next) {
#pragma unroll
                for (int u = 0; u < G3_COPY; ++u) nx[u] = gw[(t + 1) * G3_TILE_F4 + u * G3_THREADS + tid];
            }
            const f32x4* typ = (const f32x4*)(a.ty + 2 * (((wt * a.ny + y) * 2 + h) * 16));
            f32x4 ty[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) ty[u] = typ[u];
            const uint8_t* row = lds + (size_t)(t & 1) * G3_TILE_BYTES + (h * ZB + col) * G3_ROW_BYTES;
            f32x16 P1, P2, P3;
            tile_g3<FULL>(row, col, xlen, Af, P1, P2, P3);
            combine_rotate(G, P1, P2, P3, ty);
            if (has_next) {
                u32x4* nb = (u32x4*)(lds + (size_t)((t + 1) & 1) * G3_TILE_BYTES);
#pragma unroll
                for (int u = 0; u < G3_COPY; ++u) nb[u * G3_THREADS + tid] = nx[u];
            }
            __syncthreads();
        }
        // acc[r] += Tz[r] * G[r]
        const f32x4* tzp = (const f32x4*)(a.tz + 2 * ((((wt * a.nzb + zb) * 2 + h) * ZB + col) * 16));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const f32x4 v = tzp[q];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int r = 2 * q + u;
                const float tr = v[2 * u], ti = v[2 * u + 1];
                acc[(2 * r) * 64] += tr * G[2 * r] - ti * G[2 * r + 1];
                acc[(2 * r + 1) * 64] += tr * G[2 * r + 1] + ti * G[2 * r];
            }
        }
    }
}

__device__ __forceinline__ void block_g3(const FwdArgs& a, int64_t block, uint8_t* lds, float* accs)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t wt = block * G3_WAVES + wave;
    const int64_t ntiles = (int64_t)a.nxc * a.nzb * a.ny;
    const u32x4* gw = (const u32x4*)a.wtiles;

    // first stage: tile 0 -> LDS buffer 0
#pragma unroll
    for (int u = 0; u < G3_COPY; ++u) ((u32x4*)lds)[u * G3_THREADS + tid] = gw[u * G3_THREADS + tid];
    __syncthreads();

    float* accl = accs + wave * 32 * 64 + lane;   // [wave][q][lane]
#pragma unroll
    for (int q = 0; q < 32; ++q) accl[q * 64] = 0.0f;

    int64_t t = 0;
    for (int xc = 0; xc < a.nxc; ++xc) {
        const int xlen = min(G3_XC, a.x_pad - xc * G3_XC);
        f32x4 Af[3 * G3_STEPS];
        load_a_g3(a.txa + (size_t)(wt * a.nxc + xc) * G3_TILE_BYTES, lane, Af);
        // one wait for the A operand per chunk (the memory counter is in order)
        __builtin_amdgcn_s_waitcnt(0);
        if (xlen == G3_XC) chunk_g3<true>(a, wt, ntiles, gw, lds, xlen, Af, t, accl);
        else chunk_g3<false>(a, wt, ntiles, gw, lds, xlen, Af, t, accl);
    }
    const int h = lane >> 5, col = lane & 31;

    // sum over the 32 z lanes of each half (fixed butterfly order)
    float acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        float v = accl[q * 64];
        v += __shfl_xor(v, 16, 32);
        v += __shfl_xor(v, 8, 32);
        v += __shfl_xor(v, 4, 32);
        v += __shfl_xor(v, 2, 32);
        v += __shfl_xor(v, 1, 32);
        acc[q] = v;
    }
    if (col == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t pix = g3_pixel(wt, h, r);
            if (pix < a.npix) {
                const float re = acc[2 * r], im = acc[2 * r + 1];
                a.intensity[pix] = re * re + im * im;
                if (a.amplitude) ((float2*)a.amplitude)[pix] = make_float2(re, im);
            }
        }
    }
}

__global__ __launch_bounds__(G3_THREADS, 2) void fwd_g3_kernel(FwdArgs a, int64_t block_begin)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * G3_TILE_BYTES];
    __shared__ float accs[G3_WAVES * 32 * 64];
    block_g3(a, block_begin + blockIdx.x, lds, accs);
}

// Batched form: one workgroup per (request, pixel block) item in the host's order.
__global__ __launch_bounds__(G3_THREADS, 2) void fwd_g3_batch_kernel(BatchArgs b)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * G3_TILE_BYTES];
    __shared__ float accs[G3_WAVES * 32 * 64];
    const int32_t it = blockIdx.x;
    int r = 0;
    while (r + 1 < b.nreq && b.item_begin[r + 1] <= it) ++r;
    block_g3(b.req[r], (int64_t)b.block_begin[r] + (it - b.item_begin[r]), lds, accs);
}

int grid_for(int64_t total, int block) { return (int)ceil_div(total, block); }

}  // namespace

int launch_twiddles_g3(const Dims& d, const double* q_dev, const double* xs_dev, const double* ys_dev,
                       const double* zs_dev, uint8_t* txa, float* ty, float* tz, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int B = 256;
    const int64_t nwt = d.nblocks * G3_WAVES;
    const int64_t na = nwt * d.nxc3 * (G3_TILE_BYTES / 4);
    hipLaunchKernelGGL(twiddle_txa_g3, dim3(grid_for(na, B)), dim3(B), 0, s, (float*)txa, na, d.npix,
                       d.nx, d.nxc3, q_dev, xs_dev);
    const int64_t nty = nwt * d.ny * G3_WAVE_PIX;
    hipLaunchKernelGGL(twiddle_ty_g3, dim3(grid_for(nty, B)), dim3(B), 0, s, (float2*)ty, nty, d.npix,
                       d.ny, q_dev, ys_dev);
    const int64_t ntz = nwt * d.nzb * 2 * ZB * 16;
    hipLaunchKernelGGL(twiddle_tz_g3, dim3(grid_for(ntz, B)), dim3(B), 0, s, (float2*)tz, ntz, d.npix,
                       d.nz, d.nzb, q_dev, zs_dev);
    return (int)hipGetLastError();
}

int launch_forward_g3(const FwdArgs& a, int64_t block_begin, int64_t nblocks, void* stream)
{
    if (nblocks <= 0) return 0;
    hipLaunchKernelGGL(fwd_g3_kernel, dim3((unsigned)nblocks), dim3(G3_THREADS), 0,
                       (hipStream_t)stream, a, block_begin);
    return (int)hipGetLastError();
}

int launch_forward_batch_g3(const BatchArgs& b, void* stream)
{
    const int32_t items = b.nreq > 0 ? b.item_begin[b.nreq] : 0;
    if (items <= 0) return 0;
    hipLaunchKernelGGL(fwd_g3_batch_kernel, dim3(items), dim3(G3_THREADS), 0, (hipStream_t)stream, b);
    return (int)hipGetLastError();
}

}  // namespace msft
