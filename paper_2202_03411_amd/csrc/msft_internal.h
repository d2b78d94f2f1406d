// Internal declarations of the MSFT library: data layouts shared by the host
// plan code and the gfx950 kernels.  Nothing here is part of the C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "msft.h"

namespace msft {

// ---------------------------------------------------------------------------
// Contraction tiling.
//
// The x-sum C[p, (y, z)] = sum_x Tx[p, x] W[x, (y, z)] runs on
// v_mfma_f32_32x32x2_f32 (FP32) or v_mfma_f32_32x32x16_bf16 (BF16X3) with the
// complex product made real: rows are (pixel, re|im) pairs, the K dimension is
// (re|im of W, x).  A wave owns WAVE_PIX pixels (32 real rows) and keeps their
// Tx operand for one x chunk in registers; a workgroup of WAVES waves shares
// every W tile through LDS.  One W tile holds XC x values and ZB z values at a
// fixed y: 64 rows (component h, z) of 256 bytes.
// ---------------------------------------------------------------------------
constexpr int XC = 64;                      // x values per contraction chunk
constexpr int ZB = 32;                      // z values per tile (MFMA columns)
constexpr int XPAD = 8;                     // nx is padded (with zeros) to a multiple of this
constexpr int WAVE_PIX = 16;                // pixels per wave
constexpr int WAVES = 8;                    // waves per workgroup
constexpr int BLOCK_PIX = WAVE_PIX * WAVES; // pixels per workgroup = one work item
constexpr int TILE_BYTES = 16384;           // one W tile, one A-operand tile
constexpr int ROW_BYTES = 256;              // one (h, z) row of a W tile
constexpr int64_t CHIP_CUS = 256;           // compute units of one MI355X (8 XCDs x 32)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Gauss (3M) form of the FP32 contraction (flat detector and q lists).  The
// complex product T W is formed from three real products,
//   P1 = Tr Wr,  P2 = Ti Wi,  P3 = (Tr + Ti)(Wr + Wi),
//   Re = P1 - P2,  Im = P3 - P1 - P2,
// each a real MFMA contraction over x with pixels as rows and z as columns, so
// the matrix cores do 6 real flops per complex multiply-add instead of 8.  A wave
// owns G3_WAVE_PIX pixels (the 32 MFMA rows); G3_WAVES waves make one BLOCK_PIX
// pixel block, and two such workgroups share a CU.  A W tile (G3_XC x, ZB z, one
// y) holds the three planes Wr, Wi, Wr + Wi as rows (plane, x parity h, z) of 16
// floats; an A tile (one wave, one x chunk) holds Tr, Ti, Tr + Ti in MFMA
// register order.
// ---------------------------------------------------------------------------
constexpr int G3_XC = 32;
constexpr int G3_WAVE_PIX = 32;
constexpr int G3_WAVES = 4;
constexpr int G3_ROW_BYTES = G3_XC / 2 * 4;                 // 64
constexpr int G3_TILE_BYTES = 3 * 2 * ZB * G3_ROW_BYTES;    // 12 KB: W tile or A tile
// The 16-byte slot swizzle of a Gauss tile row (plane, h, z): logical slot g sits at
// g ^ g3_swizzle(z).  The LDS serves a 16-byte read in groups of 16 lanes over 64
// banks; lanes reading one logical slot of 16 consecutive rows z then hit 16
// distinct 4-bank groups: 4 (z % 4) + (g ^ (z / 4) % 4).
constexpr int g3_swizzle(int z) { return (z >> 2) & 3; }
static_assert(G3_WAVE_PIX * G3_WAVES == BLOCK_PIX, "a Gauss block is one pixel block");

// Host geometry (FP64, built without FMA contraction).
struct Geometry {
    msft_geometry g;
    int64_t npix = 0;
    std::vector<double> q;         // [npix][3]
    std::vector<double> xs, ys, zs;
};

// Validate g (ignoring det_n/theta when qlist is true); message on failure.
msft_status validate_geometry(const msft_geometry* g, bool qlist, std::string* why);
// Pixel -> q of the flat detector, p = j * N + i.
void detector_qmap(double wavelength, double theta_max_deg, int32_t n, double* q);
// Pixel -> q of the uniform transverse-q detector, p = j * N + i; q_z is NaN for a
// pixel beyond the Ewald sphere's rim (q_x^2 + q_y^2 >= k0^2).  qx[N], qy[N] get
// the per-column and per-row components.
void uniform_qmap(double wavelength, double theta_max_deg, int32_t n, double* q, double* qx,
                  double* qy);
// Voxel centres (2a + 1 - n) d / 2.
void voxel_centres(int32_t n, double d, double* c);
// max_p |q_axis| * pitch over the three axes; returns false (and the axis) if > pi.
bool sampling_ok(const Geometry& geo, int* bad_axis, double* worst);

// Device-side sizes of a plan.
struct Dims {
    int64_t npix, nblocks, nwt;   // pixels, workgroup blocks, wave tiles
    int nx, ny, nz, x_pad, nxc, nzb;
    bool g3 = false;              // Gauss (3M) tiles: FP32 flat detector and q lists
    int nxc3 = 0;                 // x chunks of G3_XC
    int64_t ntiles() const { return (int64_t)(g3 ? nxc3 : nxc) * nzb * ny; }
    size_t wtile_bytes() const { return (size_t)ntiles() * (g3 ? G3_TILE_BYTES : TILE_BYTES); }
    size_t txa_bytes() const
    {
        return g3 ? (size_t)nblocks * G3_WAVES * nxc3 * G3_TILE_BYTES : (size_t)nwt * nxc * TILE_BYTES;
    }
    // (the same sizes in the Gauss layout: [wave][y][h][16] and [wave][zb][h][z][16])
    size_t ty_bytes() const { return (size_t)nwt * ny * WAVE_PIX * 8; }
    size_t tz_bytes() const { return (size_t)nwt * nzb * 2 * ZB * 8 * 8; }
};
Dims make_dims(int64_t npix, int nx, int ny, int nz);

// Arguments of the forward contraction for one plan/target.
struct FwdArgs {
    const uint8_t* wtiles;  // effective strength, tile t = (xc * nzb + zb) * ny + y
    const uint8_t* txa;     // A operand tiles [wt][xc]
    const float* ty;        // [wt][y][h][8] complex
    const float* tz;        // [wt][zb][h][32][8] complex
    float* intensity;       // [npix]
    float* amplitude;       // [npix] complex or null
    int64_t npix;
    int32_t ny, nxc, nzb, x_pad;
    // Second stage of the separable detector (all zero otherwise): column i
    // reads its tile group at wtiles + i * group_tiles tiles; its rows j form
    // group_blocks pixel blocks; kernel pixel i * out_npad + j is written to
    // j * out_n + i when j < out_n.
    int32_t group_blocks, group_tiles, out_n, out_npad;
};

// Gauss form of the separable detector (FP32): the second stage keeps its A
// operand for at most SG2_MAXYC chunks of 32 y in registers; one (row tile of 16
// j, y chunk) of it is SG2_A_BYTES.
constexpr int SG2_MAXYC = 4;
constexpr int SG2_A_BYTES = 3 * 2 * 64 * 16;

// Separable (uniform transverse q) detector: q_x depends on the column i only,
// q_y on the row j only.  Stage 1 forms H = Tx W per column (N x ny x nz); stage 2
// contracts H over y against Ty per row with the z phase behind it.
struct SepDims {
    int32_t n = 0;      // detector side N
    int32_t npad = 0;   // N rounded up to BLOCK_PIX: rows j per column in stage 2
    int64_t nblk1 = 0;  // stage-1 blocks of BLOCK_PIX columns
    int32_t nyc = 0;    // y chunks of 64 in stage 2
    int32_t y_pad = 0;  // ny padded to XPAD
    size_t txa1_bytes(int nxc) const { return (size_t)nblk1 * WAVES * nxc * TILE_BYTES; }
    size_t txa2_bytes() const { return (size_t)(npad / WAVE_PIX) * nyc * TILE_BYTES; }
    size_t h_bytes(int nzb) const { return (size_t)n * nyc * nzb * TILE_BYTES; }
    size_t tz_bytes(int nzb) const { return (size_t)n * (npad / WAVE_PIX) * nzb * 2 * ZB * 8 * 8; }
    // Adjoint: K(i, y, z) = sum_j Ty(j, y) h(i, j) Tz(i, j, z) in tiles (i chunk, z block, y)
    // of 64 i x 32 z, then R = sum_i Tx(i, x) K(i, y, z).
    int32_t njc = 0;    // chunks of 64 rows j (npad / 64)
    int32_t nic = 0;    // chunks of 64 columns i
    size_t tyT_bytes(int ny) const { return (size_t)ceil_div(ny, BLOCK_PIX) * WAVES * njc * TILE_BYTES; }
    size_t txT_bytes(int nx) const { return (size_t)ceil_div(nx, BLOCK_PIX) * WAVES * nic * TILE_BYTES; }
    size_t k_bytes(int ny, int nzb) const { return (size_t)nic * nzb * ny * TILE_BYTES; }
    // FP32 with ny <= SG2_MAXYC * 32: the Gauss (three-product) form of both stages.
    // H tiles [i][y chunk of 32][z block] of G3_TILE_BYTES; A operands of stage 1
    // [16 columns i][x chunk of 32], of stage 2 [16 rows j][y chunk].
    bool gauss = false;
    int32_t nyc2 = 0;   // y chunks of 32
    size_t hg_bytes(int nzb) const { return (size_t)n * nyc2 * nzb * G3_TILE_BYTES; }
    size_t txa1g_bytes(int nxc3) const { return (size_t)ceil_div(n, 64) * 4 * nxc3 * SG2_A_BYTES; }
    size_t txa2g_bytes() const { return (size_t)(npad / WAVE_PIX) * nyc2 * SG2_A_BYTES; }
    // ... and of its adjoint: chunks of 32 columns i (and of 32 rows j), K in three
    // planes [i][y][z], A tables of the two passes.
    int32_t nic3 = 0;
    size_t kg_bytes(int ny, int nzb) const { return (size_t)2 * nic3 * 32 * ny * nzb * ZB * 4; }
    size_t tyTg_bytes(int ny) const { return (size_t)ceil_div(ny, 64) * 4 * nic3 * SG2_A_BYTES; }
    size_t txTg_bytes(int nx) const { return (size_t)ceil_div(nx, 128) * 4 * nic3 * G3_TILE_BYTES; }
};
SepDims make_sep_dims(int32_t n, int ny);

// Stage 1 of the separable detector (TILE output: H tiles), and the adjoint's
// contraction over the columns i (PLAIN output: R[row][y][z] complex).
struct Stage1Args {
    const uint8_t* wtiles;  // B tiles, index (xc * nzb + zb) * ny + y
    const uint8_t* txa;     // A tiles [row wave][xc]
    uint8_t* htiles;        // TILE: H tiles [i][y chunk][z block]
    float* rplain;          // PLAIN: [row][ny][nz2] complex
    int32_t n, ny, nxc, nzb, x_pad, nyc, nz2;
};

// Both stages of the separable detector in the Gauss form (see SepDims).
struct SepG3Args {
    const uint8_t* wtiles;  // W tiles in the G3 layout, index (xc * nzb + zb) * ny + y
    const uint8_t* txa1;    // stage 1 A tiles [wave of 32 columns][xc]
    uint8_t* htiles;        // H tiles [i][yc][zb]
    const uint8_t* txa2;    // stage 2 A tables [16 rows j][yc]
    const float* tz;        // the plan's Tz over stage 2's pixel order (16-row tiles)
    float* intensity;       // [N * N], pixel j * N + i
    float* amplitude;       // [N * N] complex or null
    int32_t n, npad, ny, nxc3, nyc2, nzb;
    int64_t nblk1;
};

// The Gauss form's adjoint (see SepDims): pass 2 splits its sum over the columns
// i in SEPG_ADJ_SPLIT partial sums.
constexpr int SEPG_ADJ_SPLIT = 2;
struct SepG3AdjArgs {
    const float* h;         // [N * N] complex, h_p = g_p conj(A_p), p = j * N + i
    const float* tz;        // the plan's Tz over stage 2's pixel order (16-row tiles)
    const uint8_t* tyT;     // pass 1 A tables [16 rows y][j chunk of 32]
    const uint8_t* txT;     // pass 2 A tiles [32 rows x][i chunk of 32]
    float* kplain;          // K in two planes Kr, Ki of [nic3 * 32][ny][nz2] floats
    float* rpart;           // [SEPG_ADJ_SPLIT][rows_pad][ny][nz2] complex
    int32_t n, npad, nx, ny, nzb, nz2, njc2, nic3, rows_pad;
};

// The adjoint's contraction over the detector rows j (see SepDims).
struct SepAdjArgs {
    const float* h;        // [N * N] complex, h_p = g_p conj(A_p), p = j * N + i
    const float* tz;       // the plan's Tz over stage 2's pixel order
    const uint8_t* tyT;    // A tiles exp(-i q_y(j) y): [wave of 16 y][j chunk]
    uint8_t* ktiles;       // K tiles, index (i chunk * nzb + zb) * ny + y
    int32_t n, npad, ny, nzb, njc;
};

// Arguments of the column scan producing the W tiles.
struct ScanArgs {
    const float* delta;
    const float* beta;
    uint8_t* wtiles;
    int32_t nx, ny, nz, nxc, nzb;
    int32_t strength;
    int32_t g3;   // write the Gauss tile layout (FP32 only)
    int32_t nxc3; // its x chunks of G3_XC
    float k0dz;   // k0 * dz
    float dV;     // dx * dy * dz
};

// A batch launch carries every request descriptor in its kernel arguments
// (no host -> device copy): request r owns work items [item_begin[r],
// item_begin[r + 1]), item k of it being pixel block block_begin[r] + k.
constexpr int MAX_BATCH = 24;
struct BatchArgs {
    FwdArgs req[MAX_BATCH];
    int32_t block_begin[MAX_BATCH];
    int32_t item_begin[MAX_BATCH + 1];
    int32_t nreq;
};

// Adjoint: pixels per LDS chunk of the transposed contraction (one per 8 threads),
// and y values per workgroup (two per wave of 8).
constexpr int ADJ_CHUNK = 64;
constexpr int ADJ_Y = 16;

// Split-K layout of the adjoint: pixel group s of group_pix pixels writes its
// partial R into rpart[s][x (nxc*64)][y][z (nzb*32)] complex.
struct AdjDims {
    int64_t group_pix;
    int32_t nsplit, nyb;
    size_t h_bytes, rpart_bytes;
    size_t bytes() const { return h_bytes + rpart_bytes; }
};
AdjDims make_adj_dims(const Dims& d);

struct AdjArgs {
    const double* q;   // [npix][3]
    float* h;          // [npix_pad] complex: g_p conj(A_p)
    float* rpart;      // partial strength gradients, see AdjDims
    int64_t npix, npix_pad, group_pix;
    int32_t nx, ny, nz, nxc, nzb, nyb, nsplit;
    double xs0, ys0, zs0;  // coordinate of voxel index 0 on each axis
    double dx, dy, dz;
};

struct FinArgs {
    const float* delta;
    const float* beta;
    const float* rpart;
    float* grad_delta;
    float* grad_beta;
    int32_t nx, ny, nz, nxc, nzb, nsplit, strength;
    double dV, k0dz;
};

// Shape rendering.  Real harmonics up to MAX_SH_L; the l-recurrence constants
// Q_lm = ra (cos(theta) Q_{l-1,m} - rb Q_{l-2,m}) at [l * SH_TABLE + m], the
// diagonal Q_mm = diag[m] sin(theta) Q_{m-1,m-1}, the first step Q_{m+1,m} =
// sub[m] cos(theta) Q_mm, all made on the host in FP64.
constexpr int MAX_SH_L = 12;
constexpr int SH_TABLE = MAX_SH_L + 1;
constexpr int MAX_SH_COEFFS = SH_TABLE * SH_TABLE;
constexpr int SH_GRAD_BLOCKS = 512;   // workgroups of the coefficient gradient (its partials)

struct RenderGrid {
    int32_t nx, ny, nz;
    double dx, dy, dz, edge, delta0, beta0;
};

struct ShArgs {
    RenderGrid g;
    int32_t lmax;
    double r0;
    double diag[SH_TABLE], sub[SH_TABLE];
    double ra[SH_TABLE * SH_TABLE], rb[SH_TABLE * SH_TABLE];
};

struct VolArgs {
    RenderGrid g;
    int32_t sx, sy, sz;
    double sdx, sdy, sdz;
};

// Ideal detector on the flat N x N screen: half-width t = tan(theta_max) at unit
// distance, scale = F (k0^2 / 4 pi)^2, Philox key (seed, 0).
struct IdealArgs {
    int32_t n;
    double t;
    double scale;
    uint64_t seed;
};

struct EllArgs {
    RenderGrid g;
    double ax[3];
    double rot[9];   // row-major; its columns are the body axes
};

// Kernel launchers (defined in the .hip sources); return a HIP error code.
int launch_backward(const AdjArgs& adj, const FinArgs& fin, const float* amplitude,
                    const float* grad_intensity, void* stream);
int launch_twiddles(int precision, const Dims& d, const double* q_dev, const double* xs_dev,
                    const double* ys_dev, const double* zs_dev, uint8_t* txa, float* ty,
                    float* tz, void* stream);
int launch_scan(int precision, const ScanArgs& a, void* stream);
int launch_forward(int precision, const FwdArgs& a, int64_t block_begin, int64_t nblocks, void* stream);
// Gauss form (tables from launch_twiddles_g3, tiles from a g3 scan).
int launch_twiddles_g3(const Dims& d, const double* q_dev, const double* xs_dev, const double* ys_dev,
                       const double* zs_dev, uint8_t* txa, float* ty, float* tz, void* stream);
int launch_forward_g3(const FwdArgs& a, int64_t block_begin, int64_t nblocks, void* stream);
int launch_forward_batch_g3(const BatchArgs& b, void* stream);
int launch_sep_twiddles(int precision, const Dims& d, const SepDims& sd, const double* qcol,
                        const double* qrow, const double* qk, const double* xs, const double* ys,
                        const double* zs, uint8_t* txa1, uint8_t* txa2, float* tz, void* stream);
int launch_sep_stage1(int precision, const Stage1Args& a, int64_t nblk, void* stream);
// a: second-stage arguments (group_blocks, group_tiles, out_n, out_npad set)
int launch_sep_stage2(int precision, const FwdArgs& a, void* stream);
int launch_sepg_twiddles(const SepDims& sd, int nx, int ny, int nxc3, const double* qx,
                         const double* qy, const double* xs, const double* ys, uint8_t* txa1,
                         uint8_t* txa2, void* stream);
int launch_sepg(const SepG3Args& a, void* stream);
int launch_sepg_adj_tables(const SepDims& sd, int nx, int ny, const double* xs, const double* qx,
                           const double* ys, const double* qy, uint8_t* txT, uint8_t* tyT, void* stream);
int launch_sepg_adjoint(const SepG3AdjArgs& a, void* stream);
int launch_sep_adjoint(const SepAdjArgs& ka, const Stage1Args& ra, int64_t nblk_rows, void* stream);
int launch_sep_adj_tables(const SepDims& sd, int nx, int ny, const double* xq3, const double* qx,
                          const double* yq3, const double* qy, uint8_t* txT, uint8_t* tyT,
                          void* stream);
int launch_adj_prep(const float* amplitude, const float* grad_intensity, float* h, int64_t npix,
                    int64_t npix_pad, void* stream);
int launch_adj_finalize(const FinArgs& fin, void* stream);
int launch_render_sh(const ShArgs& s, const float* coeffs, float* delta, float* beta, void* stream);
int launch_render_sh_grad(const ShArgs& s, const float* coeffs, const float* gd, const float* gb,
                          float* grad, double* partial, int nblocks, void* stream);
int launch_render_ellipsoid(const EllArgs& e, float* delta, float* beta, void* stream);
// Machine-peak probes (peaks.hip).  flops: the real flops of the launch.
int launch_peak_mfma(int precision, int iters, int nblocks, float* sink, double* flops, void* stream);
int launch_copy(const void* src, void* dst, int64_t pieces, void* stream);
int launch_detect_ideal(const IdealArgs& a, const float* intensity, float* counts, float* expected,
                        void* stream);
int launch_render_volume(const VolArgs& a, const float* sd, const float* sb, float* delta,
                         float* beta, void* stream);
int launch_forward_batch(int precision, const BatchArgs& b, void* stream);
// Device address of the fixed scratch array on `device` (which must be current),
// looked up on the first call per device; returns a HIP error code.
int static_scratch(int device, void** ptr);

}  // namespace msft

// The plan object behind msft_plan_t.
struct msft_plan_s {
    msft::Geometry geo;
    msft::Dims dims;
    int device = -1;
    bool qlist = false;
    // resident device tables
    double* q_dev = nullptr;      // [npix][3]
    double* xs_dev = nullptr;
    double* ys_dev = nullptr;
    double* zs_dev = nullptr;
    uint8_t* txa = nullptr;       // separable detector: stage-1 A operand
    float* ty = nullptr;
    float* tz = nullptr;          // separable detector: over stage 2's pixel order
    uint8_t* txa2 = nullptr;      // separable detector: stage-2 A operand
    uint8_t* txT = nullptr;       // separable detector, adjoint: exp(-i q_x(i) x), rows x
    uint8_t* tyT = nullptr;       // separable detector, adjoint: exp(-i q_y(j) y), rows y
    bool separable = false;
    msft::SepDims sep;
    size_t resident_bytes = 0;
    size_t workspace_bytes = 0;   // max of the two below
    size_t fwd_workspace = 0;     // msft_simulate: W tiles (+ H tiles, separable detector)
    size_t adj_workspace = 0;     // msft_backward
    size_t per_request = 0;       // one request's own buffers + its share of a batch workspace
};
