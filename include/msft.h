/*
 * msft.h -- C ABI of the MI355X (gfx950) Multi-Slice Fourier Transform library.
 *
 * The library computes the wide-angle coherent diffraction pattern of a voxel
 * map of the complex refractive index n = 1 - delta + i beta (Eq. (7) of "The
 * Scatman", arXiv 2202.03411) on a flat N x N detector:
 *
 *   T_s  = exp(-k0 dz sum_{s'<s} (beta_s' + i delta_s'))      incident field ratio, Eq. (8)
 *   w    = dV (n^2 - 1) T                                      effective strength, Eqs. (6), (9)
 *   A_p  = sum_{x,y,z} w(x,y,z) exp(-i q_p . r)                 Eq. (9), all slices summed
 *   I_p  = |A_p|^2                                             Sec. 2, measured intensity
 *
 * with k0 = 2 pi / lambda and q_p = k0 (khat_p - zhat) the transfer momentum of
 * pixel p on the Ewald sphere (Eq. (3)).  The paper writes the kernel as
 * exp(+i q . r) with q = k_in - k_out (Fig. 3); that is the same number, since the
 * exported q here is k_out - k_in.
 *
 * Conventions shared by every call:
 *  - Lengths share one arbitrary unit (Sec. 5.1); wavelength, pitches and
 *    q (inverse length) are double precision.
 *  - Voxel arrays are float32 [nx][ny][nz] row-major, z fastest; z is the beam
 *    axis and the beam enters at iz = 0.  Voxel centres are
 *    x_a = (2a + 1 - nx) dx / 2 (likewise y, z): the grid is centred on the origin.
 *  - Detector: a flat screen at unit distance, normal to the beam, N x N square
 *    pixels of equal size; tan(theta_max) is the outer edge of the edge pixel,
 *    so pixel centres are u_i = (2i + 1 - N) tan(theta_max) / N (same for v_j) and
 *    corner pixels see angles beyond theta_max.  Pixel p = j * N + i, i along x.
 *  - Output arrays: intensity float32 [P]; amplitude complex64 [P] as
 *    interleaved (re, im) float pairs.  P = N * N, or the length of an explicit
 *    q list.
 *  - Every device pointer is owned by the caller; the library never frees one.
 *    A plan owns its own device tables and frees them in msft_plan_destroy.
 *  - Calls taking a stream are asynchronous on it (a hipStream_t passed as
 *    void*, NULL = the null stream).  Argument errors are returned
 *    synchronously and nothing is launched; device faults surface at the next
 *    synchronising call.  No C++ exception crosses this interface.
 *  - A plan is immutable after creation and may be used from several streams.
 *    Calls that share a workspace must not overlap.
 */
#ifndef MSFT_H
#define MSFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSFT_OK = 0,
    MSFT_ERR_INVALID = 1,       /* bad argument, geometry or handle */
    MSFT_ERR_UNDERSAMPLED = 2,  /* pitch * max|q| > pi on some axis (see MSFT_ALLOW_ALIAS) */
    MSFT_ERR_NOMEM = 3,         /* device or host allocation failed */
    MSFT_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    MSFT_ERR_BUSY = 5,          /* workspace too small for the call */
    MSFT_ERR_UNSUPPORTED = 6    /* the plan cannot run this call (host-only plan, ...) */
} msft_status;

/* Arithmetic of the x-sum contraction (the dominant step). */
typedef enum {
    MSFT_FP32 = 0,   /* FP32 MFMA, FP32 accumulation; the complex x-sum as three real
                        products (Gauss), P1 = Tr Wr, P2 = Ti Wi, P3 = (Tr+Ti)(Wr+Wi) */
    MSFT_BF16X3 = 1, /* BF16 hi+lo split, hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation */
    MSFT_BF16 = 2    /* plain BF16 operands (hi*hi only), FP32 accumulation: the unsplit
                        reference point, about 1e-3 relative intensity error */
} msft_precision;

/* How the two voxel arrays become the effective strength w. */
typedef enum {
    MSFT_STRENGTH_MSFT = 0,    /* w = dV (n^2 - 1) T, T from the column scan: Eqs. (6)-(9) */
    MSFT_STRENGTH_BORN = 1,    /* w = dV (n^2 - 1), incident field undisturbed: Eq. (1) with (5) */
    MSFT_STRENGTH_DENSITY = 2  /* w = dV (delta + i beta): the two arrays are the real and
                                  imaginary parts of a scattering density rho, Eq. (1) */
} msft_strength;

/* geometry flags */
#define MSFT_ALLOW_ALIAS 1u /* accept grids whose pitch exceeds pi / max|q| on some axis */

/*
 * MSFT_DETECTOR_UNIFORM_Q: instead of the flat screen, the virtual detector of the
 * paper's slice-transform algorithm (Sec. 3, Blocks 3 and 6-7): pixels on a uniform
 * grid of transverse momentum, q_x(i) = (2i + 1 - N) q_max / N and q_y(j) likewise,
 * with q_max = k0 sin(theta_max) (the outer edge of the edge pixel along each axis
 * is at theta_max), and q_z = sqrt(k0^2 - q_x^2 - q_y^2) - k0 on the Ewald sphere.
 * A pixel with q_x^2 + q_y^2 >= k0^2 (a corner beyond the sphere's rim when
 * sin(theta_max) > 1/sqrt(2)) receives no propagating wave: its intensity and
 * amplitude are written as 0 and msft_plan_qmap reports its q_z as NaN.
 * Because q_x depends on i alone and q_y on j alone, msft_simulate runs the
 * separable form: H(i, y, z) = sum_x exp(-i q_x(i) x) w for every column i (one
 * contraction of N x nx by nx x ny nz), then for every pixel
 * A = sum_z exp(-i q_z z) sum_y exp(-i q_y(j) y) H(i, y, z) (a contraction over y
 * with the z phase behind it): about N (nx + N) ny nz complex products instead of
 * N^2 nx ny nz.  Same pixel order p = j * N + i and the same sum as the flat form
 * for these q.  Not accepted by msft_plan_qlist or msft_simulate_batch.
 * msft_backward runs the same two contractions transposed: with h = g conj(A),
 * K(i, y, z) = sum_j exp(-i q_y(j) y) h(i, j) exp(-i q_z(i, j) z), then
 * R = sum_i exp(-i q_x(i) x) K, then the column walk of the general adjoint.
 */
#define MSFT_DETECTOR_UNIFORM_Q 2u

/*
 * Experiment and target description (Sec. 3, Blocks 1 and 2): wavelength,
 * maximal scattering angle and detector resolution; voxel counts and pitch.
 * struct_size must be sizeof(msft_geometry).
 */
typedef struct {
    uint32_t struct_size;
    double wavelength;     /* lambda > 0 */
    double theta_max_deg;  /* 0 < theta_max < 90: tan(theta_max) = detector half-width */
    int32_t det_n;         /* N >= 1 (ignored by msft_plan_qlist) */
    int32_t nx, ny, nz;    /* voxel counts >= 1 */
    double dx, dy, dz;     /* voxel pitch > 0 */
    int32_t precision;     /* msft_precision */
    int32_t strength;      /* msft_strength */
    uint32_t flags;        /* MSFT_ALLOW_ALIAS | MSFT_DETECTOR_UNIFORM_Q */
} msft_geometry;

typedef struct msft_plan_s* msft_plan_t;

/*
 * Build a plan: validate the geometry, compute the FP64 pixel -> q table on the
 * host (Eq. (3) on the flat detector; bit-reproducible, no FMA contraction),
 * check sampling (pitch * max|q| <= pi per axis, the discrete form of the
 * condition dz << pi / q_z under Eq. (2)), and, for device >= 0, generate the
 * resident twiddle tables exp(-i q_x x), exp(-i q_y y), exp(-i q_z z) on that
 * device from FP64 phase arguments.  device < 0 builds a host-only plan that
 * answers the query calls but cannot simulate.  On success *out receives the
 * handle; on failure *out is NULL.  Synchronous.
 */
msft_status msft_plan(const msft_geometry* g, int device, msft_plan_t* out);

/*
 * As msft_plan, but for an explicit list of npix transfer momenta q_host[npix][3]
 * (host memory, copied) instead of a detector; g->det_n and g->theta_max_deg
 * are ignored.  Used for the small-angle (uniform-q) limit and other detectors.
 */
msft_status msft_plan_qlist(const msft_geometry* g, const double* q_host, int64_t npix,
                            int device, msft_plan_t* out);

/* Free a plan and its device tables (NULL is accepted).  Synchronises the device. */
msft_status msft_plan_destroy(msft_plan_t plan);

/*
 * Sizes of a plan (the HBM footprint a scheduler admits requests by):
 *   npix              P, the number of pixels (or q values);
 *   workspace_bytes   device scratch that one msft_simulate or msft_backward call
 *                     of this plan needs (the larger of the two: the effective
 *                     strength w in the contraction's tile layout, plus the
 *                     backward's partial sums);
 *   resident_bytes    device memory the plan itself holds (q map, twiddles);
 *   per_request_bytes device memory one request of this plan holds while it is
 *                     in flight: its delta and beta (8 bytes per voxel), its
 *                     intensity and amplitude (12 bytes per pixel) and its share
 *                     of a msft_simulate_batch workspace (the forward's scratch),
 *                     each rounded up to 256 bytes.
 * Any output pointer may be NULL.
 */
msft_status msft_plan_query(msft_plan_t plan, int64_t* npix, size_t* workspace_bytes,
                            size_t* resident_bytes, size_t* per_request_bytes);

/* Copy the plan's FP64 transfer momenta, q_host[P][3] as (qx, qy, qz). */
msft_status msft_plan_qmap(msft_plan_t plan, double* q_host);

/* Copy the voxel centre coordinates: x[nx], y[ny], z[nz] (host memory). */
msft_status msft_plan_grid(msft_plan_t plan, double* x, double* y, double* z);

/*
 * Forward model for one target (Eq. (9), Sec. 3 Blocks 5-11): column scan of
 * the incident field and strength, the x-sum as a contraction on the matrix
 * cores, the y/z phase-weighted reduction and |A|^2.
 *   delta, beta : device float32 [nx][ny][nz]
 *   intensity   : device float32 [P] (written)
 *   amplitude   : device complex64 [P] or NULL (written if given)
 *   workspace   : device buffer of ws_bytes bytes, 256-byte aligned; ws_bytes
 *                 must be at least msft_plan_query's workspace_bytes
 *                 (MSFT_ERR_BUSY otherwise, nothing launched)
 * Results do not depend on the stream, the batch a call is part of, or on
 * earlier calls: the order of every floating-point sum is fixed by the plan.
 */
msft_status msft_simulate(msft_plan_t plan, const float* delta, const float* beta,
                          float* intensity, float* amplitude, void* workspace, size_t ws_bytes,
                          void* stream);

/*
 * The two stages of msft_simulate, for callers that time or reuse them:
 * msft_simulate_scan runs the column scan (Eq. (8)) and writes the effective
 * strength w into the workspace in the contraction's tile layout;
 * msft_simulate_contract then sums it against the plan's twiddles (Eq. (9)) and writes
 * intensity (and amplitude if non-NULL).  msft_simulate_scan followed by
 * msft_simulate_contract on one stream and one workspace equals msft_simulate bit for bit.
 */
msft_status msft_simulate_scan(msft_plan_t plan, const float* delta, const float* beta,
                               void* workspace, size_t ws_bytes, void* stream);
msft_status msft_simulate_contract(msft_plan_t plan, const void* workspace, size_t ws_bytes,
                                   float* intensity, float* amplitude, void* stream);

/* One request of a batch; tile_begin/tile_end select pixel blocks (-1 = all). */
typedef struct {
    msft_plan_t plan;
    const float* delta;
    const float* beta;
    float* intensity;
    float* amplitude;   /* may be NULL */
    int32_t tile_begin; /* first pixel block (blocks of msft_pixel_block() pixels) */
    int32_t tile_end;   /* one past the last block, -1 = to the end */
} msft_request;

/* Number of pixels one work item (pixel block) of a batch covers. */
int32_t msft_pixel_block(void);

/* Device workspace bytes msft_simulate_batch needs for these requests. */
msft_status msft_batch_query(const msft_request* reqs, int32_t n, size_t* workspace_bytes);

/*
 * Forward model for n requests of possibly different plans (same precision)
 * in one launch per 24 requests: every request's pixel blocks become
 * workgroups, numbered most expensive first so that the device dispatches them
 * in that order.  Each pixel written is bit-identical to what msft_simulate
 * writes for that request alone.
 * Returns MSFT_ERR_BUSY if ws_bytes is smaller than msft_batch_query reports,
 * and MSFT_ERR_UNSUPPORTED for a plan of the uniform-q detector.
 */
msft_status msft_simulate_batch(const msft_request* reqs, int32_t n, void* workspace,
                                size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): msft_simulate with its
 * workspace in a fixed array of MSFT_NOALLOC_MAX_BYTES that the library keeps on
 * each device it runs on, from the first call on that device until the process
 * ends.  Same arguments, kernels and results (bit for bit) as msft_simulate
 * without the workspace; the caller still owns delta, beta, intensity and
 * amplitude.  The call itself allocates nothing.  Every call on one device
 * shares that device's array: calls that overlap on one device (on different
 * streams, or from different threads) race and must not be issued.  A plan
 * whose workspace_bytes-sized forward scratch exceeds MSFT_NOALLOC_MAX_BYTES is
 * refused with MSFT_ERR_UNSUPPORTED (for example 192^3 voxels in FP32); nothing is
 * launched then.
 */
#define MSFT_NOALLOC_MAX_BYTES (64u << 20)
msft_status msft_simulate_noalloc(msft_plan_t plan, const float* delta, const float* beta,
                                  float* intensity, float* amplitude, void* stream);

/*
 * Adjoint of the forward model: given the amplitudes A saved by msft_simulate
 * and g = dL/dI for a real loss L, write dL/d delta and dL/d beta (device
 * float32 [nx][ny][nz]).  With R_v = sum_p g_p conj(A_p) exp(-i q_p . r_v) the
 * chain rule through Eqs. (7)-(9) gives, along each column,
 *   dL/d delta_s = 2 Re(R_s dw_s/d delta_s) + 2 k0 dz Im(sum_{s'>s} R_s' w_s')
 *   dL/d beta_s  = 2 Re(R_s dw_s/d beta_s)  - 2 k0 dz Re(sum_{s'>s} R_s' w_s')
 * (second terms only for MSFT_STRENGTH_MSFT).  The twiddles are recomputed
 * on the fly, not read from the plan.  workspace: as for msft_simulate
 * (ws_bytes at least msft_plan_query's workspace_bytes).
 */
msft_status msft_backward(msft_plan_t plan, const float* delta, const float* beta,
                          const float* amplitude, const float* grad_intensity,
                          float* grad_delta, float* grad_beta, void* workspace, size_t ws_bytes,
                          void* stream);

/*
 * Shape rendering (Sec. 5.2): delta and beta of a sample on a voxel grid centred
 * on the origin (the grid of msft_geometry), produced on the device ahead of
 * msft_simulate.  For a voxel centre at distance r from the origin, with r_s the
 * body's surface radius along the centre's direction (+z at the origin), the
 * occupancy is o = 1 if r <= r_s else 0 (edge = 0), or the soft form
 * o = 1 / (1 + exp(-(r_s - r) / edge)) (edge > 0, a width in the grid's length
 * unit); then delta = delta0 o and beta = beta0 o.  struct_size must be
 * sizeof(msft_shape_grid).
 */
typedef struct {
    uint32_t struct_size;
    int32_t nx, ny, nz;     /* voxel counts >= 1 */
    double dx, dy, dz;      /* pitch > 0 */
    double edge;            /* >= 0 */
    double delta0, beta0;   /* optical constants inside the body */
} msft_shape_grid;

/*
 * Star body r_s(theta, phi) = r0 (1 + sum_{l <= lmax, |m| <= l} c_lm Y_lm(theta, phi))
 * with real orthonormal harmonics, theta polar from +z, m > 0 carrying cos(m phi) and
 * m < 0 sin(|m| phi), no Condon-Shortley sign (the reading of the paper's complex
 * harmonics for a real radius).  coeffs: device float32 [(lmax + 1)^2], c_lm at
 * l*l + l + m, 0 <= lmax <= 12.  delta, beta: device float32 [nx][ny][nz] (written).
 */
msft_status msft_render_sh(const msft_shape_grid* g, int32_t lmax, double r0, const float* coeffs,
                           float* delta, float* beta, void* stream);

/* Device workspace bytes msft_render_sh_backward needs (independent of the grid). */
msft_status msft_render_sh_query(int32_t lmax, size_t* workspace_bytes);

/*
 * Gradient of a loss through the soft star body (edge > 0): given dL/d delta and
 * dL/d beta (device float32 [nx][ny][nz]), write
 *   dL/dc_lm = sum_v (dL/d delta_v delta0 + dL/d beta_v beta0) o_v (1 - o_v) / edge r0 Y_lm
 * into grad_coeffs (device float32 [(lmax + 1)^2]).  Partial sums per workgroup are
 * added in a fixed order: the result does not depend on the launch.
 */
msft_status msft_render_sh_backward(const msft_shape_grid* g, int32_t lmax, double r0,
                                    const float* coeffs, const float* grad_delta,
                                    const float* grad_beta, float* grad_coeffs, void* workspace,
                                    size_t ws_bytes, void* stream);

/*
 * Ellipsoid with semi-axes axes[3] (host, > 0) along the columns of the rotation
 * rot[9] (host, row-major, orthonormal): body coordinates p = rot^T r, inside iff
 * sum (p_k / a_k)^2 <= 1; the soft form uses r_s = 1 / sqrt(sum (u_k / a_k)^2) for
 * the unit direction u = rot^T r / r.
 */
msft_status msft_render_ellipsoid(const msft_shape_grid* g, const double* axes, const double* rot,
                                  float* delta, float* beta, void* stream);

/*
 * Ideal detector (Sec. 5.2, the second example's detector that adds the photon
 * statistics of a real recording).  From the intensity I = |A|^2 of a flat-detector
 * plan (msft_simulate's output, [N][N]) it writes one recording: counts[p] is a
 * Poisson draw of mean
 *     mu_p = photon_density * (k0^2 / (4 pi))^2 * I_p * dOmega_p,
 * the scalar first-Born cross section of the volume sum A times the incident
 * fluence photon_density (photons per unit area, the plan's length unit) and the
 * exact solid angle dOmega_p of the pixel's square on the screen at unit distance.
 * The paper leaves this scaling to its supplemental material; the form above is
 * the library's reading.  The draws come from Philox4x64-10 keyed by (seed, 0),
 * block m of pixel p at counter (m, p, 0, 0), so a recording depends only on
 * (intensity, photon_density, seed) and is the same for any launch order.  Counts
 * are whole numbers stored as float32 (exact below 2^24); pixels whose mean is not
 * a positive finite number record 0.  expected (may be NULL) receives mu_p.
 * Errors: MSFT_ERR_INVALID for a q-list or uniform-q plan, NULL intensity/counts,
 * or a negative or non-finite photon_density.  Asynchronous on stream.
 */
msft_status msft_detect_ideal(msft_plan_t plan, const float* intensity, double photon_density,
                              uint64_t seed, float* counts, float* expected, void* stream);

/*
 * Volume map (Sec. 5.2: an arbitrary voxel representation of the refractive
 * index): delta and beta given on a source grid of sx x sy x sz voxels of pitch
 * (sdx, sdy, sdz), also centred on the origin, resampled at the centres of g by
 * trilinear interpolation between source voxel centres, with zero beyond the
 * source grid (values fall to zero over one source pitch past its outer centres).
 * g->edge, g->delta0 and g->beta0 are not used.  src_delta, src_beta: device
 * float32 [sx][sy][sz]; delta, beta: device float32 [nx][ny][nz] (written).
 */
msft_status msft_render_volume(const msft_shape_grid* g, int32_t sx, int32_t sy, int32_t sz,
                               double sdx, double sdy, double sdz, const float* src_delta,
                               const float* src_beta, float* delta, float* beta, void* stream);

/*
 * Machine peaks for the roofline fractions of the measured contractions (the
 * performance figures of Sec. 6): what this device sustains on pure matrix-core
 * work and on a streaming copy, beside the vendor's published peaks.
 *
 * msft_peak_mfma: nblocks workgroups of 256 threads; every wave runs `iters`
 *   rounds of four independent accumulator chains of v_mfma_f32_32x32x2_f32
 *   (precision MSFT_FP32) or v_mfma_f32_32x32x16_bf16 (MSFT_BF16X3) on register
 *   operands, then stores one float per thread into sink (device, nblocks * 256
 *   floats, written) so that no work is elided.  *flops (host) receives the real
 *   flops of the launch.  Errors: MSFT_ERR_INVALID for another precision,
 *   iters < 1, nblocks < 1, NULL sink or flops.
 * msft_copy: dst[i] = src[i] over `bytes` bytes in 16-byte pieces (device
 *   pointers, 16-byte aligned; bytes a multiple of 16); the buffers must not
 *   overlap.  Errors: MSFT_ERR_INVALID for NULL pointers, misalignment or a byte
 *   count that is not a multiple of 16.
 * Both run asynchronously on stream on the current device.
 */
msft_status msft_peak_mfma(int32_t precision, int32_t iters, int32_t nblocks, float* sink, double* flops,
                           void* stream);
msft_status msft_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Static description of a status code. */
const char* msft_status_str(msft_status s);

/* Detail of the last error returned on the calling thread ("" if none). */
const char* msft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSFT_H */
