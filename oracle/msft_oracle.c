/*
 * FP64 reference oracle for the Multi-Slice Fourier Transform (MSFT) forward
 * model and its gradient -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path never calls it and shares
 * no code, header or table with it.  Every routine is plain, slow, double
 * precision C written from the paper's equations (Sec. 2 of "The Scatman",
 * arXiv 2202.03411) and its shape descriptions (Sec. 5.2); OpenMP only splits
 * independent pixels or columns over threads, it does not reorder any single sum.
 *
 * Equation numbers follow the paper: (1) first Born approximation, (2) slicing
 * of the z integral, (3) Ewald-sphere q_z, (4) MSFT with the Ewald phase,
 * (5)/(6) scattering strength from n^2 - 1, (7) n = 1 - delta + i beta,
 * (8) projection-approximation propagation of the incident field,
 * (9) main Scatman equation, I = |Psi|^2.
 *
 * Readings taken where the paper is silent (all listed in the design notes):
 *  - Flat detector at unit distance, N x N pixels; tan(theta_max) is the outer
 *    edge of the edge pixel, pixel centres at u_i = (2i + 1 - N) t / N.
 *  - Exported transfer momentum q = k0 (khat_out - zhat); the amplitude is
 *    A = sum_v w_v exp(-i q . r_v), which is the paper's exp(+i q_paper . r)
 *    with q_paper = k_in - k_out (Fig. 3).
 *  - The field reaching slice s is attenuated by slices 0..s-1 only
 *    (E_{s=0} = E_0 in Eq. (9)): an exclusive prefix along +z.
 *  - Proportionality constants are dropped: w = dV (n^2 - 1) T exactly.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

enum { ORACLE_MSFT = 0, ORACLE_BORN = 1, ORACLE_DENSITY = 2 };

/* Threads an OpenMP region of the oracle uses. */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Wave number k0 = 2 pi / lambda. */
static double oracle_k0(double wavelength) { return (2.0 * ORACLE_PI) / wavelength; }

/*
 * Pixel -> transfer momentum for a flat N x N detector (Sec. 3, Block 1; the
 * Ewald relation of Eq. (3)).  Pixel p = j * N + i, i along detector x (u),
 * j along detector y (v).  Output q[p][3] = (qx, qy, qz).  The direction of a
 * pixel centre is (u, v, 1) / r with r = sqrt(u^2 + v^2 + 1); q = k0 (khat - zhat)
 * so qz = k0 (1/r - 1), evaluated in the cancellation-free form -k0 s / (r (r + 1)).
 */
void oracle_qmap(double wavelength, double theta_max_deg, int32_t n, double* q)
{
    const double k0 = oracle_k0(wavelength);
    const double t = tan((theta_max_deg * ORACLE_PI) / 180.0);
    for (int32_t j = 0; j < n; ++j) {
        const double v = ((double)(2 * j + 1 - n) * t) / (double)n;
        for (int32_t i = 0; i < n; ++i) {
            const double u = ((double)(2 * i + 1 - n) * t) / (double)n;
            const double uu = u * u;
            const double vv = v * v;
            const double s = uu + vv;
            const double r = sqrt(s + 1.0);
            double* qp = q + 3 * ((int64_t)j * n + i);
            qp[0] = (k0 * u) / r;
            qp[1] = (k0 * v) / r;
            qp[2] = -((k0 * s) / (r * (r + 1.0)));
        }
    }
}

/*
 * Pixel -> transfer momentum for the virtual detector of the slice-transform
 * algorithm (Sec. 3, Blocks 3 and 6): the discrete transform of a slice lands on
 * a uniform grid of transverse momentum, so pixel (i, j) has
 * qx = (2i + 1 - N) qmax / N, qy = (2j + 1 - N) qmax / N with qmax = k0 sin(theta_max),
 * and lies on the Ewald sphere: the outgoing wave vector is (qx, qy, kz) with
 * kz = sqrt(k0^2 - qx^2 - qy^2), so qz = kz - k0 = -s / (kz + k0), s = qx^2 + qy^2.
 * Where s >= k0^2 no outgoing wave exists and qz is NaN.  p = j * N + i.
 */
void oracle_qmap_uniform(double wavelength, double theta_max_deg, int32_t n, double* q)
{
    const double k0 = oracle_k0(wavelength);
    const double qmax = k0 * sin((theta_max_deg * ORACLE_PI) / 180.0);
    const double k2 = k0 * k0;
    for (int32_t j = 0; j < n; ++j) {
        const double qy = ((double)(2 * j + 1 - n) * qmax) / (double)n;
        for (int32_t i = 0; i < n; ++i) {
            const double qx = ((double)(2 * i + 1 - n) * qmax) / (double)n;
            const double s = qx * qx + qy * qy;
            double* qp = q + 3 * ((int64_t)j * n + i);
            qp[0] = qx;
            qp[1] = qy;
            if (s < k2) {
                const double kz = sqrt(k2 - s);
                qp[2] = -(s / (kz + k0));
            } else {
                qp[2] = NAN;
            }
        }
    }
}

/* Voxel centres of a grid of n cells with pitch d, centred on the origin. */
void oracle_grid(int32_t n, double d, double* c)
{
    for (int32_t a = 0; a < n; ++a) c[a] = ((double)(2 * a + 1 - n) * d) / 2.0;
}

/*
 * Effective scattering strength per voxel, w[(a*ny + b)*nz + c] as (re, im).
 *   MSFT    : w = dV (n^2 - 1) E_s / (E_0 e^{i k0 s dz})  -- Eqs. (6)-(9).  With
 *             Eq. (8) the ratio is prod_{s'<s} exp(-i k0 dz delta_s') exp(-k0 dz beta_s').
 *   BORN    : w = dV (n^2 - 1), incident field undisturbed (Eq. (1) with (5)).
 *   DENSITY : the two inputs are the real and imaginary parts of a scattering
 *             density rho (Eq. (1)); w = dV rho.
 * Inputs are [a][b][c] with c (z, the beam axis) fastest; the beam enters at c = 0.
 */
void oracle_strength(int32_t mode, int32_t nx, int32_t ny, int32_t nz,
                     double dx, double dy, double dz, double wavelength,
                     const double* delta, const double* beta, double* w)
{
    const double k0 = oracle_k0(wavelength);
    const double dV = dx * dy * dz;
    for (int32_t a = 0; a < nx; ++a) {
        for (int32_t b = 0; b < ny; ++b) {
            double sum_beta = 0.0, sum_delta = 0.0; /* over slices already passed */
            for (int32_t c = 0; c < nz; ++c) {
                const int64_t v = ((int64_t)a * ny + b) * nz + c;
                const double d = delta[v], bt = beta[v];
                double wr, wi;
                if (mode == ORACLE_DENSITY) {
                    wr = dV * d;
                    wi = dV * bt;
                } else {
                    /* n = 1 - delta + i beta (Eq. (7)); chi = n^2 - 1. */
                    const double nr = 1.0 - d, ni = bt;
                    const double chi_r = (nr * nr - ni * ni) - 1.0;
                    const double chi_i = 2.0 * nr * ni;
                    double tr = 1.0, ti = 0.0;
                    if (mode == ORACLE_MSFT) {
                        const double mag = exp(-k0 * dz * sum_beta);
                        const double ph = -k0 * dz * sum_delta;
                        tr = mag * cos(ph);
                        ti = mag * sin(ph);
                    }
                    wr = dV * (chi_r * tr - chi_i * ti);
                    wi = dV * (chi_r * ti + chi_i * tr);
                }
                w[2 * v] = wr;
                w[2 * v + 1] = wi;
                sum_beta += bt;
                sum_delta += d;
            }
        }
    }
}

/*
 * Scattered amplitude A_p = sum_v w_v exp(-i q_p . r_v) for an explicit list of
 * npix momenta q[p][3]; A[p] as (re, im).  This is Eq. (9) with the 2D Fourier
 * transform of every slice and the slice phase of Eq. (4) written as one sum.
 *   method 0 (direct)    : one sin/cos of the full phase per voxel-pixel term.
 *   method 1 (separable) : the same sum with exp(-i q.r) split exactly into
 *                          exp(-i qx x) exp(-i qy y) exp(-i qz z) tables, summed
 *                          z innermost, then y, then x.
 */
void oracle_amplitude(int32_t method, const double* q, int64_t npix,
                      int32_t nx, int32_t ny, int32_t nz,
                      double dx, double dy, double dz, const double* w, double* A)
{
    double* xs = (double*)malloc(sizeof(double) * (size_t)nx);
    double* ys = (double*)malloc(sizeof(double) * (size_t)ny);
    double* zs = (double*)malloc(sizeof(double) * (size_t)nz);
    oracle_grid(nx, dx, xs);
    oracle_grid(ny, dy, ys);
    oracle_grid(nz, dz, zs);

    #pragma omp parallel
    {
        double* ex = (double*)malloc(sizeof(double) * 2 * (size_t)nx);
        double* ey = (double*)malloc(sizeof(double) * 2 * (size_t)ny);
        double* ez = (double*)malloc(sizeof(double) * 2 * (size_t)nz);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p) {
            const double qx = q[3 * p], qy = q[3 * p + 1], qz = q[3 * p + 2];
            double ar = 0.0, ai = 0.0;
            if (method == 0) {
                for (int32_t a = 0; a < nx; ++a)
                    for (int32_t b = 0; b < ny; ++b)
                        for (int32_t c = 0; c < nz; ++c) {
                            const int64_t v = ((int64_t)a * ny + b) * nz + c;
                            const double ph = -(qx * xs[a] + qy * ys[b] + qz * zs[c]);
                            const double kr = cos(ph), ki = sin(ph);
                            ar += w[2 * v] * kr - w[2 * v + 1] * ki;
                            ai += w[2 * v] * ki + w[2 * v + 1] * kr;
                        }
            } else {
                for (int32_t a = 0; a < nx; ++a) { ex[2 * a] = cos(-qx * xs[a]); ex[2 * a + 1] = sin(-qx * xs[a]); }
                for (int32_t b = 0; b < ny; ++b) { ey[2 * b] = cos(-qy * ys[b]); ey[2 * b + 1] = sin(-qy * ys[b]); }
                for (int32_t c = 0; c < nz; ++c) { ez[2 * c] = cos(-qz * zs[c]); ez[2 * c + 1] = sin(-qz * zs[c]); }
                for (int32_t a = 0; a < nx; ++a) {
                    double sxr = 0.0, sxi = 0.0;
                    for (int32_t b = 0; b < ny; ++b) {
                        double syr = 0.0, syi = 0.0;
                        const double* wc = w + 2 * (((int64_t)a * ny + b) * nz);
                        for (int32_t c = 0; c < nz; ++c) {
                            syr += wc[2 * c] * ez[2 * c] - wc[2 * c + 1] * ez[2 * c + 1];
                            syi += wc[2 * c] * ez[2 * c + 1] + wc[2 * c + 1] * ez[2 * c];
                        }
                        sxr += syr * ey[2 * b] - syi * ey[2 * b + 1];
                        sxi += syr * ey[2 * b + 1] + syi * ey[2 * b];
                    }
                    ar += sxr * ex[2 * a] - sxi * ex[2 * a + 1];
                    ai += sxr * ex[2 * a + 1] + sxi * ex[2 * a];
                }
            }
            A[2 * p] = ar;
            A[2 * p + 1] = ai;
        }
        free(ex);
        free(ey);
        free(ez);
    }
    free(xs);
    free(ys);
    free(zs);
}

/*
 * Gradient of a real loss L(I) with respect to the voxel delta and beta, given
 * g[p] = dL/dI_p and the amplitudes A[p] of all npix pixels.
 *
 * Since I_p = |A_p|^2 and A_p is linear in w, dL = sum_v 2 Re(R_v dw_v) with
 * R_v = sum_p g_p conj(A_p) exp(-i q_p . r_v).  The chain rule through Eq. (7)
 * and the propagation of Eq. (8) then gives, for slice s of a column,
 *   dL/d delta_s = 2 Re(R_s dV T_s dchi/ddelta) + 2 Re(-i k0 dz sum_{s'>s} R_s' w_s')
 *   dL/d beta_s  = 2 Re(R_s dV T_s dchi/dbeta)  + 2 Re(  -k0 dz sum_{s'>s} R_s' w_s')
 * with dchi/ddelta = -2 n and dchi/dbeta = 2 i n (n = 1 - delta + i beta).  The
 * second terms are absent in the BORN and DENSITY modes; DENSITY has
 * dw/ddelta = dV and dw/dbeta = i dV.
 *
 * cols[k] = a * ny + b selects the columns to differentiate (ncols of them);
 * cols == NULL means every column.  Outputs gdelta/gbeta hold [k][c] for the
 * selected columns, nz values each.
 */
void oracle_backward(int32_t mode, const double* q, int64_t npix,
                     const double* g, const double* A,
                     int32_t nx, int32_t ny, int32_t nz,
                     double dx, double dy, double dz, double wavelength,
                     const double* delta, const double* beta,
                     const int64_t* cols, int64_t ncols,
                     double* gdelta, double* gbeta)
{
    const double k0 = oracle_k0(wavelength);
    const double dV = dx * dy * dz;
    double* xs = (double*)malloc(sizeof(double) * (size_t)nx);
    double* ys = (double*)malloc(sizeof(double) * (size_t)ny);
    double* zs = (double*)malloc(sizeof(double) * (size_t)nz);
    oracle_grid(nx, dx, xs);
    oracle_grid(ny, dy, ys);
    oracle_grid(nz, dz, zs);
    const int64_t ncol_all = (int64_t)nx * ny;
    const int64_t nsel = cols ? ncols : ncol_all;

    #pragma omp parallel
    {
        double* R = (double*)malloc(sizeof(double) * 2 * (size_t)nz);
        double* T = (double*)malloc(sizeof(double) * 2 * (size_t)nz);
        double* wcol = (double*)malloc(sizeof(double) * 2 * (size_t)nz);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < nsel; ++k) {
            const int64_t col = cols ? cols[k] : k;
            const int32_t a = (int32_t)(col / ny), b = (int32_t)(col % ny);
            const double* dcol = delta + col * nz;
            const double* bcol = beta + col * nz;

            /* incident-field ratio T_s and strength w_s along the column */
            double sum_beta = 0.0, sum_delta = 0.0;
            for (int32_t c = 0; c < nz; ++c) {
                double tr = 1.0, ti = 0.0;
                if (mode == ORACLE_MSFT) {
                    const double mag = exp(-k0 * dz * sum_beta);
                    const double ph = -k0 * dz * sum_delta;
                    tr = mag * cos(ph);
                    ti = mag * sin(ph);
                }
                T[2 * c] = tr;
                T[2 * c + 1] = ti;
                const double nr = 1.0 - dcol[c], ni = bcol[c];
                const double chi_r = (nr * nr - ni * ni) - 1.0, chi_i = 2.0 * nr * ni;
                wcol[2 * c] = dV * (chi_r * tr - chi_i * ti);
                wcol[2 * c + 1] = dV * (chi_r * ti + chi_i * tr);
                sum_beta += bcol[c];
                sum_delta += dcol[c];
            }

            /* R_v = sum_p g_p conj(A_p) exp(-i q_p . r_v) */
            for (int32_t c = 0; c < nz; ++c) {
                double rr = 0.0, ri = 0.0;
                for (int64_t p = 0; p < npix; ++p) {
                    const double ph = -(q[3 * p] * xs[a] + q[3 * p + 1] * ys[b] + q[3 * p + 2] * zs[c]);
                    const double kr = cos(ph), ki = sin(ph);
                    const double hr = g[p] * A[2 * p], hi = -g[p] * A[2 * p + 1];
                    rr += hr * kr - hi * ki;
                    ri += hr * ki + hi * kr;
                }
                R[2 * c] = rr;
                R[2 * c + 1] = ri;
            }

            for (int32_t c = 0; c < nz; ++c) {
                const double rr = R[2 * c], ri = R[2 * c + 1];
                double gd, gb;
                if (mode == ORACLE_DENSITY) {
                    gd = 2.0 * (rr * dV);
                    gb = 2.0 * (-ri * dV);
                } else {
                    const double nr = 1.0 - dcol[c], ni = bcol[c];
                    /* dw/ddelta (own) = dV T (-2 n), dw/dbeta (own) = dV T (2 i n) */
                    const double tr = T[2 * c], ti = T[2 * c + 1];
                    const double dd_r = dV * (tr * (-2.0 * nr) - ti * (-2.0 * ni));
                    const double dd_i = dV * (tr * (-2.0 * ni) + ti * (-2.0 * nr));
                    const double db_r = dV * (tr * (-2.0 * ni) - ti * (2.0 * nr));
                    const double db_i = dV * (tr * (2.0 * nr) + ti * (-2.0 * ni));
                    gd = 2.0 * (rr * dd_r - ri * dd_i);
                    gb = 2.0 * (rr * db_r - ri * db_i);
                    if (mode == ORACLE_MSFT) {
                        /* later slices see this voxel through T */
                        double sr = 0.0, si = 0.0;
                        for (int32_t c2 = c + 1; c2 < nz; ++c2) {
                            sr += R[2 * c2] * wcol[2 * c2] - R[2 * c2 + 1] * wcol[2 * c2 + 1];
                            si += R[2 * c2] * wcol[2 * c2 + 1] + R[2 * c2 + 1] * wcol[2 * c2];
                        }
                        /* Re(-i k0 dz S) = k0 dz Im S ; Re(-k0 dz S) = -k0 dz Re S */
                        gd += 2.0 * (k0 * dz * si);
                        gb += 2.0 * (-k0 * dz * sr);
                    }
                }
                gdelta[k * nz + c] = gd;
                gbeta[k * nz + c] = gb;
            }
        }
        free(R);
        free(T);
        free(wcol);
    }
    free(xs);
    free(ys);
    free(zs);
}

/* ------------------------------------------------------------------------- */
/* Shape rendering (Sec. 5.2): the sample's occupancy on the voxel grid.      */
/* ------------------------------------------------------------------------- */

/*
 * Real orthonormal spherical harmonic Y_lm(cos theta, phi), theta polar from +z:
 * m > 0 carries cos(m phi), m < 0 carries sin(|m| phi), no Condon-Shortley sign
 * (the reading of the paper's complex Y for a real radius).  Built from the
 * unnormalised associated Legendre function, P_m^m = (2m-1)!! sin^m theta and the
 * upward three-term recurrence in l, times sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
 */
double oracle_ylm(int32_t l, int32_t m, double ct, double phi)
{
    const int am = m < 0 ? -m : m;
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double pmm = 1.0;
    for (int k = 1; k <= am; ++k) pmm *= (2.0 * k - 1.0) * st;
    double p = pmm;
    if (l > am) {
        double a = pmm, b = ct * (2.0 * am + 1.0) * pmm;
        for (int ll = am + 2; ll <= l; ++ll) {
            const double c = ((2.0 * ll - 1.0) * ct * b - (ll + am - 1.0) * a) / (double)(ll - am);
            a = b;
            b = c;
        }
        p = b;
    }
    double ratio = 1.0;
    for (int k = l - am + 1; k <= l + am; ++k) ratio /= (double)k;
    const double nrm = sqrt((2.0 * l + 1.0) / (4.0 * ORACLE_PI) * ratio);
    if (m == 0) return nrm * p;
    if (m > 0) return sqrt(2.0) * nrm * p * cos(m * phi);
    return sqrt(2.0) * nrm * p * sin(am * phi);
}

/* Direction of voxel centre (x, y, z): cos theta and phi; +z at the origin. */
static void oracle_direction(double x, double y, double z, double* r, double* ct, double* phi)
{
    *r = sqrt(x * x + y * y + z * z);
    if (*r > 0.0) {
        *ct = z / *r;
        *phi = atan2(y, x);
    } else {
        *ct = 1.0;
        *phi = 0.0;
    }
}

/* Radius of the star body along a direction: r0 (1 + sum_lm c_lm Y_lm), c at l*l + l + m. */
static double oracle_star_radius(int32_t lmax, const double* c, double r0, double ct, double phi)
{
    double s = 0.0;
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) s += c[l * l + l + m] * oracle_ylm(l, m, ct, phi);
    return r0 * (1.0 + s);
}

/* Occupancy of a voxel at distance r for a surface at rs: hard (edge = 0, closed) or a
   sigmoid of (rs - r) / edge. */
static double oracle_occupancy(double rs, double r, double edge)
{
    if (edge <= 0.0) return r <= rs ? 1.0 : 0.0;
    return 1.0 / (1.0 + exp(-(rs - r) / edge));
}

/*
 * Star body r(theta, phi) = r0 (1 + sum c_lm Y_lm) on the centred grid:
 * delta = delta0 o, beta = beta0 o with o the occupancy above.
 */
void oracle_render_sh(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                      int32_t lmax, const double* c, double r0, double edge, double delta0,
                      double beta0, double* delta, double* beta)
{
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < nx; ++a) {
        const double x = ((double)(2 * a + 1 - nx) * dx) / 2.0;
        for (int32_t b = 0; b < ny; ++b) {
            const double y = ((double)(2 * b + 1 - ny) * dy) / 2.0;
            for (int32_t k = 0; k < nz; ++k) {
                const double z = ((double)(2 * k + 1 - nz) * dz) / 2.0;
                double r, ct, phi;
                oracle_direction(x, y, z, &r, &ct, &phi);
                const double o = oracle_occupancy(oracle_star_radius(lmax, c, r0, ct, phi), r, edge);
                const int64_t v = ((int64_t)a * ny + b) * nz + k;
                delta[v] = delta0 * o;
                beta[v] = beta0 * o;
            }
        }
    }
}

/*
 * Gradient of a loss through the soft star body (edge > 0):
 * dL/dc_lm = sum_v (gd_v delta0 + gb_v beta0) o (1 - o) / edge * r0 Y_lm.
 */
void oracle_render_sh_backward(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                               int32_t lmax, const double* c, double r0, double edge, double delta0,
                               double beta0, const double* gd, const double* gb, double* gc)
{
    const int nc = (lmax + 1) * (lmax + 1);
    for (int k = 0; k < nc; ++k) gc[k] = 0.0;
    for (int32_t a = 0; a < nx; ++a) {
        const double x = ((double)(2 * a + 1 - nx) * dx) / 2.0;
        for (int32_t b = 0; b < ny; ++b) {
            const double y = ((double)(2 * b + 1 - ny) * dy) / 2.0;
            for (int32_t k = 0; k < nz; ++k) {
                const double z = ((double)(2 * k + 1 - nz) * dz) / 2.0;
                double r, ct, phi;
                oracle_direction(x, y, z, &r, &ct, &phi);
                const double o = oracle_occupancy(oracle_star_radius(lmax, c, r0, ct, phi), r, edge);
                const int64_t v = ((int64_t)a * ny + b) * nz + k;
                const double s = (gd[v] * delta0 + gb[v] * beta0) * o * (1.0 - o) / edge * r0;
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m) gc[l * l + l + m] += s * oracle_ylm(l, m, ct, phi);
            }
        }
    }
}

/*
 * Ellipsoid with semi-axes ax[3] along the columns of the rotation rot (row-major
 * 3 x 3): body coordinates p = rot^T r, inside iff sum (p_k / a_k)^2 <= 1.  The soft
 * form uses the radius along the voxel's direction, r_e = r / rho with
 * rho = sqrt(sum (p_k / a_k)^2), so o = sigmoid((r_e - r) / edge) = sigmoid(r_e (1 - rho) / edge).
 */
void oracle_render_ellipsoid(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                             const double* ax, const double* rot, double edge, double delta0,
                             double beta0, double* delta, double* beta)
{
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < nx; ++a) {
        const double x = ((double)(2 * a + 1 - nx) * dx) / 2.0;
        for (int32_t b = 0; b < ny; ++b) {
            const double y = ((double)(2 * b + 1 - ny) * dy) / 2.0;
            for (int32_t k = 0; k < nz; ++k) {
                const double z = ((double)(2 * k + 1 - nz) * dz) / 2.0;
                const double r = sqrt(x * x + y * y + z * z);
                double rho2 = 0.0, e2 = 0.0;   /* e2: the same for the unit direction (+z at 0) */
                for (int j = 0; j < 3; ++j) {
                    const double pj = x * rot[0 * 3 + j] + y * rot[1 * 3 + j] + z * rot[2 * 3 + j];
                    rho2 += (pj / ax[j]) * (pj / ax[j]);
                    const double uj = r > 0.0 ? pj / r : rot[2 * 3 + j];
                    e2 += (uj / ax[j]) * (uj / ax[j]);
                }
                double o;
                if (edge <= 0.0) o = rho2 <= 1.0 ? 1.0 : 0.0;
                else o = oracle_occupancy(1.0 / sqrt(e2), r, edge);
                const int64_t v = ((int64_t)a * ny + b) * nz + k;
                delta[v] = delta0 * o;
                beta[v] = beta0 * o;
            }
        }
    }
}

/*
 * Volume map: delta, beta given on a source grid (sx, sy, sz voxels of pitch sd*, centred
 * on the origin) resampled at the centres of the target grid by trilinear interpolation
 * between source voxel centres, with zero beyond the source grid.
 */
static double oracle_volume_at(const double* src, int32_t sx, int32_t sy, int32_t sz, double fx,
                               double fy, double fz)
{
    const double ax = floor(fx), ay = floor(fy), az = floor(fz);
    const double wx = fx - ax, wy = fy - ay, wz = fz - az;
    double v = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                const int64_t a = (int64_t)ax + i, b = (int64_t)ay + j, c = (int64_t)az + k;
                if (a < 0 || a >= sx || b < 0 || b >= sy || c < 0 || c >= sz) continue;
                const double w = (i ? wx : 1.0 - wx) * (j ? wy : 1.0 - wy) * (k ? wz : 1.0 - wz);
                v += w * src[(a * sy + b) * sz + c];
            }
    return v;
}

void oracle_render_volume(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                          int32_t sx, int32_t sy, int32_t sz, double sdx, double sdy, double sdz,
                          const double* sd, const double* sb, double* delta, double* beta)
{
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < nx; ++a) {
        const double x = ((double)(2 * a + 1 - nx) * dx) / 2.0;
        const double fx = x / sdx + (sx - 1) / 2.0;
        for (int32_t b = 0; b < ny; ++b) {
            const double y = ((double)(2 * b + 1 - ny) * dy) / 2.0;
            const double fy = y / sdy + (sy - 1) / 2.0;
            for (int32_t k = 0; k < nz; ++k) {
                const double z = ((double)(2 * k + 1 - nz) * dz) / 2.0;
                const double fz = z / sdz + (sz - 1) / 2.0;
                const int64_t v = ((int64_t)a * ny + b) * nz + k;
                delta[v] = oracle_volume_at(sd, sx, sy, sz, fx, fy, fz);
                beta[v] = oracle_volume_at(sb, sx, sy, sz, fx, fy, fz);
            }
        }
    }
}

/*
 * Ideal detector (Sec. 5.2, second example: the detector that adds the photon
 * statistics of a real recording).  The paper leaves the scaling to its
 * supplemental material; the reading taken here is the scalar first-Born
 * scattering cross section: a pixel p of solid angle dOmega_p receives on average
 *     mu_p = F * (k0^2 / (4 pi))^2 * I_p * dOmega_p
 * photons for an incident fluence F (photons per unit area; the paper's photon
 * density), since the far-field amplitude of Eq. (1) is k0^2 / (4 pi) times the
 * volume sum A that I = |A|^2 squares.  The recorded count is one Poisson draw
 * of mean mu_p.
 */

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128
 * multiplies with the key bumped by the Weyl constants between rounds. */
static void oracle_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
    const uint64_t w0 = 0x9E3779B97F4A7C15ULL, w1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += w0;
            k[1] += w1;
        }
        const unsigned __int128 p0 = (unsigned __int128)m0 * c[0];
        const unsigned __int128 p1 = (unsigned __int128)m1 * c[2];
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        const uint64_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* Exported for the generator's known-answer pin. */
void oracle_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out)
{
    oracle_philox4x64(ctr, key, out);
}

/* The stream of uniforms of pixel p: uniform m is word m % 4 of the block with
 * counter (m / 4, p, 0, 0) under key (seed, 0), mapped to [0, 1) by its top 53 bits. */
typedef struct {
    uint64_t key[2];
    uint64_t pixel;
    uint64_t m;
    uint64_t block[4];
} oracle_stream;

static double oracle_uniform(oracle_stream* s)
{
    if ((s->m & 3) == 0) {
        const uint64_t ctr[4] = {s->m >> 2, s->pixel, 0, 0};
        oracle_philox4x64(ctr, s->key, s->block);
    }
    const uint64_t x = s->block[s->m & 3];
    s->m += 1;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/*
 * One Poisson draw of mean mu.  Below mu = 10: inversion, the smallest k whose
 * cumulative probability reaches one uniform, the terms built by
 * p_k = p_{k-1} mu / k.  From mu = 10: the transformed rejection with squeeze of
 * Hormann (1993, "PTRS"), whose hat is a transformed uniform pair (U, V).
 */
static double oracle_poisson(oracle_stream* s, double mu)
{
    if (!(mu > 0.0) || !isfinite(mu)) return 0.0;
    if (mu < 10.0) {
        const double u = oracle_uniform(s);
        double k = 0.0, p = exp(-mu), f = p;
        while (u > f && p > 0.0) {
            k += 1.0;
            p = (p * mu) / k;
            f += p;
        }
        return k;
    }
    const double smu = sqrt(mu), lmu = log(mu);
    const double b = 0.931 + 2.53 * smu;
    const double a = -0.059 + 0.02483 * b;
    const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        const double u = oracle_uniform(s) - 0.5;
        const double v = oracle_uniform(s);
        const double us = 0.5 - fabs(u);
        const double k = floor((2.0 * a / us + b) * u + mu + 0.43);
        if (us >= 0.07 && v <= vr) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        const double lhs = log(v) + log(inv_alpha) - log(a / (us * us) + b);
        const double rhs = -mu + k * lmu - lgamma(k + 1.0);
        if (lhs <= rhs) return k;
    }
}

/* Solid angle, seen from the origin, of the flat-screen rectangle [0, u] x [0, v]
 * at unit distance (signed: odd in u and in v). */
static double oracle_rect_angle(double u, double v)
{
    return atan((u * v) / sqrt(1.0 + u * u + v * v));
}

/* Solid angle of pixel (i, j) of the flat N x N detector whose outer edge is at
 * tan(theta_max): the pixel spans u in [(2i - N) t / N, (2i + 2 - N) t / N]. */
double oracle_pixel_solid_angle(double theta_max_deg, int32_t n, int32_t i, int32_t j)
{
    const double t = tan((theta_max_deg * ORACLE_PI) / 180.0);
    const double u0 = ((double)(2 * i - n) * t) / (double)n;
    const double u1 = ((double)(2 * i + 2 - n) * t) / (double)n;
    const double v0 = ((double)(2 * j - n) * t) / (double)n;
    const double v1 = ((double)(2 * j + 2 - n) * t) / (double)n;
    return oracle_rect_angle(u1, v1) - oracle_rect_angle(u0, v1) - oracle_rect_angle(u1, v0) +
           oracle_rect_angle(u0, v0);
}

/* Expected counts mu[p] and one Poisson recording counts[p] of the intensity I[p]
 * (p = j N + i) on the flat detector, for fluence F and generator seed. */
void oracle_detect_ideal(double wavelength, double theta_max_deg, int32_t n, const double* intensity,
                         double fluence, uint64_t seed, double* mu, double* counts)
{
    const double k0 = oracle_k0(wavelength);
    const double f = (k0 * k0) / (4.0 * ORACLE_PI);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t i = 0; i < n; ++i) {
            const int64_t p = (int64_t)j * n + i;
            const double m = fluence * (f * f) * intensity[p] * oracle_pixel_solid_angle(theta_max_deg, n, i, j);
            oracle_stream s = {{seed, 0}, (uint64_t)p, 0, {0, 0, 0, 0}};
            mu[p] = m;
            counts[p] = oracle_poisson(&s, m);
        }
    }
}
