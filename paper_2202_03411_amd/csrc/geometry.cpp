// Host-side FP64 geometry of the MSFT library: argument validation, the pixel ->
// transfer-momentum map of a flat detector and the voxel grid.
//
// Built with -ffp-contract=off so that every product and sum is rounded on its
// own, which makes the q table reproducible bit for bit on any x86-64 host.
#include <cmath>
#include <cstdio>

#include "msft_internal.h"

namespace msft {

static const double kPi = 3.14159265358979323846;

msft_status validate_geometry(const msft_geometry* g, bool qlist, std::string* why)
{
    char buf[256];
    auto fail = [&](const char* msg) {
        if (why) *why = msg;
        return MSFT_ERR_INVALID;
    };
    if (!g) return fail("geometry pointer is NULL");
    if (g->struct_size != sizeof(msft_geometry)) {
        std::snprintf(buf, sizeof buf, "struct_size %u != sizeof(msft_geometry) %zu",
                      g->struct_size, sizeof(msft_geometry));
        if (why) *why = buf;
        return MSFT_ERR_INVALID;
    }
    if (!(g->wavelength > 0.0) || !std::isfinite(g->wavelength)) return fail("wavelength must be > 0");
    if (!qlist) {
        if (!(g->theta_max_deg > 0.0 && g->theta_max_deg < 90.0))
            return fail("theta_max_deg must lie in (0, 90)");
        if (g->det_n < 1 || g->det_n > 16384) return fail("det_n must lie in [1, 16384]");
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail("nx, ny, nz must be >= 1");
    if (g->nx > 4096 || g->ny > 4096 || g->nz > 4096) return fail("nx, ny, nz must be <= 4096");
    if (!(g->dx > 0.0 && g->dy > 0.0 && g->dz > 0.0) || !std::isfinite(g->dx) ||
        !std::isfinite(g->dy) || !std::isfinite(g->dz))
        return fail("voxel pitch must be finite and > 0");
    if (g->precision != MSFT_FP32 && g->precision != MSFT_BF16X3 && g->precision != MSFT_BF16)
        return fail("unknown precision");
    if (g->strength != MSFT_STRENGTH_MSFT && g->strength != MSFT_STRENGTH_BORN &&
        g->strength != MSFT_STRENGTH_DENSITY)
        return fail("unknown strength mode");
    if (g->flags & ~(MSFT_ALLOW_ALIAS | MSFT_DETECTOR_UNIFORM_Q)) return fail("unknown flag bits");
    if (qlist && (g->flags & MSFT_DETECTOR_UNIFORM_Q))
        return fail("a q-list plan has no detector: MSFT_DETECTOR_UNIFORM_Q does not apply");
    const double tiles = (double)ceil_div(g->nx, XC) * (double)ceil_div(g->nz, ZB) * (double)g->ny;
    if (tiles * TILE_BYTES > 64.0 * 1024 * 1024 * 1024) return fail("voxel grid too large");
    return MSFT_OK;
}

// Flat screen at unit distance; pixel centre (u_i, v_j, 1); khat = (u, v, 1) / r;
// q = k0 (khat - zhat), so q_z = k0 (1/r - 1) = -k0 s / (r (r + 1)), s = u^2 + v^2.
void detector_qmap(double wavelength, double theta_max_deg, int32_t n, double* q)
{
    const double k0 = (2.0 * kPi) / wavelength;
    const double t = std::tan((theta_max_deg * kPi) / 180.0);
    for (int32_t j = 0; j < n; ++j) {
        const double v = ((double)(2 * j + 1 - n) * t) / (double)n;
        for (int32_t i = 0; i < n; ++i) {
            const double u = ((double)(2 * i + 1 - n) * t) / (double)n;
            const double uu = u * u;
            const double vv = v * v;
            const double s = uu + vv;
            const double r = std::sqrt(s + 1.0);
            double* qp = q + 3 * ((int64_t)j * n + i);
            qp[0] = (k0 * u) / r;
            qp[1] = (k0 * v) / r;
            qp[2] = -((k0 * s) / (r * (r + 1.0)));
        }
    }
}

// Uniform transverse-q grid: q_x(i) = (2i + 1 - N) q_max / N, q_max = k0 sin(theta_max);
// q_z = sqrt(k0^2 - s) - k0 = -s / (sqrt(k0^2 - s) + k0), s = q_x^2 + q_y^2 (the
// cancellation-free form); NaN where s >= k0^2.
void uniform_qmap(double wavelength, double theta_max_deg, int32_t n, double* q, double* qx,
                  double* qy)
{
    const double k0 = (2.0 * kPi) / wavelength;
    const double qmax = k0 * std::sin((theta_max_deg * kPi) / 180.0);
    const double kk = k0 * k0;
    for (int32_t a = 0; a < n; ++a) {
        const double v = ((double)(2 * a + 1 - n) * qmax) / (double)n;
        qx[a] = v;
        qy[a] = v;
    }
    for (int32_t j = 0; j < n; ++j)
        for (int32_t i = 0; i < n; ++i) {
            const double s = qx[i] * qx[i] + qy[j] * qy[j];
            double* qp = q + 3 * ((int64_t)j * n + i);
            qp[0] = qx[i];
            qp[1] = qy[j];
            qp[2] = s < kk ? -(s / (std::sqrt(kk - s) + k0)) : std::nan("");
        }
}

SepDims make_sep_dims(int32_t n, int ny)
{
    SepDims s;
    s.n = n;
    s.npad = (int32_t)(ceil_div(n, BLOCK_PIX) * BLOCK_PIX);
    s.nblk1 = ceil_div(n, BLOCK_PIX);
    s.y_pad = (int32_t)(ceil_div(ny, XPAD) * XPAD);
    s.nyc = (int32_t)ceil_div(ny, XC);
    s.njc = s.npad / XC;
    s.nic = (int32_t)ceil_div(n, XC);
    return s;
}

void voxel_centres(int32_t n, double d, double* c)
{
    for (int32_t a = 0; a < n; ++a) c[a] = ((double)(2 * a + 1 - n) * d) / 2.0;
}

bool sampling_ok(const Geometry& geo, int* bad_axis, double* worst)
{
    const double pitch[3] = {geo.g.dx, geo.g.dy, geo.g.dz};
    double mx[3] = {0.0, 0.0, 0.0};
    for (int64_t p = 0; p < geo.npix; ++p)
        for (int k = 0; k < 3; ++k) mx[k] = std::fmax(mx[k], std::fabs(geo.q[3 * p + k]));
    bool ok = true;
    double w = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double v = mx[k] * pitch[k];
        if (v > w) w = v;
        if (v > kPi && ok) {
            ok = false;
            if (bad_axis) *bad_axis = k;
        }
    }
    if (worst) *worst = w;
    return ok;
}

Dims make_dims(int64_t npix, int nx, int ny, int nz)
{
    Dims d;
    d.npix = npix;
    d.nblocks = ceil_div(npix, BLOCK_PIX);
    d.nwt = d.nblocks * WAVES;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.x_pad = (int)ceil_div(nx, XPAD) * XPAD;
    d.nxc = (int)ceil_div(nx, XC);
    d.nxc3 = (int)ceil_div(nx, G3_XC);
    d.nzb = (int)ceil_div(nz, ZB);
    return d;
}

// Pixel groups of the adjoint's split K: enough workgroups to fill the chip
// (about 2048) without making a group smaller than one LDS chunk.
AdjDims make_adj_dims(const Dims& d)
{
    AdjDims a;
    a.nyb = (int32_t)ceil_div(d.ny, ADJ_Y);
    const int64_t npix_pad = d.nblocks * BLOCK_PIX;
    const int64_t chunks = ceil_div(npix_pad, ADJ_CHUNK);
    const int64_t base = (int64_t)d.nxc * d.nzb * a.nyb;
    int64_t split = ceil_div(2048, base);
    if (split < 1) split = 1;
    if (split > chunks) split = chunks;
    a.group_pix = ceil_div(chunks, split) * ADJ_CHUNK;
    a.nsplit = (int32_t)ceil_div(npix_pad, a.group_pix);
    a.h_bytes = (size_t)(ceil_div(npix_pad * 8, 256) * 256);
    a.rpart_bytes = (size_t)a.nsplit * d.nxc * XC * d.ny * d.nzb * ZB * 8;
    return a;
}

}  // namespace msft
