// C ABI of the MSFT library: plan lifecycle, argument checking and the
// launches of the forward model.  Host code only; kernels live in the .hip files.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "msft_internal.h"

using namespace msft;

namespace {

thread_local std::string g_last_error;

msft_status fail(msft_status s, const std::string& why)
{
    g_last_error = why;
    return s;
}

msft_status ok()
{
    g_last_error.clear();
    return MSFT_OK;
}

// Makes `device` current for the scope of a call and restores the caller's.
struct DeviceScope {
    int prev = -1;
    bool changed = false;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int device)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != device) {
            err = hipSetDevice(device);
            changed = (err == hipSuccess);
        }
    }
    ~DeviceScope()
    {
        if (changed) (void)hipSetDevice(prev);
    }
};

msft_status hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? MSFT_ERR_NOMEM : MSFT_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void free_device(msft_plan_s* p)
{
    if (p->device < 0) return;
    DeviceScope ds(p->device);
    void* ptrs[] = {p->q_dev, p->xs_dev, p->ys_dev, p->zs_dev, p->txa, p->ty, p->tz, p->txa2,
                    p->txT, p->tyT};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    p->q_dev = p->xs_dev = p->ys_dev = p->zs_dev = nullptr;
    p->txa = p->txa2 = p->txT = p->tyT = nullptr;
    p->ty = p->tz = nullptr;
}

template <typename T>
hipError_t dev_alloc(T** out, size_t bytes, size_t* total)
{
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes ? bytes : 256);
    if (e == hipSuccess) {
        *out = (T*)ptr;
        *total += bytes;
    }
    return e;
}

// Resident tables of a plan on its device: FP64 q and coordinates, then the
// twiddle tables generated from them.
msft_status build_device_tables(msft_plan_s* p)
{
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    const Dims& d = p->dims;
    const Geometry& geo = p->geo;
    size_t total = 0;
    hipError_t e;
#define MSFT_TRY(expr, what)                  \
    do {                                      \
        e = (expr);                           \
        if (e != hipSuccess) {                \
            free_device(p);                   \
            return hip_fail(e, what);         \
        }                                     \
    } while (0)
    // The adjoint reads q per pixel; a pixel beyond the Ewald sphere's rim (q_z NaN)
    // has A = 0 and so h = 0, and any finite q_z keeps its terms at zero.
    std::vector<double> qd(geo.q);
    for (int64_t k = 2; k < 3 * geo.npix; k += 3)
        if (!std::isfinite(qd[k])) qd[k] = 0.0;
    MSFT_TRY(dev_alloc(&p->q_dev, sizeof(double) * 3 * geo.npix, &total), "hipMalloc q");
    MSFT_TRY(dev_alloc(&p->xs_dev, sizeof(double) * d.nx, &total), "hipMalloc x");
    MSFT_TRY(dev_alloc(&p->ys_dev, sizeof(double) * d.ny, &total), "hipMalloc y");
    MSFT_TRY(dev_alloc(&p->zs_dev, sizeof(double) * d.nz, &total), "hipMalloc z");
    if (p->separable) {
        const SepDims& sd = p->sep;
        MSFT_TRY(dev_alloc(&p->txa, sd.gauss ? sd.txa1g_bytes(d.nxc3) : sd.txa1_bytes(d.nxc), &total),
                 "hipMalloc Tx");
        MSFT_TRY(dev_alloc(&p->txa2, sd.gauss ? sd.txa2g_bytes() : sd.txa2_bytes(), &total), "hipMalloc Ty");
        MSFT_TRY(dev_alloc(&p->tz, p->sep.tz_bytes(d.nzb), &total), "hipMalloc Tz");
        MSFT_TRY(dev_alloc(&p->txT, sd.gauss ? sd.txTg_bytes(d.nx) : sd.txT_bytes(d.nx), &total),
                 "hipMalloc adjoint Tx");
        MSFT_TRY(dev_alloc(&p->tyT, sd.gauss ? sd.tyTg_bytes(d.ny) : sd.tyT_bytes(d.ny), &total),
                 "hipMalloc adjoint Ty");
    } else {
        MSFT_TRY(dev_alloc(&p->txa, d.txa_bytes(), &total), "hipMalloc Tx");
        MSFT_TRY(dev_alloc(&p->ty, d.ty_bytes(), &total), "hipMalloc Ty");
        MSFT_TRY(dev_alloc(&p->tz, d.tz_bytes(), &total), "hipMalloc Tz");
    }
    MSFT_TRY(hipMemcpy(p->q_dev, qd.data(), sizeof(double) * 3 * geo.npix, hipMemcpyHostToDevice),
             "copy q");
    MSFT_TRY(hipMemcpy(p->xs_dev, geo.xs.data(), sizeof(double) * d.nx, hipMemcpyHostToDevice), "copy x");
    MSFT_TRY(hipMemcpy(p->ys_dev, geo.ys.data(), sizeof(double) * d.ny, hipMemcpyHostToDevice), "copy y");
    MSFT_TRY(hipMemcpy(p->zs_dev, geo.zs.data(), sizeof(double) * d.nz, hipMemcpyHostToDevice), "copy z");
    hipStream_t s = nullptr;
    MSFT_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    if (p->separable) {
        // per-column q_x, per-row q_y (slot 0 of a [N][3] array each) and q_z over the
        // second stage's pixel order (i, j), NaN for padding rows j >= N
        const SepDims& sd = p->sep;
        std::vector<double> qcol(3 * (size_t)sd.n, 0.0), qrow(3 * (size_t)sd.n, 0.0);
        std::vector<double> qk(3 * (size_t)sd.n * sd.npad, std::nan(""));
        std::vector<double> qxv(sd.n), qyv(sd.n), xq3(3 * (size_t)d.nx, 0.0), yq3(3 * (size_t)d.ny, 0.0);
        for (int32_t a = 0; a < sd.n; ++a) {
            qcol[3 * a] = qxv[a] = geo.q[3 * (size_t)a];              // pixel (i = a, j = 0)
            qrow[3 * a] = qyv[a] = geo.q[3 * ((size_t)a * sd.n) + 1]; // pixel (i = 0, j = a)
        }
        for (int a = 0; a < d.nx; ++a) xq3[3 * a] = geo.xs[a];
        for (int a = 0; a < d.ny; ++a) yq3[3 * a] = geo.ys[a];
        for (int32_t i = 0; i < sd.n; ++i)
            for (int32_t j = 0; j < sd.n; ++j)
                qk[3 * ((size_t)i * sd.npad + j) + 2] = geo.q[3 * ((size_t)j * sd.n + i) + 2];
        std::vector<const std::vector<double>*> host = {&qcol, &qrow, &qk, &qxv, &qyv, &xq3, &yq3};
        std::vector<double*> dev(host.size(), nullptr);
        size_t scratch = 0;
        e = hipSuccess;
        for (size_t k = 0; k < host.size() && e == hipSuccess; ++k) {
            e = dev_alloc(&dev[k], sizeof(double) * host[k]->size(), &scratch);
            if (e == hipSuccess)
                e = hipMemcpy(dev[k], host[k]->data(), sizeof(double) * host[k]->size(),
                              hipMemcpyHostToDevice);
        }
        if (e == hipSuccess)
            e = (hipError_t)launch_sep_twiddles(p->geo.g.precision, d, sd, dev[0], dev[1], dev[2],
                                                p->xs_dev, p->ys_dev, p->zs_dev,
                                                sd.gauss ? nullptr : p->txa,
                                                sd.gauss ? nullptr : p->txa2, p->tz, s);
        if (e == hipSuccess && sd.gauss)
            e = (hipError_t)launch_sepg_twiddles(sd, d.nx, d.ny, d.nxc3, dev[3], dev[4], p->xs_dev,
                                                 p->ys_dev, p->txa, p->txa2, s);
        if (e == hipSuccess)
            e = sd.gauss ? (hipError_t)launch_sepg_adj_tables(sd, d.nx, d.ny, p->xs_dev, dev[3], p->ys_dev,
                                                              dev[4], p->txT, p->tyT, s)
                         : (hipError_t)launch_sep_adj_tables(sd, d.nx, d.ny, dev[5], dev[3], dev[6], dev[4],
                                                             p->txT, p->tyT, s);
        hipError_t e2 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e2;
        for (double* t : dev)
            if (t) (void)hipFree(t);
    } else if (d.g3) {
        e = (hipError_t)launch_twiddles_g3(d, p->q_dev, p->xs_dev, p->ys_dev, p->zs_dev, p->txa,
                                           p->ty, p->tz, s);
        hipError_t e2 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e2;
    } else {
        e = (hipError_t)launch_twiddles(p->geo.g.precision, d, p->q_dev, p->xs_dev, p->ys_dev,
                                        p->zs_dev, p->txa, p->ty, p->tz, s);
        hipError_t e2 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e2;
    }
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        free_device(p);
        return hip_fail(e, "twiddle generation");
    }
#undef MSFT_TRY
    p->resident_bytes = total;
    return MSFT_OK;
}

// Workspace of the separable adjoint: h [P] complex, K tiles, R [nxc*64][ny][nzb*32]
// complex; returns the total and the offsets of K and R.
size_t sep_adj_layout(const msft_plan_s* p, size_t* k_off, size_t* r_off)
{
    const Dims& d = p->dims;
    const size_t hb = align256((size_t)d.npix * 8);
    const size_t kb = align256(p->sep.gauss ? p->sep.kg_bytes(d.ny, d.nzb) : p->sep.k_bytes(d.ny, d.nzb));
    const size_t rb = align256((size_t)(p->sep.gauss ? SEPG_ADJ_SPLIT : 1) * d.nxc * XC * d.ny * d.nzb * ZB * 8);
    if (k_off) *k_off = hb;
    if (r_off) *r_off = hb + kb;
    return hb + kb + rb;
}

msft_status make_plan(const msft_geometry* g, const double* q_host, int64_t npix, int device,
                      msft_plan_t* out)
{
    if (!out) return fail(MSFT_ERR_INVALID, "out pointer is NULL");
    *out = nullptr;
    const bool qlist = (q_host != nullptr);
    std::string why;
    msft_status st = validate_geometry(g, qlist, &why);
    if (st != MSFT_OK) return fail(st, why);
    if (qlist && (npix < 1 || npix > ((int64_t)1 << 28)))
        return fail(MSFT_ERR_INVALID, "npix must lie in [1, 2^28]");

    msft_plan_s* p = new (std::nothrow) msft_plan_s;
    if (!p) return fail(MSFT_ERR_NOMEM, "plan allocation");
    p->qlist = qlist;
    p->geo.g = *g;
    try {
        if (qlist) {
            p->geo.npix = npix;
            p->geo.q.assign(q_host, q_host + 3 * npix);
            for (int64_t k = 0; k < 3 * npix; ++k)
                if (!std::isfinite(p->geo.q[k])) {
                    delete p;
                    return fail(MSFT_ERR_INVALID, "q list holds a non-finite value");
                }
        } else if (g->flags & MSFT_DETECTOR_UNIFORM_Q) {
            p->separable = true;
            p->geo.npix = (int64_t)g->det_n * g->det_n;
            p->geo.q.resize(3 * p->geo.npix);
            std::vector<double> qx(g->det_n), qy(g->det_n);
            uniform_qmap(g->wavelength, g->theta_max_deg, g->det_n, p->geo.q.data(), qx.data(),
                         qy.data());
        } else {
            p->geo.npix = (int64_t)g->det_n * g->det_n;
            p->geo.q.resize(3 * p->geo.npix);
            detector_qmap(g->wavelength, g->theta_max_deg, g->det_n, p->geo.q.data());
        }
        p->geo.xs.resize(g->nx);
        p->geo.ys.resize(g->ny);
        p->geo.zs.resize(g->nz);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(MSFT_ERR_NOMEM, "host tables");
    }
    voxel_centres(g->nx, g->dx, p->geo.xs.data());
    voxel_centres(g->ny, g->dy, p->geo.ys.data());
    voxel_centres(g->nz, g->dz, p->geo.zs.data());

    int bad = -1;
    double worst = 0.0;
    if (!(g->flags & MSFT_ALLOW_ALIAS) && !sampling_ok(p->geo, &bad, &worst)) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "undersampled: pitch * max|q| = %.4g > pi on axis %c (set MSFT_ALLOW_ALIAS)",
                      worst, "xyz"[bad < 0 ? 0 : bad]);
        delete p;
        return fail(MSFT_ERR_UNDERSAMPLED, buf);
    }
    p->dims = make_dims(p->geo.npix, g->nx, g->ny, g->nz);
    if (p->separable) {
        p->sep = make_sep_dims(g->det_n, g->ny);
        p->sep.nyc2 = (int32_t)ceil_div(g->ny, 32);
        p->sep.gauss = g->precision == MSFT_FP32 && p->sep.nyc2 <= SG2_MAXYC;
        p->sep.nic3 = (int32_t)ceil_div(g->det_n, 32);
    }
    // FP32 runs the Gauss (three-product) contractions: the flat detector and q
    // lists always, the separable detector up to SG2_MAXYC * 32 rows y
    p->dims.g3 = g->precision == MSFT_FP32 && (!p->separable || p->sep.gauss);
    size_t fwd_ws = align256(p->dims.wtile_bytes());
    size_t adj_ws = align256(make_adj_dims(p->dims).bytes());
    if (p->separable) {
        fwd_ws += align256(p->sep.gauss ? p->sep.hg_bytes(p->dims.nzb) : p->sep.h_bytes(p->dims.nzb));
        adj_ws = sep_adj_layout(p, nullptr, nullptr);
    }
    p->fwd_workspace = fwd_ws;
    p->adj_workspace = adj_ws;
    p->workspace_bytes = std::max(fwd_ws, adj_ws);
    // delta, beta in; intensity and amplitude out; the request's W tiles in a batch
    p->per_request = align256(sizeof(float) * (size_t)g->nx * g->ny * g->nz) * 2 +
                     align256(sizeof(float) * (size_t)p->geo.npix) +
                     align256(2 * sizeof(float) * (size_t)p->geo.npix) + fwd_ws;
    p->device = device;
    if (device >= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || device >= count) {
            p->device = -1;
            delete p;
            return fail(MSFT_ERR_DEVICE, "no such HIP device");
        }
        st = build_device_tables(p);
        if (st != MSFT_OK) {
            p->device = -1;
            delete p;
            return st;
        }
    }
    *out = p;
    return ok();
}

bool aligned256(const void* ptr) { return ((uintptr_t)ptr & 255) == 0; }

// A caller's workspace: 256-byte aligned and at least `need` bytes.
msft_status check_workspace(const void* ws, size_t ws_bytes, size_t need)
{
    if (!aligned256(ws)) return fail(MSFT_ERR_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < need) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "workspace of %zu bytes, the call needs %zu", ws_bytes, need);
        return fail(MSFT_ERR_BUSY, buf);
    }
    return MSFT_OK;
}

FwdArgs forward_args(const msft_plan_s* p, const void* wtiles, float* intensity, float* amplitude)
{
    FwdArgs a;
    a.wtiles = (const uint8_t*)wtiles;
    a.txa = p->txa;
    a.ty = p->ty;
    a.tz = p->tz;
    a.intensity = intensity;
    a.amplitude = amplitude;
    a.npix = p->dims.npix;
    a.ny = p->dims.ny;
    a.nxc = p->dims.g3 ? p->dims.nxc3 : p->dims.nxc;
    a.nzb = p->dims.nzb;
    a.x_pad = p->dims.x_pad;
    a.group_blocks = a.group_tiles = a.out_n = a.out_npad = 0;
    return a;
}

// Second stage of the separable detector: H tiles (after the W tiles in the
// workspace) contracted over y; one tile group of nyc * nzb tiles per column i.
FwdArgs sep_stage2_args(const msft_plan_s* p, const void* workspace, float* intensity,
                        float* amplitude)
{
    const SepDims& sd = p->sep;
    FwdArgs a;
    a.wtiles = (const uint8_t*)workspace + align256(p->dims.wtile_bytes());
    a.txa = p->txa2;
    a.ty = nullptr;
    a.tz = p->tz;
    a.intensity = intensity;
    a.amplitude = amplitude;
    a.npix = (int64_t)sd.n * sd.npad;
    a.ny = 1;
    a.nxc = sd.nyc;
    a.nzb = p->dims.nzb;
    a.x_pad = sd.y_pad;
    a.group_blocks = sd.npad / BLOCK_PIX;
    a.group_tiles = sd.nyc * p->dims.nzb;
    a.out_n = sd.n;
    a.out_npad = sd.npad;
    return a;
}

// Both stages in the Gauss form: H tiles after the W tiles in the workspace.
SepG3Args sepg_args(const msft_plan_s* p, const void* workspace, float* intensity, float* amplitude)
{
    const SepDims& sd = p->sep;
    SepG3Args a;
    a.wtiles = (const uint8_t*)workspace;
    a.txa1 = p->txa;
    a.htiles = (uint8_t*)workspace + align256(p->dims.wtile_bytes());
    a.txa2 = p->txa2;
    a.tz = p->tz;
    a.intensity = intensity;
    a.amplitude = amplitude;
    a.n = sd.n;
    a.npad = sd.npad;
    a.ny = p->dims.ny;
    a.nxc3 = p->dims.nxc3;
    a.nyc2 = sd.nyc2;
    a.nzb = p->dims.nzb;
    a.nblk1 = sd.nblk1;
    return a;
}

Stage1Args sep_stage1_args(const msft_plan_s* p, const void* workspace)
{
    Stage1Args a;
    a.wtiles = (const uint8_t*)workspace;
    a.txa = p->txa;
    a.htiles = (uint8_t*)workspace + align256(p->dims.wtile_bytes());
    a.n = p->sep.n;
    a.ny = p->dims.ny;
    a.nxc = p->dims.nxc;
    a.nzb = p->dims.nzb;
    a.x_pad = p->dims.x_pad;
    a.nyc = p->sep.nyc;
    return a;
}

// The contraction of a plan after the scan: one launch for the flat detector,
// the two stages for the separable one.
int launch_contraction(const msft_plan_s* p, const void* workspace, float* intensity,
                       float* amplitude, void* stream)
{
    const int prec = p->geo.g.precision;
    if (p->separable && p->sep.gauss) return launch_sepg(sepg_args(p, workspace, intensity, amplitude), stream);
    if (p->dims.g3)
        return launch_forward_g3(forward_args(p, workspace, intensity, amplitude), 0, p->dims.nblocks,
                                 stream);
    if (!p->separable)
        return launch_forward(prec, forward_args(p, workspace, intensity, amplitude), 0,
                              p->dims.nblocks, stream);
    int e = launch_sep_stage1(prec, sep_stage1_args(p, workspace), p->sep.nblk1, stream);
    if (e) return e;
    return launch_sep_stage2(prec, sep_stage2_args(p, workspace, intensity, amplitude), stream);
}

ScanArgs scan_args(const msft_plan_s* p, const float* delta, const float* beta, void* wtiles)
{
    const msft_geometry& g = p->geo.g;
    ScanArgs s;
    s.delta = delta;
    s.beta = beta;
    s.wtiles = (uint8_t*)wtiles;
    s.nx = g.nx;
    s.ny = g.ny;
    s.nz = g.nz;
    s.nxc = p->dims.nxc;
    s.nzb = p->dims.nzb;
    s.strength = g.strength;
    s.g3 = p->dims.g3 ? 1 : 0;
    s.nxc3 = p->dims.nxc3;
    const double k0 = (2.0 * 3.14159265358979323846) / g.wavelength;
    s.k0dz = (float)(k0 * g.dz);
    s.dV = (float)(g.dx * g.dy * g.dz);
    return s;
}

msft_status check_runnable(const msft_plan_s* p)
{
    if (!p) return fail(MSFT_ERR_INVALID, "plan is NULL");
    if (p->device < 0) return fail(MSFT_ERR_UNSUPPORTED, "host-only plan cannot simulate");
    return MSFT_OK;
}

msft_status shape_grid_args(const msft_shape_grid* g, RenderGrid* out)
{
    if (!g) return fail(MSFT_ERR_INVALID, "shape grid is NULL");
    if (g->struct_size != sizeof(msft_shape_grid))
        return fail(MSFT_ERR_INVALID, "struct_size != sizeof(msft_shape_grid)");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > 4096 || g->ny > 4096 || g->nz > 4096)
        return fail(MSFT_ERR_INVALID, "nx, ny, nz must lie in [1, 4096]");
    if (!(g->dx > 0.0 && g->dy > 0.0 && g->dz > 0.0) || !std::isfinite(g->dx) ||
        !std::isfinite(g->dy) || !std::isfinite(g->dz))
        return fail(MSFT_ERR_INVALID, "voxel pitch must be finite and > 0");
    if (!(g->edge >= 0.0) || !std::isfinite(g->edge)) return fail(MSFT_ERR_INVALID, "edge must be >= 0");
    if (!std::isfinite(g->delta0) || !std::isfinite(g->beta0))
        return fail(MSFT_ERR_INVALID, "delta0 and beta0 must be finite");
    out->nx = g->nx;
    out->ny = g->ny;
    out->nz = g->nz;
    out->dx = g->dx;
    out->dy = g->dy;
    out->dz = g->dz;
    out->edge = g->edge;
    out->delta0 = g->delta0;
    out->beta0 = g->beta0;
    return MSFT_OK;
}

// Recurrence constants of the normalised Legendre values, FP64 on the host.
msft_status sh_args(const msft_shape_grid* g, int32_t lmax, double r0, ShArgs* s)
{
    msft_status st = shape_grid_args(g, &s->g);
    if (st != MSFT_OK) return st;
    if (lmax < 0 || lmax > MAX_SH_L) return fail(MSFT_ERR_INVALID, "lmax must lie in [0, 12]");
    if (!(r0 > 0.0) || !std::isfinite(r0)) return fail(MSFT_ERR_INVALID, "r0 must be finite and > 0");
    s->lmax = lmax;
    s->r0 = r0;
    for (int m = 0; m < SH_TABLE; ++m) {
        s->diag[m] = m > 0 ? std::sqrt((2.0 * m + 1.0) / (2.0 * m)) : 1.0;
        s->sub[m] = std::sqrt(2.0 * m + 3.0);
    }
    for (int l = 0; l < SH_TABLE; ++l)
        for (int m = 0; m < SH_TABLE; ++m) {
            double a = 0.0, b = 0.0;
            if (l >= m + 2) {
                const double ll = l, mm = m;
                a = std::sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
                b = std::sqrt(((ll - 1.0) * (ll - 1.0) - mm * mm) / (4.0 * (ll - 1.0) * (ll - 1.0) - 1.0));
            }
            s->ra[l * SH_TABLE + m] = a;
            s->rb[l * SH_TABLE + m] = b;
        }
    return MSFT_OK;
}

}  // namespace

extern "C" {

msft_status msft_render_sh(const msft_shape_grid* g, int32_t lmax, double r0, const float* coeffs,
                           float* delta, float* beta, void* stream)
{
    ShArgs s;
    msft_status st = sh_args(g, lmax, r0, &s);
    if (st != MSFT_OK) return st;
    if (!coeffs || !delta || !beta) return fail(MSFT_ERR_INVALID, "NULL argument");
    int e = launch_render_sh(s, coeffs, delta, beta, stream);
    if (e) return hip_fail((hipError_t)e, "render launch");
    return ok();
}

msft_status msft_render_sh_query(int32_t lmax, size_t* workspace_bytes)
{
    if (lmax < 0 || lmax > MAX_SH_L) return fail(MSFT_ERR_INVALID, "lmax must lie in [0, 12]");
    if (workspace_bytes) *workspace_bytes = (size_t)SH_GRAD_BLOCKS * MAX_SH_COEFFS * sizeof(double);
    return ok();
}

msft_status msft_render_sh_backward(const msft_shape_grid* g, int32_t lmax, double r0,
                                    const float* coeffs, const float* grad_delta,
                                    const float* grad_beta, float* grad_coeffs, void* workspace,
                                    size_t ws_bytes, void* stream)
{
    ShArgs s;
    msft_status st = sh_args(g, lmax, r0, &s);
    if (st != MSFT_OK) return st;
    if (!(g->edge > 0.0)) return fail(MSFT_ERR_INVALID, "the gradient needs a soft edge (edge > 0)");
    if (!coeffs || !grad_delta || !grad_beta || !grad_coeffs || !workspace)
        return fail(MSFT_ERR_INVALID, "NULL argument");
    if (!aligned256(workspace)) return fail(MSFT_ERR_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < (size_t)SH_GRAD_BLOCKS * MAX_SH_COEFFS * sizeof(double))
        return fail(MSFT_ERR_BUSY, "workspace smaller than msft_render_sh_query");
    int e = launch_render_sh_grad(s, coeffs, grad_delta, grad_beta, grad_coeffs, (double*)workspace,
                                  SH_GRAD_BLOCKS, stream);
    if (e) return hip_fail((hipError_t)e, "render gradient launch");
    return ok();
}

msft_status msft_render_volume(const msft_shape_grid* g, int32_t sx, int32_t sy, int32_t sz,
                               double sdx, double sdy, double sdz, const float* src_delta,
                               const float* src_beta, float* delta, float* beta, void* stream)
{
    VolArgs a;
    msft_status st = shape_grid_args(g, &a.g);
    if (st != MSFT_OK) return st;
    if (sx < 1 || sy < 1 || sz < 1 || sx > 4096 || sy > 4096 || sz > 4096)
        return fail(MSFT_ERR_INVALID, "source voxel counts must lie in [1, 4096]");
    if (!(sdx > 0.0 && sdy > 0.0 && sdz > 0.0) || !std::isfinite(sdx) || !std::isfinite(sdy) ||
        !std::isfinite(sdz))
        return fail(MSFT_ERR_INVALID, "source pitch must be finite and > 0");
    if (!src_delta || !src_beta || !delta || !beta) return fail(MSFT_ERR_INVALID, "NULL argument");
    a.sx = sx;
    a.sy = sy;
    a.sz = sz;
    a.sdx = sdx;
    a.sdy = sdy;
    a.sdz = sdz;
    int e = launch_render_volume(a, src_delta, src_beta, delta, beta, stream);
    if (e) return hip_fail((hipError_t)e, "render launch");
    return ok();
}

msft_status msft_render_ellipsoid(const msft_shape_grid* g, const double* axes, const double* rot,
                                  float* delta, float* beta, void* stream)
{
    EllArgs a;
    msft_status st = shape_grid_args(g, &a.g);
    if (st != MSFT_OK) return st;
    if (!axes || !rot || !delta || !beta) return fail(MSFT_ERR_INVALID, "NULL argument");
    for (int k = 0; k < 3; ++k) {
        if (!(axes[k] > 0.0) || !std::isfinite(axes[k]))
            return fail(MSFT_ERR_INVALID, "semi-axes must be finite and > 0");
        a.ax[k] = axes[k];
    }
    for (int k = 0; k < 9; ++k) {
        if (!std::isfinite(rot[k])) return fail(MSFT_ERR_INVALID, "rotation must be finite");
        a.rot[k] = rot[k];
    }
    int e = launch_render_ellipsoid(a, delta, beta, stream);
    if (e) return hip_fail((hipError_t)e, "render launch");
    return ok();
}


msft_status msft_detect_ideal(msft_plan_t plan, const float* intensity, double photon_density,
                              uint64_t seed, float* counts, float* expected, void* stream)
{
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (plan->qlist || plan->separable)
        return fail(MSFT_ERR_INVALID, "the Ideal detector needs a flat-detector plan");
    if (!intensity || !counts) return fail(MSFT_ERR_INVALID, "intensity and counts must be non-NULL");
    if (!(photon_density >= 0.0) || !std::isfinite(photon_density))
        return fail(MSFT_ERR_INVALID, "photon_density must be finite and >= 0");
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    const msft_geometry& g = plan->geo.g;
    const double kPi = 3.14159265358979323846;
    const double k0 = (2.0 * kPi) / g.wavelength;
    const double f = (k0 * k0) / (4.0 * kPi);
    IdealArgs a;
    a.n = g.det_n;
    a.t = std::tan((g.theta_max_deg * kPi) / 180.0);
    a.scale = photon_density * (f * f);
    a.seed = seed;
    int e = launch_detect_ideal(a, intensity, counts, expected, stream);
    if (e) return hip_fail((hipError_t)e, "detector launch");
    return ok();
}

msft_status msft_peak_mfma(int32_t precision, int32_t iters, int32_t nblocks, float* sink, double* flops,
                           void* stream)
{
    if (precision != MSFT_FP32 && precision != MSFT_BF16X3)
        return fail(MSFT_ERR_INVALID, "precision must be MSFT_FP32 or MSFT_BF16X3");
    if (iters < 1 || nblocks < 1 || !sink || !flops)
        return fail(MSFT_ERR_INVALID, "iters and nblocks must be >= 1, sink and flops non-NULL");
    int e = launch_peak_mfma(precision, iters, nblocks, sink, flops, stream);
    if (e) return hip_fail((hipError_t)e, "peak launch");
    return ok();
}

msft_status msft_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    if (!src || !dst || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return fail(MSFT_ERR_INVALID, "src and dst must be 16-byte aligned and bytes a multiple of 16");
    if (bytes == 0) return ok();
    int e = launch_copy(src, dst, (int64_t)(bytes / 16), stream);
    if (e) return hip_fail((hipError_t)e, "copy launch");
    return ok();
}

msft_status msft_plan(const msft_geometry* g, int device, msft_plan_t* out)
{
    return make_plan(g, nullptr, 0, device, out);
}

msft_status msft_plan_qlist(const msft_geometry* g, const double* q_host, int64_t npix, int device,
                            msft_plan_t* out)
{
    if (!q_host) return fail(MSFT_ERR_INVALID, "q_host is NULL");
    return make_plan(g, q_host, npix, device, out);
}

msft_status msft_plan_destroy(msft_plan_t plan)
{
    if (!plan) return ok();
    if (plan->device >= 0) {
        DeviceScope ds(plan->device);
        (void)hipDeviceSynchronize();
    }
    free_device(plan);
    delete plan;
    return ok();
}

msft_status msft_plan_query(msft_plan_t plan, int64_t* npix, size_t* workspace_bytes,
                            size_t* resident_bytes, size_t* per_request_bytes)
{
    if (!plan) return fail(MSFT_ERR_INVALID, "plan is NULL");
    if (npix) *npix = plan->geo.npix;
    if (workspace_bytes) *workspace_bytes = plan->workspace_bytes;
    if (resident_bytes) *resident_bytes = plan->resident_bytes;
    if (per_request_bytes) *per_request_bytes = plan->per_request;
    return ok();
}

msft_status msft_plan_qmap(msft_plan_t plan, double* q_host)
{
    if (!plan || !q_host) return fail(MSFT_ERR_INVALID, "NULL argument");
    std::memcpy(q_host, plan->geo.q.data(), sizeof(double) * 3 * plan->geo.npix);
    return ok();
}

msft_status msft_plan_grid(msft_plan_t plan, double* x, double* y, double* z)
{
    if (!plan) return fail(MSFT_ERR_INVALID, "plan is NULL");
    if (x) std::memcpy(x, plan->geo.xs.data(), sizeof(double) * plan->geo.xs.size());
    if (y) std::memcpy(y, plan->geo.ys.data(), sizeof(double) * plan->geo.ys.size());
    if (z) std::memcpy(z, plan->geo.zs.data(), sizeof(double) * plan->geo.zs.size());
    return ok();
}

// The scan and the contraction of one target, the plan's device current.
static msft_status simulate_launch(msft_plan_t plan, const float* delta, const float* beta,
                                   float* intensity, float* amplitude, void* workspace, void* stream)
{
    const ScanArgs sa = scan_args(plan, delta, beta, workspace);
    int e = launch_scan(plan->geo.g.precision, sa, stream);
    if (e) return hip_fail((hipError_t)e, "scan launch");
    e = launch_contraction(plan, workspace, intensity, amplitude, stream);
    if (e) return hip_fail((hipError_t)e, "forward launch");
    return ok();
}

msft_status msft_simulate(msft_plan_t plan, const float* delta, const float* beta, float* intensity,
                          float* amplitude, void* workspace, size_t ws_bytes, void* stream)
{
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (!delta || !beta || !intensity || !workspace)
        return fail(MSFT_ERR_INVALID, "delta, beta, intensity and workspace must be non-NULL");
    st = check_workspace(workspace, ws_bytes, plan->fwd_workspace);
    if (st != MSFT_OK) return st;
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    return simulate_launch(plan, delta, beta, intensity, amplitude, workspace, stream);
}

msft_status msft_simulate_noalloc(msft_plan_t plan, const float* delta, const float* beta,
                                  float* intensity, float* amplitude, void* stream)
{
    if (!plan) return fail(MSFT_ERR_INVALID, "plan is NULL");
    if (plan->fwd_workspace > (size_t)MSFT_NOALLOC_MAX_BYTES) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "the plan's forward scratch is %zu bytes; the fixed scratch holds %zu",
                      plan->fwd_workspace, (size_t)MSFT_NOALLOC_MAX_BYTES);
        return fail(MSFT_ERR_UNSUPPORTED, buf);
    }
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (!delta || !beta || !intensity)
        return fail(MSFT_ERR_INVALID, "delta, beta and intensity must be non-NULL");
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    void* scratch = nullptr;
    const int e = static_scratch(plan->device, &scratch);
    if (e) return hip_fail((hipError_t)e, "fixed scratch address");
    return simulate_launch(plan, delta, beta, intensity, amplitude, scratch, stream);
}

msft_status msft_simulate_scan(msft_plan_t plan, const float* delta, const float* beta, void* workspace,
                               size_t ws_bytes, void* stream)
{
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (!delta || !beta || !workspace) return fail(MSFT_ERR_INVALID, "NULL argument");
    st = check_workspace(workspace, ws_bytes, plan->fwd_workspace);
    if (st != MSFT_OK) return st;
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    int e = launch_scan(plan->geo.g.precision, scan_args(plan, delta, beta, workspace), stream);
    if (e) return hip_fail((hipError_t)e, "scan launch");
    return ok();
}

msft_status msft_simulate_contract(msft_plan_t plan, const void* workspace, size_t ws_bytes,
                                   float* intensity, float* amplitude, void* stream)
{
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (!workspace || !intensity) return fail(MSFT_ERR_INVALID, "NULL argument");
    st = check_workspace(workspace, ws_bytes, plan->fwd_workspace);
    if (st != MSFT_OK) return st;
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    int e = launch_contraction(plan, workspace, intensity, amplitude, stream);
    if (e) return hip_fail((hipError_t)e, "forward launch");
    return ok();
}

int32_t msft_pixel_block(void) { return BLOCK_PIX; }

static msft_status batch_layout(const msft_request* reqs, int32_t n, std::vector<size_t>* offs,
                                size_t* total)
{
    if (n < 0 || (n > 0 && !reqs)) return fail(MSFT_ERR_INVALID, "bad request array");
    size_t off = 0;
    if (offs) offs->resize(n);
    for (int32_t r = 0; r < n; ++r) {
        msft_status st = check_runnable(reqs[r].plan);
        if (st != MSFT_OK) return st;
        if (reqs[r].plan->separable)
            return fail(MSFT_ERR_UNSUPPORTED, "batches take flat-detector plans only");
        if (offs) (*offs)[r] = off;
        off += align256(reqs[r].plan->dims.wtile_bytes());
    }
    *total = off;
    return MSFT_OK;
}

msft_status msft_batch_query(const msft_request* reqs, int32_t n, size_t* workspace_bytes)
{
    size_t total = 0;
    msft_status st = batch_layout(reqs, n, nullptr, &total);
    if (st != MSFT_OK) return st;
    if (workspace_bytes) *workspace_bytes = total;
    return ok();
}

msft_status msft_simulate_batch(const msft_request* reqs, int32_t n, void* workspace, size_t ws_bytes,
                                void* stream)
{
    std::vector<size_t> offs;
    size_t total = 0;
    msft_status st = batch_layout(reqs, n, &offs, &total);
    if (st != MSFT_OK) return st;
    if (n == 0) return ok();
    if (!workspace || !aligned256(workspace))
        return fail(MSFT_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < total) return fail(MSFT_ERR_BUSY, "workspace smaller than msft_batch_query");
    const int device = reqs[0].plan->device;
    const int precision = reqs[0].plan->geo.g.precision;
    std::vector<int32_t> b0(n), b1(n);
    for (int32_t r = 0; r < n; ++r) {
        const msft_request& q = reqs[r];
        if (q.plan->device != device) return fail(MSFT_ERR_INVALID, "requests span several devices");
        if (q.plan->geo.g.precision != precision)
            return fail(MSFT_ERR_INVALID, "requests mix precisions");
        if (!q.delta || !q.beta || !q.intensity)
            return fail(MSFT_ERR_INVALID, "request delta, beta, intensity must be non-NULL");
        const int64_t nb = q.plan->dims.nblocks;
        const int64_t lo = q.tile_begin < 0 ? 0 : q.tile_begin;
        const int64_t hi = q.tile_end < 0 ? nb : q.tile_end;
        if (lo > hi || hi > nb) return fail(MSFT_ERR_INVALID, "request tile range out of bounds");
        b0[r] = (int32_t)lo;
        b1[r] = (int32_t)hi;
    }
    DeviceScope ds(device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    uint8_t* ws = (uint8_t*)workspace;
    for (int32_t r = 0; r < n; ++r) {
        if (b1[r] == b0[r]) continue;
        const ScanArgs sa = scan_args(reqs[r].plan, reqs[r].delta, reqs[r].beta, ws + offs[r]);
        int e = launch_scan(precision, sa, stream);
        if (e) return hip_fail((hipError_t)e, "scan launch");
    }
    // Work items of the most expensive blocks first (cost ~ voxels per block).
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const Dims& da = reqs[a].plan->dims;
        const Dims& db = reqs[b].plan->dims;
        return (int64_t)da.x_pad * da.ny * da.nzb > (int64_t)db.x_pad * db.ny * db.nzb;
    });
    for (size_t k0 = 0; k0 < order.size(); k0 += MAX_BATCH) {
        BatchArgs b;
        std::memset(&b, 0, sizeof b);
        int32_t items = 0;
        int32_t nr = 0;
        for (size_t k = k0; k < order.size() && k < k0 + MAX_BATCH; ++k) {
            const int32_t r = order[k];
            if (b1[r] == b0[r]) continue;
            b.req[nr] = forward_args(reqs[r].plan, ws + offs[r], reqs[r].intensity, reqs[r].amplitude);
            b.block_begin[nr] = b0[r];
            b.item_begin[nr] = items;
            items += b1[r] - b0[r];
            ++nr;
        }
        b.nreq = nr;
        b.item_begin[nr] = items;
        if (items == 0) continue;
        // every plan of one precision is flat here, so all or none use the Gauss tiles
        int e = reqs[0].plan->dims.g3 ? launch_forward_batch_g3(b, stream)
                                      : launch_forward_batch(precision, b, stream);
        if (e) return hip_fail((hipError_t)e, "batch launch");
    }
    return ok();
}

msft_status msft_backward(msft_plan_t plan, const float* delta, const float* beta,
                          const float* amplitude, const float* grad_intensity, float* grad_delta,
                          float* grad_beta, void* workspace, size_t ws_bytes, void* stream)
{
    msft_status st = check_runnable(plan);
    if (st != MSFT_OK) return st;
    if (!delta || !beta || !amplitude || !grad_intensity || !grad_delta || !grad_beta || !workspace)
        return fail(MSFT_ERR_INVALID, "NULL argument");
    st = check_workspace(workspace, ws_bytes, plan->adj_workspace);
    if (st != MSFT_OK) return st;
    const Dims& d = plan->dims;
    const msft_geometry& g = plan->geo.g;
    const AdjDims ad = make_adj_dims(d);
    uint8_t* ws = (uint8_t*)workspace;
    AdjArgs a;
    a.q = plan->q_dev;
    a.h = (float*)ws;
    a.rpart = (float*)(ws + ad.h_bytes);
    a.npix = d.npix;
    a.npix_pad = d.nblocks * BLOCK_PIX;
    a.group_pix = ad.group_pix;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.nxc = d.nxc;
    a.nzb = d.nzb;
    a.nyb = ad.nyb;
    a.nsplit = ad.nsplit;
    a.xs0 = plan->geo.xs[0];
    a.ys0 = plan->geo.ys[0];
    a.zs0 = plan->geo.zs[0];
    a.dx = g.dx;
    a.dy = g.dy;
    a.dz = g.dz;
    FinArgs f;
    f.delta = delta;
    f.beta = beta;
    f.rpart = a.rpart;
    f.grad_delta = grad_delta;
    f.grad_beta = grad_beta;
    f.nx = d.nx;
    f.ny = d.ny;
    f.nz = d.nz;
    f.nxc = d.nxc;
    f.nzb = d.nzb;
    f.nsplit = ad.nsplit;
    f.strength = g.strength;
    f.dV = g.dx * g.dy * g.dz;
    f.k0dz = (2.0 * 3.14159265358979323846) / g.wavelength * g.dz;
    DeviceScope ds(plan->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    if (plan->separable) {
        // the two transposed contractions of the separable detector, then the same
        // column walk as the general adjoint (one pixel group)
        size_t k_off = 0, r_off = 0;
        sep_adj_layout(plan, &k_off, &r_off);
        const SepDims& sd = plan->sep;
        if (sd.gauss) {
            SepG3AdjArgs ga;
            ga.h = (const float*)ws;
            ga.tz = plan->tz;
            ga.tyT = plan->tyT;
            ga.txT = plan->txT;
            ga.kplain = (float*)(ws + k_off);
            ga.rpart = (float*)(ws + r_off);
            ga.n = sd.n;
            ga.npad = sd.npad;
            ga.nx = d.nx;
            ga.ny = d.ny;
            ga.nzb = d.nzb;
            ga.nz2 = d.nzb * ZB;
            ga.njc2 = sd.nic3;
            ga.nic3 = sd.nic3;
            ga.rows_pad = d.nxc * XC;
            f.rpart = ga.rpart;
            f.nsplit = SEPG_ADJ_SPLIT;
            int e = launch_adj_prep(amplitude, grad_intensity, (float*)ws, d.npix, d.npix, stream);
            if (!e) e = launch_sepg_adjoint(ga, stream);
            if (!e) e = launch_adj_finalize(f, stream);
            if (e) return hip_fail((hipError_t)e, "backward launch");
            return ok();
        }
        SepAdjArgs ka;
        ka.h = (const float*)ws;
        ka.tz = plan->tz;
        ka.tyT = plan->tyT;
        ka.ktiles = ws + k_off;
        ka.n = sd.n;
        ka.npad = sd.npad;
        ka.ny = d.ny;
        ka.nzb = d.nzb;
        ka.njc = sd.njc;
        Stage1Args ra;
        ra.wtiles = ws + k_off;
        ra.txa = plan->txT;
        ra.htiles = nullptr;
        ra.rplain = (float*)(ws + r_off);
        ra.n = d.nx;
        ra.ny = d.ny;
        ra.nxc = sd.nic;
        ra.nzb = d.nzb;
        ra.x_pad = sd.nic * XC;
        ra.nyc = 0;
        ra.nz2 = d.nzb * ZB;
        f.rpart = ra.rplain;
        f.nsplit = 1;
        int e = launch_adj_prep(amplitude, grad_intensity, (float*)ws, d.npix, d.npix, stream);
        if (!e) e = launch_sep_adjoint(ka, ra, ceil_div(d.nx, BLOCK_PIX), stream);
        if (!e) e = launch_adj_finalize(f, stream);
        if (e) return hip_fail((hipError_t)e, "backward launch");
        return ok();
    }
    int e = launch_backward(a, f, amplitude, grad_intensity, stream);
    if (e) return hip_fail((hipError_t)e, "backward launch");
    return ok();
}

const char* msft_status_str(msft_status s)
{
    switch (s) {
    case MSFT_OK: return "ok";
    case MSFT_ERR_INVALID: return "invalid argument";
    case MSFT_ERR_UNDERSAMPLED: return "voxel grid undersamples the detector's q range";
    case MSFT_ERR_NOMEM: return "out of memory";
    case MSFT_ERR_DEVICE: return "HIP runtime error";
    case MSFT_ERR_BUSY: return "workspace too small";
    case MSFT_ERR_UNSUPPORTED: return "unsupported for this plan";
    }
    return "unknown status";
}

const char* msft_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
