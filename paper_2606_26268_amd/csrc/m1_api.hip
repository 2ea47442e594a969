// m1_api.hip -- host side of the C ABI declared in include/m1.h: argument
// validation, the separable grid metric, buffer ownership, the step state
// machine and error reporting.  Kernels live in transport.hip, implicit.hip,
// diag.hip and mlp.hip.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "m1_internal.h"
#include "mlp_device.h"

namespace m1 {

// last error text of the calling thread, in a fixed buffer (setting it
// allocates nothing)
static thread_local char g_err[512];

void set_error(const char *msg) { std::snprintf(g_err, sizeof(g_err), "%s", msg); }
void set_error(const std::string &msg) { set_error(msg.c_str()); }

static m1_status fail(m1_status s, const std::string &msg)
{
    set_error(msg);
    return s;
}

// The C interface lets no exception through: a host allocation that fails
// inside the library (std::bad_alloc, or std::length_error for an absurd
// size) makes the call return M1_ENOMEM, with a message that itself
// allocates nothing.
static m1_status host_oom(const char *msg)
{
    set_error(msg);
    return M1_ENOMEM;
}

static m1_status hip_fail(hipError_t e, const char *what)
{
    return fail(M1_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// --------------------------------------------------------------------------
// grid metric (host, FP64)
// --------------------------------------------------------------------------

struct HostMetric {
    std::vector<double> winv[3], hp[3], hm[3], alo[3], ahi[3], trA[3], trB[3], hd[3], hI[3], hJ[3];
    std::vector<double> inv_reff, cot_eff, vol[3];
};

// lower / upper face and centre of (ghost) index t along d: periodic ghosts
// are shifted copies, outflow ghosts repeat the edge cell width
static void ghost_coords(const m1_ctx *c, int d, int t, double &lo, double &ce, double &hi)
{
    const int n = c->n[d];
    const std::vector<double> &x = c->faces[d];
    if (t >= 0 && t < n) {
        lo = x[t];
        hi = x[t + 1];
    } else if (c->bc[d][t < 0 ? 0 : 1] == M1_BC_PERIODIC) {
        int w = t, shift = 0;
        while (w < 0) { w += n; --shift; }
        while (w >= n) { w -= n; ++shift; }
        const double L = x[n] - x[0];
        lo = x[w] + shift * L;
        hi = x[w + 1] + shift * L;
    } else if (c->bc[d][t < 0 ? 0 : 1] == M1_BC_REFLECT) {
        // mirror image of the interior cell across the wall
        const int m = t < 0 ? -1 - t : 2 * n - 1 - t;
        const double wall = t < 0 ? x[0] : x[n];
        lo = 2.0 * wall - x[m + 1];
        hi = 2.0 * wall - x[m];
    } else if (t < 0) {
        const double h = x[1] - x[0];
        lo = x[0] + t * h;
        hi = lo + h;
    } else {
        const double h = x[n] - x[n - 1];
        lo = x[n] + (t - n) * h;
        hi = lo + h;
    }
    ce = 0.5 * (lo + hi);
}

static void build_metric(const m1_ctx *c, HostMetric &M)
{
    const int n0 = c->n[0], n1 = c->n[1];
    for (int d = 0; d < 3; ++d) {
        const int n = c->n[d];
        M.winv[d].assign(n + 4, 0.0);
        M.hp[d].assign(n + 4, 0.0);
        M.hm[d].assign(n + 4, 0.0);
        double plo, pce, phi;
        ghost_coords(c, d, -2, plo, pce, phi);
        for (int t = -1; t <= n + 1; ++t) {
            double lo, ce, hi;
            ghost_coords(c, d, t, lo, ce, hi);
            M.winv[d][t + 2] = 1.0 / (ce - pce);
            M.hp[d][t + 2] = hi - ce;
            M.hm[d][t + 2] = ce - lo;
            pce = ce;
        }
        M.alo[d].assign(n, 0.0);
        M.ahi[d].assign(n, 0.0);
        M.hd[d].assign(n, 0.0);
        M.vol[d].assign(n, 0.0);
        M.trA[d].assign(n0, 1.0);
        M.trB[d].assign(n1, 1.0);
        M.hI[d].assign(n0, 1.0);
        M.hJ[d].assign(n1, 1.0);
    }
    M.inv_reff.assign(n0, 0.0);
    M.cot_eff.assign(n1, 0.0);
    const std::vector<double> &x0 = c->faces[0], &x1 = c->faces[1], &x2 = c->faces[2];
    for (int d = 0; d < 3; ++d)
        for (int t = 0; t < c->n[d]; ++t) M.hd[d][t] = c->faces[d][t + 1] - c->faces[d][t];
    if (c->geom == M1_CARTESIAN) {
        for (int d = 0; d < 3; ++d)
            for (int t = 0; t < c->n[d]; ++t) {
                const double w = c->faces[d][t + 1] - c->faces[d][t];
                M.alo[d][t] = M.ahi[d][t] = 1.0 / w;
                M.vol[d][t] = w;
            }
    } else if (c->geom == M1_CYLINDRICAL) {   // (R, phi, z)
        for (int i = 0; i < n0; ++i) {
            const double a = x0[i], b = x0[i + 1], ring = 0.5 * (b * b - a * a);
            M.alo[0][i] = a / ring;
            M.ahi[0][i] = b / ring;
            M.trA[1][i] = (b - a) / ring;
            M.inv_reff[i] = (b - a) / ring;
            M.hI[1][i] = 0.5 * (a + b);
            M.vol[0][i] = ring;
        }
        for (int j = 0; j < n1; ++j) {
            const double w = x1[j + 1] - x1[j];
            M.alo[1][j] = M.ahi[1][j] = 1.0 / w;
            M.vol[1][j] = w;
        }
        for (int k = 0; k < c->n[2]; ++k) {
            const double w = x2[k + 1] - x2[k];
            M.alo[2][k] = M.ahi[2][k] = 1.0 / w;
            M.vol[2][k] = w;
        }
    } else {                                   // (r, theta, phi)
        for (int i = 0; i < n0; ++i) {
            const double a = x0[i], b = x0[i + 1];
            const double shell = (b * b * b - a * a * a) / 3.0, ring = 0.5 * (b * b - a * a);
            M.alo[0][i] = a * a / shell;
            M.ahi[0][i] = b * b / shell;
            M.trA[1][i] = ring / shell;
            M.trA[2][i] = ring / shell;
            M.inv_reff[i] = (b * b - a * a) / (2.0 * shell);
            M.hI[1][i] = 0.5 * (a + b);
            M.hI[2][i] = 0.5 * (a + b);
            M.vol[0][i] = shell;
        }
        for (int j = 0; j < n1; ++j) {
            const double a = x1[j], b = x1[j + 1], dmu = std::cos(a) - std::cos(b);
            M.alo[1][j] = std::sin(a) / dmu;
            M.ahi[1][j] = std::sin(b) / dmu;
            M.trB[2][j] = (b - a) / dmu;
            M.cot_eff[j] = (std::sin(b) - std::sin(a)) / dmu;
            M.hJ[2][j] = std::sin(0.5 * (a + b));
            M.vol[1][j] = dmu;
        }
        for (int k = 0; k < c->n[2]; ++k) {
            const double w = x2[k + 1] - x2[k];
            M.alo[2][k] = M.ahi[2][k] = 1.0 / w;
            M.vol[2][k] = w;
        }
    }
}

// upload all metric arrays into one device allocation, in both precisions
static m1_status upload_metric(m1_ctx *c, const HostMetric &M)
{
    std::vector<const std::vector<double> *> arrs;
    for (int d = 0; d < 3; ++d) {
        arrs.push_back(&M.winv[d]);
        arrs.push_back(&M.hp[d]);
        arrs.push_back(&M.hm[d]);
        arrs.push_back(&M.alo[d]);
        arrs.push_back(&M.ahi[d]);
        arrs.push_back(&M.trA[d]);
        arrs.push_back(&M.trB[d]);
        arrs.push_back(&M.hd[d]);
        arrs.push_back(&M.hI[d]);
        arrs.push_back(&M.hJ[d]);
    }
    arrs.push_back(&M.inv_reff);
    arrs.push_back(&M.cot_eff);
    const size_t na = arrs.size();
    std::vector<size_t> off64(na), off32(na), offv(3);
    size_t pos = 0;
    auto align = [](size_t p) { return (p + 255) & ~size_t(255); };
    for (size_t a = 0; a < na; ++a) { off64[a] = pos; pos = align(pos + arrs[a]->size() * 8); }
    for (size_t a = 0; a < na; ++a) { off32[a] = pos; pos = align(pos + arrs[a]->size() * 4); }
    for (int d = 0; d < 3; ++d) { offv[d] = pos; pos = align(pos + M.vol[d].size() * 8); }
    std::vector<unsigned char> host(pos, 0);
    for (size_t a = 0; a < na; ++a) {
        std::memcpy(&host[off64[a]], arrs[a]->data(), arrs[a]->size() * 8);
        float *f = reinterpret_cast<float *>(&host[off32[a]]);
        for (size_t t = 0; t < arrs[a]->size(); ++t) f[t] = float((*arrs[a])[t]);
    }
    for (int d = 0; d < 3; ++d) std::memcpy(&host[offv[d]], M.vol[d].data(), M.vol[d].size() * 8);
    hipError_t e = device_alloc(&c->metric_buf, pos);
    if (e != hipSuccess) return fail(M1_ENOMEM, "metric allocation failed");
    e = hipMemcpy(c->metric_buf, host.data(), pos, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "metric upload");
    unsigned char *base = static_cast<unsigned char *>(c->metric_buf);
    auto p64 = [&](size_t a) { return reinterpret_cast<const double *>(base + off64[a]); };
    auto p32 = [&](size_t a) { return reinterpret_cast<const float *>(base + off32[a]); };
    for (int d = 0; d < 3; ++d) {
        const size_t b = 10 * d;
        c->met64.winv[d] = p64(b + 0); c->met32.winv[d] = p32(b + 0);
        c->met64.hp[d] = p64(b + 1);   c->met32.hp[d] = p32(b + 1);
        c->met64.hm[d] = p64(b + 2);   c->met32.hm[d] = p32(b + 2);
        c->met64.alo[d] = p64(b + 3);  c->met32.alo[d] = p32(b + 3);
        c->met64.ahi[d] = p64(b + 4);  c->met32.ahi[d] = p32(b + 4);
        c->met64.trA[d] = p64(b + 5);  c->met32.trA[d] = p32(b + 5);
        c->met64.trB[d] = p64(b + 6);  c->met32.trB[d] = p32(b + 6);
        c->met64.hd[d] = p64(b + 7);   c->met32.hd[d] = p32(b + 7);
        c->met64.hI[d] = p64(b + 8);   c->met32.hI[d] = p32(b + 8);
        c->met64.hJ[d] = p64(b + 9);   c->met32.hJ[d] = p32(b + 9);
        c->vol_dev[d] = reinterpret_cast<double *>(base + offv[d]);
    }
    c->met64.inv_reff = p64(30); c->met32.inv_reff = p32(30);
    c->met64.cot_eff = p64(31);  c->met32.cot_eff = p32(31);
    for (int d = c->ndim; d < 3; ++d) c->ign[d] = M.alo[d][0] != M.ahi[d][0];
    return M1_OK;
}

static size_t elem_size(const m1_ctx *c) { return c->par.precision == M1_F32 ? 4 : 8; }

static long ncells(const m1_ctx *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }

// --------------------------------------------------------------------------
// static buffer of the allocation-free step
// --------------------------------------------------------------------------

// One copy per device, held by every device that loads the library until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// a device address: its device address is looked up once per device
// (noalloc_setup, from m1_create with that device current) and only that
// pointer is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[M1_NOALLOC_MAX_BYTES];

constexpr int NOALLOC_DEVICES = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_DEVICES] = {};
static hipError_t g_noalloc_err[NOALLOC_DEVICES] = {};
static bool g_noalloc_done[NOALLOC_DEVICES] = {};

static void noalloc_setup(int dev)
{
    if (dev < 0 || dev >= NOALLOC_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_done[dev]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_noalloc_err[dev] = e;
    g_noalloc_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_noalloc_done[dev] = true;
}

static void *noalloc_ptr(int dev)
{
    if (dev < 0 || dev >= NOALLOC_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_done[dev] ? g_noalloc_ptr[dev] : nullptr;
}

} // namespace m1

using namespace m1;

extern "C" {

m1_status m1_params_default(double c_hat, m1_params *p)
{
    if (!p) return fail(M1_EINVAL, "m1_params_default: NULL output");
    p->c = c_hat;
    p->a_rad = 1.0;
    p->gamma = 5.0 / 3.0;
    p->precision = M1_P64;
    p->e_floor = 1e-30;
    p->recon = M1_RECON_FPRESERVE;
    p->riemann = M1_RIEMANN_HLL;
    p->absorb_only = 0;
    p->second_order = 0;
    p->limiter = M1_LIMITER_PLM;
    p->stream_reads = M1_STREAM_AUTO;
    return M1_OK;
}

m1_status m1_create(const m1_grid *g, m1_geometry geom, double c_hat, const m1_params *p, m1_ctx **out) try
{
    if (!g || !out) return fail(M1_EINVAL, "m1_create: NULL argument");
    *out = nullptr;
    if (g->ndim < 1 || g->ndim > 3) return fail(M1_EINVAL, "m1_create: ndim must be 1, 2 or 3");
    if (geom < M1_CARTESIAN || geom > M1_SPHERICAL) return fail(M1_EINVAL, "m1_create: unknown geometry");
    if (!(c_hat > 0.0) || !std::isfinite(c_hat)) return fail(M1_EINVAL, "m1_create: c_hat must be > 0");
    long total = 1;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1) return fail(M1_EINVAL, "m1_create: n[d] must be >= 1");
        if (d >= g->ndim && g->n[d] != 1) return fail(M1_EINVAL, "m1_create: n[d] must be 1 for inactive d");
        if (!g->faces[d]) return fail(M1_EINVAL, "m1_create: NULL faces");
        for (int s = 0; s < 2; ++s)
            if (g->bc[d][s] < M1_BC_PERIODIC || g->bc[d][s] > M1_BC_FIXED)
                return fail(M1_EINVAL, "m1_create: unknown boundary condition");
        if ((g->bc[d][0] == M1_BC_PERIODIC) != (g->bc[d][1] == M1_BC_PERIODIC))
            return fail(M1_EINVAL, "m1_create: periodic boundaries must be paired");
        if (d < g->ndim && g->n[d] < 2 && (g->bc[d][0] == M1_BC_REFLECT || g->bc[d][1] == M1_BC_REFLECT))
            return fail(M1_EINVAL, "m1_create: a reflective direction needs at least 2 cells");
        for (int t = 0; t < g->n[d]; ++t)
            if (!(g->faces[d][t + 1] > g->faces[d][t]))
                return fail(M1_EINVAL, "m1_create: faces must be strictly increasing");
        total *= g->n[d];
    }
    // cell indices are 32-bit in the kernels, including the padded last
    // block of a launch
    if (total > (1L << 31) - (1L << 16)) return fail(M1_EINVAL, "m1_create: too many cells (at most 2^31 - 2^16)");
    if (geom != M1_CARTESIAN && g->faces[0][0] < 0.0)
        return fail(M1_EINVAL, "m1_create: negative radius");
    if (geom == M1_SPHERICAL && (g->faces[1][0] < 0.0 || g->faces[1][g->n[1]] > M_PI + 1e-12))
        return fail(M1_EINVAL, "m1_create: theta outside [0, pi]");
    m1_params par;
    m1_params_default(c_hat, &par);
    if (p) par = *p;
    if (par.precision != M1_P64 && par.precision != M1_F32)
        return fail(M1_EINVAL, "m1_create: unknown precision");
    if (par.recon < M1_RECON_FPRESERVE || par.recon > M1_RECON_CLIP || par.riemann < M1_RIEMANN_HLL ||
        par.riemann > M1_RIEMANN_LF)
        return fail(M1_EINVAL, "m1_create: unknown reconstruction or Riemann solver");
    if (par.absorb_only != 0 && par.absorb_only != 1)
        return fail(M1_EINVAL, "m1_create: absorb_only must be 0 or 1");
    if (par.second_order != 0 && par.second_order != 1)
        return fail(M1_EINVAL, "m1_create: second_order must be 0 or 1");
    if (par.limiter != M1_LIMITER_PLM && par.limiter != M1_LIMITER_LIMO3)
        return fail(M1_EINVAL, "m1_create: unknown limiter");
    if (par.stream_reads < M1_STREAM_AUTO || par.stream_reads > M1_STREAM_OFF)
        return fail(M1_EINVAL, "m1_create: unknown stream_reads mode");
    if (!(par.c > 0.0) || !(par.gamma > 1.0) || !(par.a_rad > 0.0))
        return fail(M1_EINVAL, "m1_create: c, a_rad must be > 0 and gamma > 1");
    m1_ctx *c = new (std::nothrow) m1_ctx();
    if (!c) return fail(M1_ENOMEM, "m1_create: host allocation failed");
    try {
        c->ndim = g->ndim;
        c->geom = geom;
        c->c_hat = c_hat;
        c->par = par;
        for (int d = 0; d < 3; ++d) {
            c->n[d] = g->n[d];
            c->bc[d][0] = g->bc[d][0];
            c->bc[d][1] = g->bc[d][1];
            c->faces[d].assign(g->faces[d], g->faces[d] + g->n[d] + 1);
        }
        hipGetDevice(&c->device);
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cu > 0)
            c->cus = cu;
        noalloc_setup(c->device);
        c->op.kind = OPK_CONST;
        HostMetric M;
        build_metric(c, M);
        m1_status s = upload_metric(c, M);
        if (s != M1_OK) {
            m1_destroy(c);
            return s;
        }
    } catch (const std::exception &) {
        m1_destroy(c);        // the partly built context goes with the error
        return host_oom("m1_create: host allocation failed");
    }
    *out = c;
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_create: host allocation failed");
}

m1_status m1_destroy(m1_ctx *c)
{
    if (!c) return M1_OK;
    if (c->metric_buf) hipFree(c->metric_buf);
    if (c->scratch) hipFree(c->scratch);
    if (c->table_dev) hipFree(c->table_dev);
    if (c->mlp_dev) hipFree(c->mlp_dev);
    if (c->rk2_save) hipFree(c->rk2_save);
    delete c;
    return M1_OK;
}

m1_status m1_set_stream(m1_ctx *c, void *stream)
{
    if (!c) return fail(M1_EINVAL, "m1_set_stream: NULL context");
    c->stream = static_cast<hipStream_t>(stream);
    return M1_OK;
}

static bool aligned(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

m1_status m1_bind_state(m1_ctx *c, const m1_fields *f) try
{
    if (!c || !f) return fail(M1_EINVAL, "m1_bind_state: NULL argument");
    const void *ptrs[9] = {f->E, f->Fx, f->Fy, f->Fz, f->rho, f->mx, f->my, f->mz, f->Eg};
    for (int a = 0; a < 9; ++a)
        if (!aligned(ptrs[a])) return fail(M1_EINVAL, "m1_bind_state: NULL or non-256-byte-aligned pointer");
    const long N = ncells(c);
    const size_t es = elem_size(c);
    const size_t per = ((N * es + 255) / 256) * 256;
    const size_t ndiag = (1024 + 1) * 8;
    // transported state and optical depth per group, the rho kappa_P cache
    const int G = c->grp.m;
    const size_t nfield = 5 * (size_t)G + 1;
    const size_t bytes = nfield * per + CNT_BYTES + ndiag * sizeof(double);
    // allocate the new buffers first and swap them in only when every
    // allocation succeeded: a failed rebind leaves the previous binding (its
    // buffers and fields) intact and usable
    void *nscr = nullptr, *nrk = nullptr;
    hipError_t e = device_alloc(&nscr, bytes);
    if (e != hipSuccess) return fail(M1_ENOMEM, "m1_bind_state: scratch allocation failed");
    size_t rad = 0;
    if (c->par.second_order) {
        // the first-stage state of m1_step_rk2: the four radiation fields of
        // all groups (group-major, as the bound arrays), then mx, my, mz, E_g
        rad = ((size_t(G) * N * es + 255) / 256) * 256;
        e = device_alloc(&nrk, 4 * rad + 4 * N * sizeof(double));
        if (e != hipSuccess) {
            hipFree(nscr);
            return fail(M1_ENOMEM, "m1_bind_state: second-order buffer allocation failed");
        }
    }
    if (c->scratch) hipFree(c->scratch);
    if (c->rk2_save) hipFree(c->rk2_save);
    c->scratch = nscr;
    c->rk2_save = nrk;
    c->rk2_rad_bytes = rad;
    unsigned char *b = static_cast<unsigned char *>(c->scratch);
    // layout: star (group g, field v) at (4 g + v) per, tau of group g at
    // (4 G + g) per, rho kappa_P at 5 G per
    c->plane_bytes = per;
    for (int v = 0; v < 4; ++v) c->star[v] = b + v * per;
    c->tau = b + 4 * (size_t)G * per;
    c->rkp = b + 5 * (size_t)G * per;
    c->cnt = reinterpret_cast<unsigned long long *>(b + nfield * per);
    c->partials = reinterpret_cast<double *>(b + nfield * per + CNT_BYTES);
    c->f = *f;
    c->bound = true;
    c->transported = false;
    e = hipMemsetAsync(c->cnt, 0, CNT_BYTES, c->stream);
    if (e == hipSuccess) e = launch_opacity_init(c);
    if (e != hipSuccess) {
        // the new buffers stay owned by the context; the binding is not usable
        c->bound = false;
        return hip_fail(e, "m1_bind_state: counter reset / opacity cache");
    }
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_bind_state: host allocation failed");
}

static m1_status refresh(m1_ctx *c)
{
    if (!c->bound) return M1_OK;
    hipError_t e = launch_opacity_init(c);
    if (e != hipSuccess) return hip_fail(e, "opacity cache");
    return M1_OK;
}

m1_status m1_set_opacity_model(m1_ctx *c, int kind, const double *p)
{
    if (!c || !p) return fail(M1_EINVAL, "m1_set_opacity_model: NULL argument");
    if (kind == M1_OPAC_CONSTANT) {
        if (p[0] < 0 || p[1] < 0 || p[2] < 0) return fail(M1_EINVAL, "opacities must be >= 0");
        c->op.kind = OPK_CONST;
        c->op.kP = p[0];
        c->op.kR = p[1];
        c->op.sigma = p[2];
    } else if (kind == M1_OPAC_POWERLAW) {
        if (!(p[0] >= 0) || !(p[1] > 0) || !(p[3] > 0) || p[5] < 0)
            return fail(M1_EINVAL, "power law needs k0 >= 0, rho0 > 0, T0 > 0, sigma >= 0");
        c->op.kind = OPK_POWERLAW;
        c->op.k0 = p[0];
        c->op.rho0 = p[1];
        c->op.alpha = p[2];
        c->op.T0 = p[3];
        c->op.beta = p[4];
        c->op.sigma = p[5];
    } else {
        return fail(M1_EINVAL, "m1_set_opacity_model: unknown kind");
    }
    opacity_f32(c->op);
    return refresh(c);
}

m1_status m1_set_opacity_table(m1_ctx *c, int nr, int nt, double lr0, double lr1, double lt0, double lt1,
                               double lr_off, double lt_off, const float *kP, const float *kR, double sigma) try
{
    if (!c || !kP || !kR) return fail(M1_EINVAL, "m1_set_opacity_table: NULL argument");
    if (nr < 2 || nt < 2 || !(lr1 > lr0) || !(lt1 > lt0) || sigma < 0)
        return fail(M1_EINVAL, "m1_set_opacity_table: need nr, nt >= 2, increasing axes, sigma >= 0");
    const size_t n = size_t(nr) * nt;
    // device layout: the two tables as given, then (16-byte aligned) one
    // record per table cell with its four node values of kappa_P and of
    // kappa_R, so that a lookup reads two 16-byte words instead of
    // gathering eight values from four rows
    const size_t ncell = size_t(nr - 1) * (nt - 1), off = (2 * n + 3) & ~size_t(3);
    std::vector<float> host(off + 8 * ncell, 0.0f);
    std::copy(kP, kP + n, host.begin());
    std::copy(kR, kR + n, host.begin() + n);
    for (int j = 0; j + 1 < nt; ++j)
        for (int i = 0; i + 1 < nr; ++i) {
            const size_t o = size_t(j) * nr + i;
            float *r = &host[off + 8 * (size_t(j) * (nr - 1) + i)];
            const size_t node[4] = {o, o + 1, o + nr, o + nr + 1};
            for (int q = 0; q < 4; ++q) {
                r[q] = kP[node[q]];
                r[4 + q] = kR[node[q]];
            }
        }
    // the new table is uploaded before the old one is released: on failure
    // the context keeps its previous opacity source unchanged
    float *tab = nullptr;
    hipError_t e = device_alloc(reinterpret_cast<void **>(&tab), host.size() * sizeof(float));
    if (e != hipSuccess) return fail(M1_ENOMEM, "m1_set_opacity_table: allocation failed");
    e = hipMemcpy(tab, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(tab);
        return hip_fail(e, "m1_set_opacity_table: upload");
    }
    if (c->table_dev) hipFree(c->table_dev);
    c->table_dev = tab;
    c->op.kind = OPK_TABLE;
    c->op.nr = nr;
    c->op.nt = nt;
    c->op.lr0 = lr0;
    c->op.lr1 = lr1;
    c->op.lt0 = lt0;
    c->op.lt1 = lt1;
    c->op.lr_inv = 1.0 / (lr1 - lr0);
    c->op.lt_inv = 1.0 / (lt1 - lt0);
    c->op.lr_off = lr_off;
    c->op.lt_off = lt_off;
    c->op.tab_kP = c->table_dev;
    c->op.tab_kR = c->table_dev + n;
    c->op.tab_cells = c->table_dev + off;
    c->op.sigma = sigma;
    opacity_f32(c->op);
    return refresh(c);
} catch (const std::exception &) {
    return host_oom("m1_set_opacity_table: host allocation failed");
}

m1_status m1_set_opacity_mlp(m1_ctx *c, const m1_mlp *w) try
{
    if (!c || !w || !w->theta) return fail(M1_EINVAL, "m1_set_opacity_mlp: NULL argument");
    if (!c->table_dev) return fail(M1_ESTATE, "m1_set_opacity_mlp: set the table first (input axes)");
    if (!(w->norm[1] > 0) || !(w->norm[3] > 0)) return fail(M1_EINVAL, "m1_set_opacity_mlp: std must be > 0");
    if (mlp_pack(c, w->theta, w->norm) != 0) return M1_EDEVICE;
    c->op.kind = OPK_MLP;
    return refresh(c);
} catch (const std::exception &) {
    return host_oom("m1_set_opacity_mlp: host allocation failed");
}

m1_status m1_mlp_train(m1_ctx *c, const m1_train_cfg *cfg, m1_train_report *rep) try
{
    if (!c || !cfg || !rep || !cfg->samples || !cfg->theta_init)
        return fail(M1_EINVAL, "m1_mlp_train: NULL argument");
    if (!c->table_dev) return fail(M1_ESTATE, "m1_mlp_train: set the table first (training targets)");
    if (cfg->batch < 64 || cfg->batch > 4096 || cfg->batch % 64 || cfg->n_train < cfg->batch ||
        cfg->n_eval < 1 || cfg->steps < 1 || !(cfg->lr > 0) || cfg->lr_final < 0 ||
        (cfg->keep_init != 0 && cfg->keep_init != 1))
        return fail(M1_EINVAL, "m1_mlp_train: bad configuration");
    int r = mlp_train(c, cfg, rep);
    if (r != 0) return r < 0 ? m1_status(r) : M1_EDEVICE;
    c->op.kind = OPK_MLP;
    return refresh(c);
} catch (const std::exception &) {
    return host_oom("m1_mlp_train: host allocation failed");
}

m1_status m1_mlp_get(m1_ctx *c, float *theta, double *norm) try
{
    if (!c || !theta || !norm) return fail(M1_EINVAL, "m1_mlp_get: NULL argument");
    if (c->mlp_theta.size() != M1_MLP_NPARAM) return fail(M1_ESTATE, "m1_mlp_get: no network set");
    std::memcpy(theta, c->mlp_theta.data(), M1_MLP_NPARAM * sizeof(float));
    for (int i = 0; i < 4; ++i) norm[i] = c->op.norm[i];
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_mlp_get: host allocation failed");
}

m1_status m1_mlp_gradient(m1_ctx *c, const float *samples, long n, const float *theta, float *grad,
                          double *loss) try
{
    if (!c || !samples || !theta || !grad || !loss) return fail(M1_EINVAL, "m1_mlp_gradient: NULL argument");
    if (n < 64 || n % 64) return fail(M1_EINVAL, "m1_mlp_gradient: n must be a positive multiple of 64");
    if (!c->table_dev || c->mlp_theta.size() != M1_MLP_NPARAM)
        return fail(M1_ESTATE, "m1_mlp_gradient: set the table and a network first");
    int r = mlp_gradient(c, samples, n, theta, grad, loss);
    if (r != 0) return r < 0 ? m1_status(r) : M1_EDEVICE;
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_mlp_gradient: host allocation failed");
}

m1_status m1_opacity_eval(m1_ctx *c, long n, const double *rho, const double *T, double *kP, double *kR)
{
    if (!c || n < 0 || (n > 0 && (!rho || !T || !kP || !kR))) return fail(M1_EINVAL, "m1_opacity_eval: bad argument");
    if (c->grp.m > 1) return fail(M1_ENOTSUP, "m1_opacity_eval: the gray opacity model is unused with groups");
    hipError_t e = launch_opacity_eval(c, n, rho, T, kP, kR);
    if (e != hipSuccess) return hip_fail(e, "m1_opacity_eval");
    return M1_OK;
}

m1_status m1_max_dt(const m1_ctx *c, double cfl, double *dt)
{
    if (!c || !dt || !(cfl > 0)) return fail(M1_EINVAL, "m1_max_dt: bad argument");
    HostMetric M;
    build_metric(c, M);
    double worst = 0.0;
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                const int idx[3] = {i, j, k};
                double s = 0.0;
                // extent = (radius factor x sine factor) x coordinate width
                for (int d = 0; d < c->ndim; ++d)
                    s += 1.0 / (M.hI[d][i] * M.hJ[d][j] * M.hd[d][idx[d]]);
                worst = s > worst ? s : worst;
            }
    *dt = cfl / (c->c_hat * worst);
    return M1_OK;
}

m1_status m1_set_groups(m1_ctx *c, int m, const double *edges, const double *kP, const double *kR,
                        double sigma) try
{
    if (!c) return fail(M1_EINVAL, "m1_set_groups: NULL context");
    if (c->bound) return fail(M1_ESTATE, "m1_set_groups: call before m1_bind_state");
    if (m < 1 || m > M1_MAX_GROUPS) return fail(M1_EINVAL, "m1_set_groups: need 1 <= m <= M1_MAX_GROUPS");
    if (m == 1) {
        c->grp.m = 1;
        return M1_OK;
    }
    if (!edges || !kP || !kR) return fail(M1_EINVAL, "m1_set_groups: NULL array");
    for (int g = 0; g + 1 < m; ++g)
        if (!(edges[g] > 0) || !std::isfinite(edges[g]) || (g > 0 && !(edges[g] > edges[g - 1])))
            return fail(M1_EINVAL, "m1_set_groups: edges must be positive and increasing");
    for (int g = 0; g < m; ++g)
        if (!(kP[g] >= 0) || !(kR[g] >= 0) || !std::isfinite(kP[g]) || !std::isfinite(kR[g]))
            return fail(M1_EINVAL, "m1_set_groups: opacities must be finite and >= 0");
    if (!(sigma >= 0)) return fail(M1_EINVAL, "m1_set_groups: sigma must be >= 0");
    c->grp.m = m;
    for (int g = 0; g < m; ++g) {
        c->grp.edges[g] = g + 1 < m ? edges[g] : 0.0;
        c->grp.kP[g] = kP[g];
        c->grp.kR[g] = kR[g];
    }
    c->grp.sigma = sigma;
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_set_groups: host allocation failed");
}

// every fixed side has its ghost state
static bool fixed_states_ready(const m1_ctx *c)
{
    for (int d = 0; d < c->ndim; ++d)
        for (int s = 0; s < 2; ++s)
            if (c->bc[d][s] == M1_BC_FIXED && !c->bc_state_set[d][s]) return false;
    return true;
}

m1_status m1_set_boundary_state(m1_ctx *c, int dir, int side, const double state[4])
{
    if (!c || !state) return fail(M1_EINVAL, "m1_set_boundary_state: NULL argument");
    if (dir < 0 || dir > 2 || side < 0 || side > 1)
        return fail(M1_EINVAL, "m1_set_boundary_state: dir must be 0..2 and side 0 or 1");
    if (c->bc[dir][side] != M1_BC_FIXED)
        return fail(M1_EINVAL, "m1_set_boundary_state: that side is not a fixed boundary");
    const double F2 = state[1] * state[1] + state[2] * state[2] + state[3] * state[3];
    if (!(state[0] > 0) || !std::isfinite(state[0]) || !(F2 <= state[0] * state[0]))
        return fail(M1_EINVAL, "m1_set_boundary_state: need E > 0 and |F| <= E");
    for (int v = 0; v < 4; ++v) c->bc_state[dir][side][v] = state[v];
    c->bc_state_set[dir][side] = true;
    return M1_OK;
}

m1_status m1_set_irradiation(m1_ctx *c, const double *q)
{
    if (!c) return fail(M1_EINVAL, "m1_set_irradiation: NULL context");
    if (q && reinterpret_cast<uintptr_t>(q) % alignof(double))
        return fail(M1_EINVAL, "m1_set_irradiation: misaligned array");
    c->irr = q;
    return M1_OK;
}

m1_status m1_step_explicit(m1_ctx *c, double dt)
{
    if (!c) return fail(M1_EINVAL, "m1_step_explicit: NULL context");
    if (!c->bound) return fail(M1_ESTATE, "m1_step_explicit: no state bound");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(M1_EINVAL, "m1_step_explicit: dt must be > 0");
    if (!fixed_states_ready(c)) return fail(M1_ESTATE, "m1_step_explicit: a fixed boundary has no state");
    hipError_t e = launch_transport(c, dt);
    if (e != hipSuccess) return hip_fail(e, "m1_step_explicit launch");
    c->transported = true;
    return M1_OK;
}

m1_status m1_step_implicit(m1_ctx *c, double dt)
{
    if (!c) return fail(M1_EINVAL, "m1_step_implicit: NULL context");
    if (!c->bound || !c->transported)
        return fail(M1_ESTATE, "m1_step_implicit: must follow m1_step_explicit");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(M1_EINVAL, "m1_step_implicit: dt must be > 0");
    hipError_t e = launch_implicit(c, dt);
    if (e != hipSuccess) return hip_fail(e, "m1_step_implicit launch");
    c->transported = false;
    return M1_OK;
}

m1_status m1_step_noalloc(m1_ctx *c, const m1_fields *f, double dt)
{
    // no allocation on any path: errors are literal or formatted into a
    // stack buffer, the launchers keep their own state in fixed tables
    if (!c || !f) {
        set_error("m1_step_noalloc: NULL argument");
        return M1_EINVAL;
    }
    const void *ptrs[9] = {f->E, f->Fx, f->Fy, f->Fz, f->rho, f->mx, f->my, f->mz, f->Eg};
    for (int a = 0; a < 9; ++a)
        if (!aligned(ptrs[a])) {
            set_error("m1_step_noalloc: NULL or non-256-byte-aligned pointer");
            return M1_EINVAL;
        }
    if (!(dt > 0) || !std::isfinite(dt)) {
        set_error("m1_step_noalloc: dt must be > 0");
        return M1_EINVAL;
    }
    if (c->grp.m > 1) {
        set_error("m1_step_noalloc: gray states only (no frequency groups)");
        return M1_ENOTSUP;
    }
    if (!fixed_states_ready(c)) {
        set_error("m1_step_noalloc: a fixed boundary has no state");
        return M1_ESTATE;
    }
    const size_t per = ((size_t(ncells(c)) * elem_size(c) + 255) / 256) * 256;
    const size_t need = 6 * per + CNT_BYTES;
    if (need > size_t(M1_NOALLOC_MAX_BYTES)) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "m1_step_noalloc: the grid needs %zu bytes of scratch, the static buffer holds %zu",
                      need, size_t(M1_NOALLOC_MAX_BYTES));
        set_error(msg);
        return M1_EINVAL;
    }
    unsigned char *base = static_cast<unsigned char *>(noalloc_ptr(c->device));
    if (!base) {
        set_error("m1_step_noalloc: the static scratch buffer has no device address on this device");
        return M1_EDEVICE;
    }
    // the launchers read the binding from the context: point it at the
    // caller's arrays and the static buffer for this call, then restore it
    const m1_fields f0 = c->f;
    void *const star0[4] = {c->star[0], c->star[1], c->star[2], c->star[3]};
    void *const tau0 = c->tau, *const rkp0 = c->rkp;
    unsigned long long *const cnt0 = c->cnt;
    const size_t plane0 = c->plane_bytes;
    const bool bound0 = c->bound, transported0 = c->transported;
    c->f = *f;
    for (int v = 0; v < 4; ++v) c->star[v] = base + v * per;
    c->tau = base + 4 * per;
    c->rkp = base + 5 * per;
    c->cnt = reinterpret_cast<unsigned long long *>(base + 6 * per);
    c->plane_bytes = per;
    // the counters start at zero; everything else is written before it is read
    hipError_t e = launch_zero_words(c->cnt, CNT_BYTES / sizeof(unsigned long long), c->stream);
    if (e == hipSuccess) e = launch_opacity_init(c);
    if (e == hipSuccess) e = launch_transport(c, dt);
    if (e == hipSuccess) e = launch_implicit(c, dt);
    c->f = f0;
    for (int v = 0; v < 4; ++v) c->star[v] = star0[v];
    c->tau = tau0;
    c->rkp = rkp0;
    c->cnt = cnt0;
    c->plane_bytes = plane0;
    c->bound = bound0;
    c->transported = transported0;
    if (e != hipSuccess) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "m1_step_noalloc launch: %s", hipGetErrorString(e));
        set_error(msg);
        return M1_EDEVICE;
    }
    return M1_OK;
}

m1_status m1_step_rk2(m1_ctx *c, double dt)
{
    if (!c) return fail(M1_EINVAL, "m1_step_rk2: NULL context");
    if (!c->bound) return fail(M1_ESTATE, "m1_step_rk2: no state bound");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(M1_EINVAL, "m1_step_rk2: dt must be > 0");
    if (!fixed_states_ready(c)) return fail(M1_ESTATE, "m1_step_rk2: a fixed boundary has no state");
    if (!c->rk2_save)
        return fail(M1_ESTATE, "m1_step_rk2: create the context with m1_params.second_order = 1");
    const size_t per = c->rk2_rad_bytes;
    // U1 = S(T(U^n)) into the save buffer (the caller's arrays keep U^n),
    // then U2 = S(T(U1)) written directly as (U^n + U2) / 2, the opacity
    // cache following each stage's written state
    unsigned char *sv = static_cast<unsigned char *>(c->rk2_save);
    const void *u1[4] = {sv, sv + per, sv + 2 * per, sv + 3 * per};
    hipError_t e = launch_transport(c, dt);
    if (e == hipSuccess) e = launch_implicit_rk2(c, dt, 1);
    if (e == hipSuccess) e = launch_transport_from(c, dt, u1);
    if (e == hipSuccess) e = launch_implicit_rk2(c, dt, 2);
    if (e != hipSuccess) return hip_fail(e, "m1_step_rk2 stage");
    c->transported = false;
    return M1_OK;
}

m1_status m1_transported(m1_ctx *c, void **E, void **Fx, void **Fy, void **Fz)
{
    if (!c || !E || !Fx || !Fy || !Fz) return fail(M1_EINVAL, "m1_transported: NULL argument");
    if (!c->bound) return fail(M1_ESTATE, "m1_transported: no state bound");
    if (c->grp.m > 1) return fail(M1_ENOTSUP, "m1_transported: gray states only");
    *E = c->star[0];
    *Fx = c->star[1];
    *Fy = c->star[2];
    *Fz = c->star[3];
    return M1_OK;
}

m1_status m1_refresh_opacity(m1_ctx *c)
{
    if (!c) return fail(M1_EINVAL, "m1_refresh_opacity: NULL context");
    if (!c->bound) return fail(M1_ESTATE, "m1_refresh_opacity: no state bound");
    return refresh(c);
}

m1_status m1_sync(m1_ctx *c)
{
    if (!c) return fail(M1_EINVAL, "m1_sync: NULL context");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "m1_sync");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "m1_sync");
    return M1_OK;
}

m1_status m1_diagnostics(m1_ctx *c, m1_diag *out) try
{
    if (!c || !out) return fail(M1_EINVAL, "m1_diagnostics: NULL argument");
    if (!c->bound) return fail(M1_ESTATE, "m1_diagnostics: no state bound");
    double v[8];
    hipError_t e = launch_diag(c, v);
    if (e != hipSuccess) return hip_fail(e, "m1_diagnostics");
    std::vector<unsigned long long> slots(CNT_BYTES / sizeof(unsigned long long));
    e = hipMemcpy(slots.data(), c->cnt, CNT_BYTES, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "m1_diagnostics counters");
    unsigned long long cnt[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i)
        for (int s = 0; s < CNT_SLOTS; ++s) cnt[i] += slots[(size_t(i) * CNT_SLOTS + s) * CNT_STRIDE];
    out->rad_energy = v[0];
    out->total_energy = v[1];
    out->momentum[0] = v[2];
    out->momentum[1] = v[3];
    out->momentum[2] = v[4];
    out->min_E = v[5];
    out->max_f = v[6];
    for (int i = 0; i < 4; ++i) out->counters[i] = (long long)cnt[i];
    return M1_OK;
} catch (const std::exception &) {
    return host_oom("m1_diagnostics: host allocation failed");
}

const char *m1_last_error(void) { return g_err; }

} // extern "C"
