// implicit.hip -- implicit radiation-matter step and the opacity cache.
//
// Per cell (Sect. 2.8): T^n from the gas energy, the 2x2 backward-Euler
// system of Eq. implicit_matrix solved analytically in FP64, flux damping of
// Eq. source_discrete2, the gas total energy and momentum from the rescaled
// conservation laws (Sect. 2.7), f <= 1, and the opacity cache (rho kappa_P,
// optical depth rho chi h_max) re-evaluated at the new temperature for the
// next transport and implicit steps.
#include "m1_internal.h"
#include "m1_device.h"
#include "opacity_device.h"
#include "mlp_device.h"

namespace m1 {

template <typename R>
struct IArgs {
    R *E, *Fx, *Fy, *Fz;              // caller's radiation (written)
    const R *Es, *Fxs, *Fys, *Fzs;    // transported state
    const double *rho;
    double *mx, *my, *mz, *Eg;
    R *rkp, *tau;                     // opacity cache (read at T^n, written at T^{n+1})
    int n[3];
    int ndim;
    CellIndex ix;
    Metric<R> m;
    OpacityParams op;
    ImplicitConsts k;
    const double *irr;                // irradiation heating per cell, or null
    int absorb;                       // absorption without emission
    const double *gin[4];             // gas read (mx, my, mz, E_g); the written arrays in place
    const R *ravg[4];                 // second-order step: radiation written as (ravg + new) / 2, or null
    const double *gavg[4];            // and the gas likewise
    unsigned long long *cnt;
};

// largest cell extent over the active directions (optical depth of a cell)
template <typename R>
__device__ __forceinline__ R cell_hmax(const Metric<R> &m, int ndim, int i, int j, int k)
{
    R h = m.hd[0][i] * m.hI[0][i] * m.hJ[0][j];
    if (ndim >= 2) {
        const R h1 = m.hd[1][j] * m.hI[1][i] * m.hJ[1][j];
        h = h1 > h ? h1 : h;
    }
    if (ndim >= 3) {
        const R h2 = m.hd[2][k] * m.hI[2][i] * m.hJ[2][j];
        h = h2 > h ? h2 : h;
    }
    return h;
}

// Gas temperature with the reciprocal density supplied:
// T = (E_g - |m|^2 / (2 rho)) (gamma - 1) / rho.
// Written with explicit fused multiply-adds, so that every inlined copy
// rounds the same way whatever the compiler would contract around it.
__device__ __forceinline__ double gas_T_r(double inv_rho, double mx, double my, double mz, double Eg,
                                          double gm1)
{
    const double m2 = __builtin_fma(mx, mx, __builtin_fma(my, my, mz * mz));
    return __builtin_fma(-0.5 * inv_rho, m2, Eg) * (gm1 * inv_rho);
}

// Gas temperature of a stored state, in exactly the arithmetic the implicit
// step uses for the temperature at which it refreshes the opacity cache, so
// that a cache derived from a stored state (binding, refresh) equals the one
// the step left: a state saved and bound again continues bit for bit.
__device__ __forceinline__ double gas_T_stored(double rho, double mx, double my, double mz, double Eg, double gm1)
{
    return gas_T_r(Num<double>::rcp(rho), mx, my, mz, Eg, gm1);
}

// One opacity-cache entry: the absorption rate rho kappa_P and the cell's
// optical depth rho (kappa_R + sigma) h.  Contraction is off here, so the
// sum cannot fuse with the last product of the opacity evaluation in one
// kernel and not in another: the implicit step and the refresh from a stored
// state write the same bits, and a saved state bound again continues exactly.
template <typename R, typename K>
__device__ __forceinline__ void cache_entry(K rho, K kP, K kR, K sigma, R hm, R &rkp, R &tau)
{
#pragma clang fp contract(off)
    rkp = R(rho * kP);
    tau = R(rho * (kR + sigma)) * hm;
}

// Element t of the run of cells starting at base: the block's base offset is
// added to the array pointer on the scalar unit, so every access takes the
// scalar base and one shared 32-bit lane offset (no per-array 64-bit address
// arithmetic on the vector unit).
template <typename P>
__device__ __forceinline__ P &at(P *p, long base, unsigned t)
{
    return (p + base)[t];
}

// Read of element t of an input of the implicit step, which reads each
// input once per step.  NT: with the nontemporal hint, which streams past
// the caches (a probe of this kernel's read/write mix: 7.4 TB/s with it,
// 5.9 without) and leaves the last-level cache to the step's outputs, which
// the next transport reads; but inputs that are still in that cache (a
// working set within a few hundred MB, fresh from the transport) are then
// fetched from HBM again.  See NT_MIN_BYTES.
template <bool NT, typename P>
__device__ __forceinline__ P ld(const P *p, long base, unsigned t)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p + base + t);
    else
        return (p + base)[t];
}

// One cell of the implicit step (cell base + t of the block's run of cells);
// returns the new gas temperature and, in rho, the cell's density.  Four
// FP64 reciprocals per cell (hardware estimate refined by two Newton steps,
// about 1 ulp): 1/rho, the determinant, the flux damping factor and the
// optical depth per length.
template <typename R, bool CONST_OPAC, bool NT>
__device__ __forceinline__ double implicit_cell(const IArgs<R> &a, long base, unsigned t, R hmax, double &rho)
{
    rho = ld<NT>(a.rho, base, t);
    double mx = ld<NT>(a.gin[0], base, t), my = ld<NT>(a.gin[1], base, t), mz = ld<NT>(a.gin[2], base, t);
    double Eg = ld<NT>(a.gin[3], base, t);
    const double inv_rho = Num<double>::rcp(rho);
    const double Cv = rho * a.k.inv_gm1;
    const double T = gas_T_r(inv_rho, mx, my, mz, Eg, a.k.gm1);
    double rkP, rchi;
    if (CONST_OPAC) {
        rkP = rho * a.op.kP;
        rchi = rho * (a.op.kR + a.op.sigma);
    } else {
        rkP = double(ld<NT>(a.rkp, base, t));
        rchi = double(ld<NT>(a.tau, base, t)) * Num<double>::rcp(double(hmax));
    }
    const double Es = double(ld<NT>(a.Es, base, t));
    const double Fs[3] = {double(ld<NT>(a.Fxs, base, t)), double(ld<NT>(a.Fys, base, t)), double(ld<NT>(a.Fzs, base, t))};
    // Eq. implicit_matrix with gamma_abs,red = dt c_hat kappa_P rho and
    // gamma_abs = dt c kappa_P rho, inverted by Cramer's rule in a
    // cancellation-free arrangement (det > 0)
    const double gr = a.k.dt_ch * rkP;
    const double g = a.k.dt_c * rkP;
    const double aT3 = a.k.a * T * T * T, aT4 = aT3 * T;
    const double det = Cv * (1.0 + gr) + 4.0 * g * aT3;
    // irradiation energy deposited in the step enters the S_1 row (Sect. 2.9)
    double S = 0.0;
    if (a.irr) S = ld<NT>(a.irr, base, t) * a.k.dt;
    // uniform branch: the absorption-only form costs the default path nothing
    double E1;
    if (a.absorb)
        E1 = Es / (1.0 + gr);
    else
        E1 = (Cv * (Es + gr * aT4) + 4.0 * aT3 * (g * Es + gr * S)) * Num<double>::rcp(det);
    const double inv_damp = Num<double>::rcp(1.0 + a.k.dt_ch * rchi);   // Eq. source_discrete2
    double F1[3] = {Fs[0] * inv_damp, Fs[1] * inv_damp, Fs[2] * inv_damp};
    const double Fn = Num<double>::sqrt_(F1[0] * F1[0] + F1[1] * F1[1] + F1[2] * F1[2]);
    const bool clipped = Fn > E1;
    if (clipped) {
        const double s = E1 / Fn;
        F1[0] *= s;
        F1[1] *= s;
        F1[2] *= s;
    }
    count_hits(a.cnt, 2, clipped);
    // stored (possibly float) values define the exchanged amounts, so the
    // rescaled totals E_g + (c/c_hat) E and m + F/c_hat are conserved
    R E1r = R(E1), F1r[3] = {R(F1[0]), R(F1[1]), R(F1[2])};
    Eg += S - a.k.c_ratio * (double(E1r) - Es);
    mx -= (double(F1r[0]) - Fs[0]) * a.k.inv_ch;
    my -= (double(F1r[1]) - Fs[1]) * a.k.inv_ch;
    mz -= (double(F1r[2]) - Fs[2]) * a.k.inv_ch;
    if (a.ravg[0]) {
        // second-order step: U^{n+1} = (U^n + U2) / 2 (the averaging partner
        // is read before this cell is written)
        E1r = R(0.5 * (double(ld<NT>(a.ravg[0], base, t)) + double(E1r)));
        for (int v = 0; v < 3; ++v) F1r[v] = R(0.5 * (double(ld<NT>(a.ravg[1 + v], base, t)) + double(F1r[v])));
        mx = 0.5 * (ld<NT>(a.gavg[0], base, t) + mx);
        my = 0.5 * (ld<NT>(a.gavg[1], base, t) + my);
        mz = 0.5 * (ld<NT>(a.gavg[2], base, t) + mz);
        Eg = 0.5 * (ld<NT>(a.gavg[3], base, t) + Eg);
    }
    at(a.E, base, t) = E1r;
    at(a.Fx, base, t) = F1r[0];
    at(a.Fy, base, t) = F1r[1];
    at(a.Fz, base, t) = F1r[2];
    at(a.Eg, base, t) = Eg;
    at(a.mx, base, t) = mx;
    at(a.my, base, t) = my;
    at(a.mz, base, t) = mz;
    return gas_T_r(inv_rho, mx, my, mz, Eg, a.k.gm1);
}

template <typename R, int OPK, bool NT>
__global__ void __launch_bounds__(256) k_implicit(IArgs<R> a)
{
    const int n0 = a.n[0], n1 = a.n[1];
    const int N = n0 * n1 * a.n[2];
    const long base = long(blockIdx.x) * blockDim.x;
    const unsigned t = threadIdx.x;
    const int id = int(base) + int(t);
    if (id >= N) return;
    int i, j, k;
    a.ix.split(id, i, j, k);
    // the cell extent serves both the optical depth read and the one written
    const R hm = OPK == OPK_CONST ? R(0) : cell_hmax(a.m, a.ndim, i, j, k);
    double rho_d;
    const double T1 = implicit_cell<R, OPK == OPK_CONST, NT>(a, base, t, hm, rho_d);
    if (OPK != OPK_CONST) {
        const R rho = R(rho_d);
        R kP, kR;
        opacity_analytic<R, OPK>(a.op, rho, R(T1), kP, kR);
        cache_entry(rho, kP, kR, R(a.op.sigma), hm, at(a.rkp, base, t), at(a.tau, base, t));
    }
}

// MLP opacity: every lane of a wavefront takes part in the network
// evaluation (one 64-cell chunk per wavefront), so lanes past the last cell
// compute on a clamped index instead of exiting early.  The cell update runs
// before the weights are staged into LDS: its many array pointers are then
// dead during the staging, which keeps the kernel within the scalar register
// file (staged first, the pointers were spilled to vector lanes).
template <typename R, bool NT>
__global__ void __launch_bounds__(256, 4) k_implicit_mlp(IArgs<R> a)
{
    const int n0 = a.n[0], n1 = a.n[1];
    const int N = n0 * n1 * a.n[2];
    const int lane = threadIdx.x & 63;
    __shared__ MlpShared sh;
    {
        const long base = long(blockIdx.x) * blockDim.x;
        const unsigned t = threadIdx.x;
        const int id = int(base) + int(t);
        const bool live = id < N;
        const int idc = live ? id : N - 1;
        int i, j, k;
        a.ix.split(idc, i, j, k);
        const R hm = cell_hmax(a.m, a.ndim, i, j, k);
        // lanes past the last cell evaluate the network at rho = T = 1
        double T1 = 1.0, rho_d = 1.0;
        if (live) T1 = implicit_cell<R, false, NT>(a, base, t, hm, rho_d);
        const float rho = float(rho_d);
        mlp_stage(a.op.mlp, sh, threadIdx.x, blockDim.x);
        __syncthreads();
        float kP, kR;
        mlp_opacity_shared(a.op, sh, rho, float(T1), lane, kP, kR);
        if (live) {
            cache_entry(rho, kP, kR, a.op.f32.sigma, hm, at(a.rkp, base, t), at(a.tau, base, t));
        }
    }
}

template <typename R>
static void fill_args(m1_ctx *c, IArgs<R> &a, const Metric<R> &met, double dt)
{
    a.E = static_cast<R *>(c->f.E);
    a.Fx = static_cast<R *>(c->f.Fx);
    a.Fy = static_cast<R *>(c->f.Fy);
    a.Fz = static_cast<R *>(c->f.Fz);
    a.Es = static_cast<const R *>(c->star[0]);
    a.Fxs = static_cast<const R *>(c->star[1]);
    a.Fys = static_cast<const R *>(c->star[2]);
    a.Fzs = static_cast<const R *>(c->star[3]);
    a.rho = c->f.rho;
    a.mx = c->f.mx;
    a.my = c->f.my;
    a.mz = c->f.mz;
    a.Eg = c->f.Eg;
    a.rkp = static_cast<R *>(c->rkp);
    a.tau = static_cast<R *>(c->tau);
    for (int d = 0; d < 3; ++d) a.n[d] = c->n[d];
    a.ndim = c->ndim;
    a.ix.set(c->n[0], c->n[1]);
    a.m = met;
    a.op = c->op;
    a.k.dt = dt;
    a.k.c_hat = c->c_hat;
    a.k.c = c->par.c;
    a.k.a = c->par.a_rad;
    a.k.gamma = c->par.gamma;
    a.k.gm1 = c->par.gamma - 1.0;
    a.k.inv_gm1 = 1.0 / a.k.gm1;
    a.k.dt_ch = dt * c->c_hat;
    a.k.dt_c = dt * c->par.c;
    a.k.inv_ch = 1.0 / c->c_hat;
    a.k.c_ratio = c->par.c * a.k.inv_ch;
    a.irr = c->irr;
    a.absorb = c->par.absorb_only;
    a.gin[0] = a.mx;
    a.gin[1] = a.my;
    a.gin[2] = a.mz;
    a.gin[3] = a.Eg;
    for (int v = 0; v < 4; ++v) {
        a.ravg[v] = nullptr;
        a.gavg[v] = nullptr;
    }
    a.cnt = c->cnt;
}

// Stage of the second-order step (stage 0: an ordinary in-place step).
// Stage 1 reads the caller's gas and writes U1 (radiation and gas) to the
// save buffer; stage 2 reads U1's gas from there and writes (U^n + U2) / 2
// into the caller's arrays, the opacity cache following the written state.
// The buffer holds the four radiation fields of all groups (group-major, a
// field every rk2_rad_bytes) and then the four gas fields.
template <typename R>
static void rk2_stage_args(m1_ctx *c, IArgs<R> &a, int stage)
{
    if (stage == 0) return;
    const long N = long(c->n[0]) * c->n[1] * c->n[2];
    unsigned char *sv = static_cast<unsigned char *>(c->rk2_save);
    R *srad[4];
    double *sgas[4];
    for (int v = 0; v < 4; ++v) {
        srad[v] = reinterpret_cast<R *>(sv + v * c->rk2_rad_bytes);
        sgas[v] = reinterpret_cast<double *>(sv + 4 * c->rk2_rad_bytes) + v * N;
    }
    if (stage == 1) {
        a.E = srad[0];
        a.Fx = srad[1];
        a.Fy = srad[2];
        a.Fz = srad[3];
        a.mx = sgas[0];
        a.my = sgas[1];
        a.mz = sgas[2];
        a.Eg = sgas[3];
        const double *g[4] = {c->f.mx, c->f.my, c->f.mz, c->f.Eg};
        for (int v = 0; v < 4; ++v) a.gin[v] = g[v];
    } else {
        const R *r[4] = {static_cast<const R *>(c->f.E), static_cast<const R *>(c->f.Fx),
                         static_cast<const R *>(c->f.Fy), static_cast<const R *>(c->f.Fz)};
        const double *g[4] = {c->f.mx, c->f.my, c->f.mz, c->f.Eg};
        for (int v = 0; v < 4; ++v) {
            a.gin[v] = sgas[v];
            a.ravg[v] = r[v];
            a.gavg[v] = g[v];
        }
    }
}

// Streaming reads in the implicit step above this many bytes per step.
// Measured on one box (A/B of both forms, 100-step runs): on the 256^3 box
// and the 192x96x192 grid in FP64 the hint made the whole step 1.6 % and
// 5.5 % faster (the next transport then finds the step's outputs in the
// 256 MB last-level cache), and the network form's 2 %; on the 128^3 box
// (285 MB FP64, 220 MB FP32) the inputs were still cached and the implicit
// kernel took 18-25 % longer with it.  The FP32 table form at 192x96x192
// (425 MB) came out 1 % slower, the one measured case above the line
// that did not gain.  The multigroup kernel follows the same rule (eight
// groups at 128^3: its launch 6-9 % faster, the step 1.3-1.4 %).
constexpr double NT_MIN_BYTES = 384.0 * (1 << 20);

// whether the implicit step of a context streams its reads (m1_params.stream_reads)
static bool stream_reads(const m1_ctx *c, double bytes)
{
    if (c->par.stream_reads == M1_STREAM_ON) return true;
    if (c->par.stream_reads == M1_STREAM_OFF) return false;
    return bytes >= NT_MIN_BYTES;
}

template <typename R>
static hipError_t launch_i(m1_ctx *c, double dt, const Metric<R> &met, int stage = 0)
{
    IArgs<R> a;
    fill_args(c, a, met, dt);
    rk2_stage_args(c, a, stage);
    const int N = c->n[0] * c->n[1] * c->n[2];
    dim3 block(256), grid((N + 255) / 256);
    // the step's bytes: E*, F* in, E, F out, the gas in and out, the
    // opacity cache in and out
    const double bytes = double(N) * (8.0 * sizeof(R) + 72.0 + (c->op.kind == OPK_CONST ? 0.0 : 4.0 * sizeof(R)));
    if (stream_reads(c, bytes)) {
        switch (c->op.kind) {
        case OPK_CONST: hipLaunchKernelGGL((k_implicit<R, OPK_CONST, true>), grid, block, 0, c->stream, a); break;
        case OPK_POWERLAW: hipLaunchKernelGGL((k_implicit<R, OPK_POWERLAW, true>), grid, block, 0, c->stream, a); break;
        case OPK_TABLE: hipLaunchKernelGGL((k_implicit<R, OPK_TABLE, true>), grid, block, 0, c->stream, a); break;
        default: hipLaunchKernelGGL((k_implicit_mlp<R, true>), grid, block, 0, c->stream, a); break;
        }
    } else {
        switch (c->op.kind) {
        case OPK_CONST: hipLaunchKernelGGL((k_implicit<R, OPK_CONST, false>), grid, block, 0, c->stream, a); break;
        case OPK_POWERLAW: hipLaunchKernelGGL((k_implicit<R, OPK_POWERLAW, false>), grid, block, 0, c->stream, a); break;
        case OPK_TABLE: hipLaunchKernelGGL((k_implicit<R, OPK_TABLE, false>), grid, block, 0, c->stream, a); break;
        default: hipLaunchKernelGGL((k_implicit_mlp<R, false>), grid, block, 0, c->stream, a); break;
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multigroup (one gray fluid per frequency group, (m+1)^2 implicit system)
// ---------------------------------------------------------------------------

// Fraction of the Planck energy density below x = h nu / k T,
// (15 / pi^4) int_0^x t^3 / (e^t - 1) dt.  Below x = 5/2: the power series
// of t^3 / (e^t - 1) integrated term by term, coefficients B_k / ((k + 3) k!)
// with B_k the Bernoulli numbers, through k = 42 (the series converges for
// x < 2 pi; at x = 5/2 the omitted terms are below 2e-18 of the sum); above:
// 1 minus the tail sum_n e^{-n x} (x^3/n + 3 x^2/n^2 + 6 x/n^3 + 6/n^4),
// summed until its terms drop below double precision (at most 17 of them
// above 5/2).  The split at 5/2 rather than 1 bounds the tail loop, whose
// length otherwise grows as 1/x and dominated the multigroup implicit step.
__device__ double planck_fraction(double x)
{
    constexpr double NORM = 0.15398973382026503;   // 15 / pi^4
    if (x <= 0.0) return 0.0;
    if (x < 2.5) {
        // B_k / ((k + 3) k!) for k = 2, 4, ..., 42 (odd B_k > 1 vanish)
        constexpr double C[21] = {
            0.016666666666666666, -0.00019841269841269841, 3.6743092298647855e-06, -7.5156325156325161e-08,
            1.6059043836821615e-09, -3.5227934257916621e-11, 7.8720803121674577e-13, -1.7840422612224122e-14,
            4.0886009791799258e-16, -9.4559508632959214e-18, 2.2036011313440918e-19, -5.1683202540046385e-21,
            1.2188644964239542e-22, -2.8882314280766281e-24, 6.8725831889020704e-26, -1.641368762534915e-27,
            3.9328985827428784e-29, -9.451269078629001e-31, 2.2772522578280597e-32, -5.5000521295363484e-34,
            1.3312603916626966e-35};
        const double x2 = x * x;
        // x^3 (1/3 - x/8 + x^2 (C_2 + C_4 x^2 + ...))
        double p = C[20];
        for (int j = 19; j >= 0; --j) p = __builtin_fma(p, x2, C[j]);
        const double series = (1.0 / 3.0) + x * (-0.125) + x2 * p;
        return NORM * x * x2 * series;
    }
    // 1/n, n = 1 .. 17 (the most terms the tail takes above 5/2)
    constexpr double RN[18] = {0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9,
                               1.0 / 10, 1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17};
    const double e1 = exp(-x);
    const double x2 = x * x, x3 = x2 * x;
    double e = e1, tail = 0.0;
    for (int n = 1; n <= 17 && e > 1e-18 * e1; ++n) {
        const double rn = RN[n];
        tail += e * rn * (x3 + rn * (3.0 * x2 + rn * (6.0 * x + rn * 6.0)));
        e *= e1;
    }
    return 1.0 - NORM * tail;
}

template <typename R>
struct MgArgs {
    GroupParams gp;
    long N;
    size_t plane;                     // bytes between scratch fields
    const unsigned char *star;        // transported group states
};

// Optical depth of every group from the gas density (constant opacities).
template <typename R>
__global__ void __launch_bounds__(256) k_tau_mg(IArgs<R> a, MgArgs<R> g, unsigned char *tau)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.N) return;
    int i, j, k;
    a.ix.split(id, i, j, k);
    const R h = cell_hmax(a.m, a.ndim, i, j, k);
    const double rho = a.rho[id];
    for (int q = 0; q < g.gp.m; ++q)
        reinterpret_cast<R *>(tau + q * g.plane)[id] = R(rho * (g.gp.kR[q] + g.gp.sigma)) * h;
}

// One cell of the multigroup implicit step.  The (m+1)^2 system
//   (1 + gr_g) E'_g - 4 gr_g b_g a T^3 T' = E*_g - 3 gr_g b_g a T^4
//   -sum_g g_g E'_g + (C_v + 4 sum_g g_g b_g a T^3) T' = C_v T + 3 sum_g g_g b_g a T^4 + S
// is an arrowhead matrix: eliminating the group rows leaves one equation
// for T' whose coefficients are sums of positive terms,
//   D  = C_v + sum_g 4 g_g b_g a T^3 / (1 + gr_g),
//   L  = a (4 T^3 T' - 3 T^4) = a T^3 (C_v T + 4 S + 4 sum_g g_g E*_g / (1 + gr_g)) / D,
//   E'_g = (E*_g + gr_g b_g L) / (1 + gr_g),
// O(m) work and no cancellation.
template <typename R, int MG, bool NT>
__global__ void __launch_bounds__(256) k_implicit_mg(IArgs<R> a, MgArgs<R> g)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.N) return;
    const int m = g.gp.m;
    const double rho = ld<NT>(a.rho, 0, id);
    double mx = ld<NT>(a.gin[0], 0, id), my = ld<NT>(a.gin[1], 0, id), mz = ld<NT>(a.gin[2], 0, id);
    double Eg = ld<NT>(a.gin[3], 0, id);
    const double inv_rho = Num<double>::rcp(rho);
    const double Cv = rho * a.k.inv_gm1;
    const double T = gas_T_r(inv_rho, mx, my, mz, Eg, a.k.gm1);
    const double S = a.irr ? ld<NT>(a.irr, 0, id) * a.k.dt : 0.0;
    const double aT3 = a.k.a * T * T * T;
    const double iT = Num<double>::rcp(T);
    // pass 1: group fractions, transported energies and the reduced equation
    // for the temperature (per-group values stay in registers: MG >= m)
    double b[MG], Es[MG], inv1[MG];
    double D = Cv, Lnum = Cv * T + 4.0 * S, lo = 0.0;
#pragma unroll
    for (int q = 0; q < MG; ++q) {
        if (q < m) {
            const double hi = q + 1 < m ? planck_fraction(g.gp.edges[q] * iT) : 1.0;
            b[q] = hi - lo;
            lo = hi;
            Es[q] = double(ld<NT>(reinterpret_cast<const R *>(g.star + 4 * q * g.plane), 0, id));
            const double kr = rho * g.gp.kP[q];
            inv1[q] = Num<double>::rcp(1.0 + a.k.dt_ch * kr);
            const double gg = a.k.dt_c * kr;
            D += 4.0 * gg * b[q] * aT3 * inv1[q];
            Lnum += 4.0 * gg * Es[q] * inv1[q];
        }
    }
    const double L = aT3 * Lnum * Num<double>::rcp(D);
    // pass 2: group energies, damped fluxes, rescaled totals
    double dE = 0.0, dF[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < MG; ++q) {
        if (q < m) {
            const double gr = a.k.dt_ch * rho * g.gp.kP[q];
            const double E1 = a.absorb ? Es[q] * inv1[q] : (Es[q] + gr * b[q] * L) * inv1[q];
            const double inv_damp = Num<double>::rcp(1.0 + a.k.dt_ch * rho * (g.gp.kR[q] + g.gp.sigma));
            double F1[3], Fs[3];
            for (int v = 0; v < 3; ++v) {
                Fs[v] = double(ld<NT>(reinterpret_cast<const R *>(g.star + (4 * q + 1 + v) * g.plane), 0, id));
                F1[v] = Fs[v] * inv_damp;
            }
            const double Fn = Num<double>::sqrt_(F1[0] * F1[0] + F1[1] * F1[1] + F1[2] * F1[2]);
            const bool clipped = Fn > E1;
            if (clipped) {
                const double sc = E1 / Fn;
                F1[0] *= sc;
                F1[1] *= sc;
                F1[2] *= sc;
            }
            count_hits(a.cnt, 2, clipped);
            R E1r = R(E1), F1r[3] = {R(F1[0]), R(F1[1]), R(F1[2])};
            dE += double(E1r) - Es[q];
            for (int v = 0; v < 3; ++v) dF[v] += double(F1r[v]) - Fs[v];
            const long o = q * g.N + id;
            if (a.ravg[0]) {
                // second-order step: (U^n + U2) / 2, the partner read before
                // this cell is written
                E1r = R(0.5 * (double(ld<NT>(a.ravg[0], o, 0)) + double(E1r)));
                for (int v = 0; v < 3; ++v) F1r[v] = R(0.5 * (double(ld<NT>(a.ravg[1 + v], o, 0)) + double(F1r[v])));
            }
            a.E[o] = E1r;
            a.Fx[o] = F1r[0];
            a.Fy[o] = F1r[1];
            a.Fz[o] = F1r[2];
        }
    }
    Eg += S - a.k.c_ratio * dE;
    mx -= dF[0] * a.k.inv_ch;
    my -= dF[1] * a.k.inv_ch;
    mz -= dF[2] * a.k.inv_ch;
    if (a.ravg[0]) {
        mx = 0.5 * (ld<NT>(a.gavg[0], 0, id) + mx);
        my = 0.5 * (ld<NT>(a.gavg[1], 0, id) + my);
        mz = 0.5 * (ld<NT>(a.gavg[2], 0, id) + mz);
        Eg = 0.5 * (ld<NT>(a.gavg[3], 0, id) + Eg);
    }
    a.Eg[id] = Eg;
    a.mx[id] = mx;
    a.my[id] = my;
    a.mz[id] = mz;
}

template <typename R>
static MgArgs<R> mg_args(m1_ctx *c)
{
    MgArgs<R> g;
    g.gp = c->grp;
    g.N = long(c->n[0]) * c->n[1] * c->n[2];
    g.plane = c->plane_bytes;
    g.star = static_cast<const unsigned char *>(c->star[0]);
    return g;
}

template <typename R, bool NT>
static void launch_mg_kernel(m1_ctx *c, dim3 grid, dim3 block, const IArgs<R> &a, const MgArgs<R> &g)
{
    if (g.gp.m <= 4)
        hipLaunchKernelGGL((k_implicit_mg<R, 4, NT>), grid, block, 0, c->stream, a, g);
    else if (g.gp.m <= 8)
        hipLaunchKernelGGL((k_implicit_mg<R, 8, NT>), grid, block, 0, c->stream, a, g);
    else if (g.gp.m <= 16)
        hipLaunchKernelGGL((k_implicit_mg<R, 16, NT>), grid, block, 0, c->stream, a, g);
    else
        hipLaunchKernelGGL((k_implicit_mg<R, 32, NT>), grid, block, 0, c->stream, a, g);
}

template <typename R>
static hipError_t launch_i_mg(m1_ctx *c, double dt, const Metric<R> &met, int stage = 0)
{
    IArgs<R> a;
    fill_args(c, a, met, dt);
    rk2_stage_args(c, a, stage);
    const MgArgs<R> g = mg_args<R>(c);
    const dim3 grid(unsigned((g.N + 255) / 256)), block(256);
    const double bytes = double(g.N) * (8.0 * sizeof(R) * g.gp.m + 72.0);
    if (stream_reads(c, bytes))
        launch_mg_kernel<R, true>(c, grid, block, a, g);
    else
        launch_mg_kernel<R, false>(c, grid, block, a, g);
    return hipGetLastError();
}

hipError_t launch_implicit_rk2(m1_ctx *c, double dt, int stage)
{
    if (c->grp.m > 1) {
        if (c->par.precision == M1_F32) return launch_i_mg<float>(c, dt, c->met32, stage);
        return launch_i_mg<double>(c, dt, c->met64, stage);
    }
    if (c->par.precision == M1_F32) return launch_i<float>(c, dt, c->met32, stage);
    return launch_i<double>(c, dt, c->met64, stage);
}

hipError_t launch_implicit(m1_ctx *c, double dt)
{
    if (c->grp.m > 1) {
        if (c->par.precision == M1_F32) return launch_i_mg<float>(c, dt, c->met32);
        return launch_i_mg<double>(c, dt, c->met64);
    }
    if (c->par.precision == M1_F32) return launch_i<float>(c, dt, c->met32);
    return launch_i<double>(c, dt, c->met64);
}

// ---------------------------------------------------------------------------
// opacity cache from the current gas state
// ---------------------------------------------------------------------------

template <typename R, int OPK>
__global__ void __launch_bounds__(256) k_opacity_init(IArgs<R> a)
{
    const int n0 = a.n[0], n1 = a.n[1];
    const int N = n0 * n1 * a.n[2];
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    int i, j, k;
    a.ix.split(id, i, j, k);
    const double T = gas_T_stored(a.rho[id], a.mx[id], a.my[id], a.mz[id], a.Eg[id], a.k.gm1);
    const R rho = R(a.rho[id]);
    R kP, kR;
    opacity_analytic<R, OPK>(a.op, rho, R(T), kP, kR);
    cache_entry(rho, kP, kR, R(a.op.sigma), cell_hmax(a.m, a.ndim, i, j, k), a.rkp[id], a.tau[id]);
}

template <typename R>
__global__ void __launch_bounds__(256) k_opacity_init_mlp(IArgs<R> a)
{
    const int n0 = a.n[0], n1 = a.n[1];
    const int N = n0 * n1 * a.n[2];
    const int lane = threadIdx.x & 63;
    __shared__ MlpShared sh;
    mlp_stage(a.op.mlp, sh, threadIdx.x, blockDim.x);
    __syncthreads();
    {
        const int id = blockIdx.x * blockDim.x + threadIdx.x;
        const bool live = id < N;
        const int idc = live ? id : N - 1;
        int i, j, k;
        a.ix.split(idc, i, j, k);
        const double T = gas_T_stored(a.rho[idc], a.mx[idc], a.my[idc], a.mz[idc], a.Eg[idc], a.k.gm1);
        const float rho = float(a.rho[idc]);
        float kP, kR;
        mlp_opacity_shared(a.op, sh, rho, float(T), lane, kP, kR);
        if (live) {
            cache_entry(rho, kP, kR, a.op.f32.sigma, cell_hmax(a.m, a.ndim, i, j, k), a.rkp[id], a.tau[id]);
        }
    }
}

template <typename R>
static hipError_t launch_init(m1_ctx *c, const Metric<R> &met)
{
    IArgs<R> a;
    fill_args(c, a, met, 0.0);
    const int N = c->n[0] * c->n[1] * c->n[2];
    dim3 block(256), grid((N + 255) / 256);
    switch (c->op.kind) {
    case OPK_CONST: hipLaunchKernelGGL((k_opacity_init<R, OPK_CONST>), grid, block, 0, c->stream, a); break;
    case OPK_POWERLAW: hipLaunchKernelGGL((k_opacity_init<R, OPK_POWERLAW>), grid, block, 0, c->stream, a); break;
    case OPK_TABLE: hipLaunchKernelGGL((k_opacity_init<R, OPK_TABLE>), grid, block, 0, c->stream, a); break;
    default:
        hipLaunchKernelGGL((k_opacity_init_mlp<R>), grid, block, 0, c->stream, a);
        break;
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_init_mg(m1_ctx *c, const Metric<R> &met)
{
    IArgs<R> a;
    fill_args(c, a, met, 0.0);
    const MgArgs<R> g = mg_args<R>(c);
    hipLaunchKernelGGL((k_tau_mg<R>), dim3(unsigned((g.N + 255) / 256)), dim3(256), 0, c->stream, a, g,
                       static_cast<unsigned char *>(c->tau));
    return hipGetLastError();
}

hipError_t launch_opacity_init(m1_ctx *c)
{
    if (c->grp.m > 1) {
        if (c->par.precision == M1_F32) return launch_init_mg<float>(c, c->met32);
        return launch_init_mg<double>(c, c->met64);
    }
    if (c->par.precision == M1_F32) return launch_init<float>(c, c->met32);
    return launch_init<double>(c, c->met64);
}

// ---------------------------------------------------------------------------
// pointwise evaluation of the active opacity source (tests, tools)
// ---------------------------------------------------------------------------

template <int OPK>
__global__ void __launch_bounds__(256) k_opacity_eval(OpacityParams op, long n, const double *rho,
                                                      const double *T, double *kP, double *kR)
{
    const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= n) return;
    double a, b;
    opacity_analytic<double, OPK>(op, rho[id], T[id], a, b);
    kP[id] = a;
    kR[id] = b;
}

__global__ void __launch_bounds__(256) k_opacity_eval_mlp(OpacityParams op, long n, const double *rho,
                                                          const double *T, double *kP, double *kR)
{
    const int lane = threadIdx.x & 63;
    __shared__ MlpShared sh;
    mlp_stage(op.mlp, sh, threadIdx.x, blockDim.x);
    __syncthreads();
    {
        const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
        const bool live = id < n;
        const long idc = live ? id : n - 1;
        float a, b;
        mlp_opacity_shared(op, sh, float(rho[idc]), float(T[idc]), lane, a, b);
        if (live) {
            kP[id] = a;
            kR[id] = b;
        }
    }
}

hipError_t launch_opacity_eval(m1_ctx *c, long n, const double *rho, const double *T, double *kP,
                               double *kR)
{
    if (n <= 0) return hipSuccess;
    dim3 block(256);
    dim3 grid((unsigned)((n + 255) / 256));
    switch (c->op.kind) {
    case OPK_CONST: hipLaunchKernelGGL((k_opacity_eval<OPK_CONST>), grid, block, 0, c->stream, c->op, n, rho, T, kP, kR); break;
    case OPK_POWERLAW: hipLaunchKernelGGL((k_opacity_eval<OPK_POWERLAW>), grid, block, 0, c->stream, c->op, n, rho, T, kP, kR); break;
    case OPK_TABLE: hipLaunchKernelGGL((k_opacity_eval<OPK_TABLE>), grid, block, 0, c->stream, c->op, n, rho, T, kP, kR); break;
    default:
        hipLaunchKernelGGL(k_opacity_eval_mlp, grid, block, 0, c->stream, c->op, n, rho, T, kP, kR);
        break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// RK2 averaging: U <- (U_saved + U) / 2 for E, F (form precision) and m, E_g
// ---------------------------------------------------------------------------

} // namespace m1

