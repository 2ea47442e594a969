// m1_device.h -- device-side building blocks of the M1 step for gfx950:
// Levermore closure with the Sect. 2.6 signal speeds and the physical flux
// of one state, the HLL interface flux with the optical-depth limiter, the
// van Leer and LimO3 slopes and the f-preserving face fix
// (Eq. f_reconstruct).
// Templated on the working precision R (double or float).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/m1.h"

namespace m1 {

// Arithmetic primitives per precision.  FP64 (arguments are positive normal
// numbers, or zero for the square root):
//  * reciprocal: the hardware estimate refined by two Newton steps
//    r <- r (2 - x r), each doubling the correct bits (within an ulp or two);
//  * square root: Goldschmidt iteration from the hardware reciprocal square
//    root y, g = x y and h = y / 2 refined together, then two Newton
//    corrections g <- g + (x - g^2) h; correctly rounded on every argument
//    tried from 1e-300 to 1e300, with no range scaling or special-case
//    handling beyond zero (the callers pass no subnormal or infinite
//    arguments: squared norms below the smallest normal number are taken
//    as zero before any reciprocal);
//  * reciprocal square root: the hardware estimate refined by two Newton
//    steps y <- y + y (1 - x y^2) / 2.
// All stay far inside the 1e-12 parity tolerance.  FP32: the hardware
// reciprocal, square root and reciprocal square root (about 1 ulp), inside
// 1e-5.
template <typename R> struct Num;
template <> struct Num<double> {
    // smallest normal number: |F|^2 below it is taken as F = 0, so that the
    // inverse |F|^-2 stays finite
    static constexpr double tiny = __DBL_MIN__;
    static __device__ __forceinline__ double sqrt_(double x)
    {
        const double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        const double r = __builtin_fma(-h, g, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
        double d = __builtin_fma(-g, g, x);
        g = __builtin_fma(d, h, g);
        d = __builtin_fma(-g, g, x);
        g = __builtin_fma(d, h, g);
        return x > 0.0 ? g : 0.0;
    }
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        return r;
    }
    static __device__ __forceinline__ double rsqrt(double x)
    {
        double y = __builtin_amdgcn_rsq(x);
        y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
        y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
        return y;
    }
};
template <> struct Num<float> {
    static constexpr float tiny = __FLT_MIN__;
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
};

// Adds to counter `which` the number of active lanes of the wavefront with
// hit set, by one atomic from the lowest such lane into the wavefront's slot
// of the counter (every active lane calls it).  Fix-up counters see up to
// millions of events per launch (a multigroup step clips several per cent of
// its cell-groups); atomics of every wavefront on one address serialised
// them and more than doubled the multigroup implicit step.
__device__ __forceinline__ void count_hits(unsigned long long *cnt, int which, bool hit)
{
    const unsigned long long m = __ballot(hit);
    if (m != 0ull && __lane_id() == unsigned(__ffsll((long long)m) - 1)) {
        const unsigned wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        const unsigned slot = wave & (CNT_SLOTS - 1);
        atomicAdd(cnt + (size_t(which) * CNT_SLOTS + slot) * CNT_STRIDE, (unsigned long long)__popcll(m));
    }
}

// minimum / maximum as single instructions (finite arguments)
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }

// Closure quantities of one radiation state (E, F) seen from direction d:
// lambda_-, lambda_+ (Sect. 2.6) and the flux (F_d, E D_{xd}, E D_{yd},
// E D_{zd}) (Sect. 2.1, Eqs. rad1/rad2), all in units of c_hat.
template <typename R>
struct Wave {
    R lm, lp;
    R phi[4];
};

template <typename R, int D>
__device__ __forceinline__ Wave<R> closure_wave(R E, R Fx, R Fy, R Fz)
{
    Wave<R> w;
    const R F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const R Fn = F2 >= Num<R>::tiny ? Num<R>::sqrt_(F2) : R(0);    // F = 0 below the normal range
    R f = Fn / E;
    f = f > R(1) ? R(1) : f;
    const R f2 = f * f;
    const R s = Num<R>::sqrt_(R(4) - R(3) * f2);
    const R xi = (R(3) + R(4) * f2) / (R(5) + R(2) * s);
    const R Fd = D == 0 ? Fx : (D == 1 ? Fy : Fz);
    // n = F / |F| (n = 0 for F = 0)
    const R inv = Fn > R(0) ? R(1) / Fn : R(0);
    const R mu = Fd * inv;
    R z2 = (R(2) / R(3)) * (R(4) - R(3) * f2 - s) + R(2) * mu * mu * (R(2) - f2 - s);
    z2 = z2 < R(0) ? R(0) : z2;
    const R zeta = Num<R>::sqrt_(z2);
    const R a = (f * mu - zeta) / s, b = (f * mu + zeta) / s;
    w.lm = a < b ? a : b;
    w.lp = a < b ? b : a;
    const R iso = R(0.5) * (R(1) - xi) * E;
    const R an = R(0.5) * (R(3) * xi - R(1)) * E;
    const R nd = mu;
    w.phi[0] = Fd;
    w.phi[1] = an * (Fx * inv) * nd + (D == 0 ? iso : R(0));
    w.phi[2] = an * (Fy * inv) * nd + (D == 1 ? iso : R(0));
    w.phi[3] = an * (Fz * inv) * nd + (D == 2 ? iso : R(0));
    return w;
}

// HLL flux c_hat * Phi* between face states UL | UR (Sect. 2.5) with the
// speeds lambda_L = min lambda_-, lambda_R = max lambda_+ clamped to
// -+4/(3 tau) for tau > 0 (Sect. 2.6), S_L = min(lambda_L, 0),
// S_R = max(lambda_R, 0); S_L = S_R = 0 falls back to the average flux.
template <typename R, int D>
__device__ __forceinline__ void hll_flux(const R UL[4], const R UR[4], R tau, R c_hat, R out[4],
                                         int riemann = M1_RIEMANN_HLL)
{
    const Wave<R> wl = closure_wave<R, D>(UL[0], UL[1], UL[2], UL[3]);
    const Wave<R> wr = closure_wave<R, D>(UR[0], UR[1], UR[2], UR[3]);
    R lamL = wl.lm < wr.lm ? wl.lm : wr.lm;
    R lamR = wl.lp > wr.lp ? wl.lp : wr.lp;
    if (tau > R(0)) {
        const R lim = R(4) / (R(3) * tau);
        lamL = lamL < -lim ? -lim : lamL;
        lamR = lamR > lim ? lim : lamR;
    }
    if (riemann == M1_RIEMANN_LF) {
        const R aL = lamL < R(0) ? -lamL : lamL, aR = lamR < R(0) ? -lamR : lamR;
        const R sp = aL > aR ? aL : aR;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = c_hat * (R(0.5) * (wl.phi[q] + wr.phi[q]) - R(0.5) * sp * (UR[q] - UL[q]));
        return;
    }
    const R SL = lamL < R(0) ? lamL : R(0);
    const R SR = lamR > R(0) ? lamR : R(0);
    if (SR > SL) {
        const R k = c_hat / (SR - SL);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            out[q] = k * (SR * wl.phi[q] - SL * wr.phi[q] + SL * SR * (UR[q] - UL[q]));
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = c_hat * R(0.5) * (wl.phi[q] + wr.phi[q]);
    }
}

// van Leer limited slope of divided differences (harmonic mean, 0 at extrema).
template <typename R>
__device__ __forceinline__ R vanleer(R dl, R dr)
{
    const R p = dl * dr;
    return p > R(0) ? (R(2) * p) / (dl + dr) : R(0);
}

// f-preserving fix of a reconstructed face state against its donor cell
// centre (Eq. f_reconstruct): keep F_face iff f_face <= 1 and f_face >
// f_centre, else F_face = F_centre * E_face / E_centre; E_face <= 0 falls back
// to the centre state.
template <typename R>
__device__ __forceinline__ void ffix(R U[4], const R C[4])
{
    if (U[0] > R(0)) {
        const R ff = Num<R>::sqrt_(U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0];
        const R fc = Num<R>::sqrt_(C[1] * C[1] + C[2] * C[2] + C[3] * C[3]) / C[0];
        if (!(ff <= R(1) && ff > fc)) {
            const R r = U[0] / C[0];
            U[1] = C[1] * r;
            U[2] = C[2] * r;
            U[3] = C[3] * r;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) U[q] = C[q];
    }
}


// ---------------------------------------------------------------------------
// Face-flux building blocks with a run-time direction (used by the tiled
// kernel, where one wavefront mixes x and y faces).  Same mathematics as
// closure_wave / hll_flux / ffix, arranged to need four reciprocals and two
// square roots per state: with E^-1, |F|^-2 and s = sqrt(4 - 3 f^2) (in
// FP64 s and 1 / s come from one refined reciprocal square root instead,
// s = (4 - 3 f^2) / sqrt(4 - 3 f^2): eight FP64 operations fewer; in FP32
// that form, one transcendental fewer, raised the 100-step deviation of the
// flux from the FP64 form by a quarter, so FP32 keeps the hardware square
// root and reciprocal),
//   f mu = F_d / E (unclamped f) or F_d / |F| (f clamped to 1),
//   n_i n_d = F_i F_d / |F|^2,  lambda_-+ = (f mu -+ zeta) / s.
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ Wave<R> closure_wave_rt(R E, R Fx, R Fy, R Fz, int d)
{
    Wave<R> w;
    const R F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const R iE = Num<R>::rcp(E);
    R f2 = F2 * iE * iE;
    const bool clamped = f2 > R(1);
    f2 = vmin(f2, R(1));
    const R s2 = R(4) - R(3) * f2;                 // in [1, 4]
    R s, is64 = R(0);
    if constexpr (sizeof(R) == 8) {
        is64 = Num<R>::rsqrt(s2);
        s = s2 * is64;
    } else {
        s = Num<R>::sqrt_(s2);
    }
    // Levermore: xi = (3 + 4 f^2) / (5 + 2 s) = (5 - 2 s) / 3, so
    // (1 - xi) / 2 = (s - 1) / 3 and (3 xi - 1) / 2 = 2 - s
    // |F|^2 under the smallest normal number counts as F = 0: its inverse
    // square would overflow, and a far-field flux that small (the numerical
    // tail ahead of a front) carries no direction worth resolving
    const R iFn = F2 >= Num<R>::tiny ? Num<R>::rsqrt(F2) : R(0);
    const R iF2 = iFn * iFn;
    const R Fd = d == 0 ? Fx : (d == 1 ? Fy : Fz);
    const R mu2 = Fd * Fd * iF2;
    const R z2 = vmax((R(2) / R(3)) * (R(4) - R(3) * f2 - s) + R(2) * mu2 * (R(2) - f2 - s), R(0));
    const R zeta = Num<R>::sqrt_(z2);
    const R fmu = Fd * (clamped ? iFn : iE);
    const R is = sizeof(R) == 8 ? is64 : Num<R>::rcp(s);
    w.lm = (fmu - zeta) * is;
    w.lp = (fmu + zeta) * is;
    const R iso = (s - R(1)) * (R(1) / R(3)) * E;
    const R c = (R(2) - s) * E * iF2 * Fd;
    w.phi[0] = Fd;
    w.phi[1] = c * Fx + (d == 0 ? iso : R(0));
    w.phi[2] = c * Fy + (d == 1 ? iso : R(0));
    w.phi[3] = c * Fz + (d == 2 ? iso : R(0));
    return w;
}

// f-preserving fix with squared norms: with r = E_f / E_c, keep F_face iff
// |F_f|^2 <= E_f^2 and |F_f|^2 > |F_c|^2 r^2 (E > 0), i.e. f_face <= 1 and
// f_face > f_centre; otherwise F_face = r F_centre.
template <typename R>
__device__ __forceinline__ void ffix_sq(R U[4], const R C[4])
{
    if (U[0] > R(0)) {
        const R Ff2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
        const R Fc2 = C[1] * C[1] + C[2] * C[2] + C[3] * C[3];
        const R r = U[0] * Num<R>::rcp(C[0]);
        const bool keep = Ff2 <= U[0] * U[0] && Ff2 > Fc2 * (r * r);
        if (!keep) {
            U[1] = C[1] * r;
            U[2] = C[2] * r;
            U[3] = C[3] * r;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) U[q] = C[q];
    }
}

// Donor-cell quantities of the f-preserving fix, |F_c|^2 and 1 / E_c,
// computed once per cell and plane for all the faces the cell feeds.
template <typename R>
struct Centre {
    R f2, ie;
};
template <typename R>
__device__ __forceinline__ Centre<R> centre_of(const R C[4])
{
    return {C[1] * C[1] + C[2] * C[2] + C[3] * C[3], Num<R>::rcp(C[0])};
}

// ffix_sq with the donor cell's quantities supplied
// (E_face <= 0 falls back to the centre state: ratio 1 and E_face = E_c).
template <typename R>
__device__ __forceinline__ void ffix_sq_c(R U[4], const R C[4], Centre<R> cc)
{
    const bool pos = U[0] > R(0);
    const R Ff2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    const R r = pos ? U[0] * cc.ie : R(1);
    const bool keep = pos && Ff2 <= U[0] * U[0] && Ff2 > cc.f2 * (r * r);
    if (!keep) {
        U[1] = C[1] * r;
        U[2] = C[2] * r;
        U[3] = C[3] * r;
    }
    U[0] = pos ? U[0] : C[0];
}

// Face treatment selected at run time: the f-preserving fix (default), the
// "PLUTO" flat fallback or the simple clip (the alternatives of Sect. 2.5 and
// the beam comparison of Sect. 3.2); both alternatives act only when
// |R(F)| > R(E) and fall back to the flat state for R(E) <= 0.
template <typename R>
__device__ __forceinline__ void face_fix(int recon, R U[4], const R C[4])
{
    if (recon == M1_RECON_FPRESERVE) {
        ffix_sq(U, C);
        return;
    }
    const R Ff2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    if (U[0] > R(0) && Ff2 <= U[0] * U[0]) return;
    if (recon == M1_RECON_CLIP && U[0] > R(0)) {
        const R sc = U[0] * Num<R>::rcp(Num<R>::sqrt_(Ff2));
        U[1] *= sc;
        U[2] *= sc;
        U[3] *= sc;
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) U[q] = C[q];
}

// the hardware's legacy multiply, 0 x anything = 0 (through the compiler's
// intrinsic, so its scheduling and hazard rules apply)
extern "C" __device__ float amdgcn_fmul_legacy(float, float) __asm("llvm.amdgcn.fmul.legacy");

// van Leer limited slope without a branch, as
// (dl |dr| + |dl| dr) / (|dl| + |dr|): the harmonic mean 2 dl dr / (dl + dr)
// when the signs agree, zero when they differ or either is zero.  FP32 uses
// the legacy multiply (0 x inf = 0), so dl = dr = 0 gives 0 without a select
// (and a subnormal |dl| + |dr|, whose reciprocal overflows, has num = 0).
template <typename R>
__device__ __forceinline__ R vanleer_fast(R dl, R dr);
template <>
__device__ __forceinline__ float vanleer_fast<float>(float dl, float dr)
{
    const float num = __builtin_fmaf(__builtin_fabsf(dl), dr, dl * __builtin_fabsf(dr));
    return amdgcn_fmul_legacy(num, __builtin_amdgcn_rcpf(__builtin_fabsf(dl) + __builtin_fabsf(dr)));
}
template <>
__device__ __forceinline__ double vanleer_fast<double>(double dl, double dr)
{
    const double den = __builtin_fabs(dl) + __builtin_fabs(dr);
    const double num = __builtin_fma(__builtin_fabs(dl), dr, dl * __builtin_fabs(dr));
    // |dl| + |dr| under the smallest normal number gives 0 (the limited
    // slope is below half of it), keeping the reciprocal finite
    return den >= Num<double>::tiny ? num * Num<double>::rcp(den) : 0.0;
}

// HLL flux c_hat Phi* at the face between donor cells b (left) and c (right)
// along d from their states, van Leer slopes (sb, sc; per unit length) and
// f-fix quantities (cb, cc):
// face states q_b + s_b hp_b and q_c - s_c hm_c, the face fix, both
// closures and the optical-depth-limited HLL (or LF) flux.
template <typename R>
__device__ __forceinline__ void face_flux_s(int d, const R qb[4], const R qc[4], const R sb[4], const R sc[4],
                                            Centre<R> cb, Centre<R> cc, R hpL, R hmR, R tauL, R tauR, R c_hat,
                                            R out[4], int recon = M1_RECON_FPRESERVE,
                                            int riemann = M1_RIEMANN_HLL)
{
    R UL[4], UR[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        UL[v] = qb[v] + sb[v] * hpL;
        UR[v] = qc[v] - sc[v] * hmR;
    }
    if (recon == M1_RECON_FPRESERVE) {
        ffix_sq_c(UL, qb, cb);
        ffix_sq_c(UR, qc, cc);
    } else {
        face_fix(recon, UL, qb);
        face_fix(recon, UR, qc);
    }
    const Wave<R> wl = closure_wave_rt(UL[0], UL[1], UL[2], UL[3], d);
    const Wave<R> wr = closure_wave_rt(UR[0], UR[1], UR[2], UR[3], d);
    const R tau = R(0.5) * (tauL + tauR);
    // optical-depth limit 4 / (3 tau) (none for tau = 0, or below the
    // normal range)
    const R lim = tau >= Num<R>::tiny ? R(4) / R(3) * Num<R>::rcp(tau) : R(__builtin_inf());
    const R lamL = vmax(vmin(wl.lm, wr.lm), -lim);
    const R lamR = vmin(vmax(wl.lp, wr.lp), lim);
    if (riemann == M1_RIEMANN_LF) {
        // Lax-Friedrichs-Rusanov: largest limited speed magnitude
        const R sp = vmax(__builtin_fabs(lamL), __builtin_fabs(lamR));
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = c_hat * (R(0.5) * (wl.phi[q] + wr.phi[q]) - R(0.5) * sp * (UR[q] - UL[q]));
        return;
    }
    const R SL = vmin(lamL, R(0));
    const R SR = vmax(lamR, R(0));
    if (SR > SL) {
        const R k = c_hat * Num<R>::rcp(SR - SL);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = k * (SR * wl.phi[q] - SL * wr.phi[q] + SL * SR * (UR[q] - UL[q]));
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = c_hat * R(0.5) * (wl.phi[q] + wr.phi[q]);
    }
}

// van Leer slopes of the four fields of cell m from cells m-1, m, m+1 and the
// inverse centre spacings wl = 1/(x_m - x_{m-1}), wr = 1/(x_{m+1} - x_m).
template <typename R>
__device__ __forceinline__ void slopes4(const R qm[4], const R q0[4], const R qp[4], R wl, R wr, R s[4])
{
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = vanleer_fast((q0[v] - qm[v]) * wl, (qp[v] - q0[v]) * wr);
}

// LimO3 limited slope (Cada and Torrilhon 2009, the compact third-order
// reconstruction Sect. 2.5 names) of a cell for its face on the side of the
// divided difference dnear, dfar being the one on the other side:
// phi(theta) dnear with theta = dfar / dnear and
//   phi = max(0, min(p3, max(-theta/2, min(2 theta, p3, 3/2)))),
//   p3 = (2 + theta) / 3 (the unlimited third-order reconstruction).
// Evaluated without a division: with s = sign(dnear), a = s dfar and
// b = |dnear|, phi dnear = s b phi, and b >= 0 scales through every min and
// max, so phi dnear = s max(0, min(q, max(-a/2, min(2a, q, 3b/2)))) with
// q = (2b + a) / 3; dnear = 0 gives 0 (the limit of phi dnear).
template <typename R>
__device__ __forceinline__ R limo3(R dfar, R dnear)
{
    const R s = dnear < R(0) ? R(-1) : R(1);
    const R a = s * dfar, b = s * dnear;
    const R q = (R(2) * b + a) * R(1.0 / 3.0);
    const R inner = vmin(vmin(R(2) * a, q), R(1.5) * b);
    return s * vmax(R(0), vmin(q, vmax(R(-0.5) * a, inner)));
}

// LimO3 slopes of the four fields of cell m from cells m-1, m, m+1: lo for
// the lower face (near side m-1), hi for the upper face (near side m+1).
template <typename R>
__device__ __forceinline__ void limo3_slopes4(const R qm[4], const R q0[4], const R qp[4], R wl, R wr, R lo[4],
                                              R hi[4])
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const R dl = (q0[v] - qm[v]) * wl, dr = (qp[v] - q0[v]) * wr;
        hi[v] = limo3(dl, dr);
        lo[v] = limo3(dr, dl);
    }
}

} // namespace m1
