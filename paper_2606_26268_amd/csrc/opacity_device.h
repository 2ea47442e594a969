// opacity_device.h -- absorption opacities at (rho, T) on the device:
// constant, power law and bilinear interpolation of a log10 kappa table.
// The MLP surrogate lives in mlp_device.h (it needs a whole wavefront).
#pragma once
#include <hip/hip_runtime.h>

#include "m1_internal.h"

namespace m1 {

template <typename R> struct OMath;
template <> struct OMath<double> {
    static __device__ __forceinline__ double log10_(double x) { return log10(x); }
    static __device__ __forceinline__ double exp10_(double x) { return exp10(x); }
    static __device__ __forceinline__ double pow_(double x, double y) { return pow(x, y); }
    static __device__ __forceinline__ double floor_(double x) { return floor(x); }
};
template <> struct OMath<float> {
    static __device__ __forceinline__ float log10_(float x) { return log10f(x); }
    static __device__ __forceinline__ float exp10_(float x) { return exp10f(x); }
    static __device__ __forceinline__ float pow_(float x, float y) { return powf(x, y); }
    static __device__ __forceinline__ float floor_(float x) { return floorf(x); }
};

// Table coordinates (log10 rho + lr_off, log10 T + lt_off) clamped to the axes.
// Here and in the interpolation below contraction is off: inlined into
// different kernels, the sums would otherwise fuse with neighbouring products
// (the logarithm's last step, a weight) in one kernel and not in another, and
// the opacity cache written by the implicit step would differ in the last bit
// from the one derived again from the stored state.
template <typename R>
__device__ __forceinline__ void table_coords(const OpacityParams &op, R rho, R T, R &lr, R &lt)
{
#pragma clang fp contract(off)
    lr = OMath<R>::log10_(rho) + R(op.lr_off);
    lt = OMath<R>::log10_(T) + R(op.lt_off);
    lr = lr < R(op.lr0) ? R(op.lr0) : (lr > R(op.lr1) ? R(op.lr1) : lr);
    lt = lt < R(op.lt0) ? R(op.lt0) : (lt > R(op.lt1) ? R(op.lt1) : lt);
}

// Bilinear interpolation of log10 kappa_P and kappa_R at clamped (lr, lt);
// both tables share the node grid; the four node values of the cell come
// from its record (see OpacityParams::tab_cells).
template <typename R>
__device__ __forceinline__ void table_lookup(const OpacityParams &op, R lr, R lt, R &lkP, R &lkR)
{
#pragma clang fp contract(off)
    const R u = (lr - R(op.lr0)) / (R(op.lr1) - R(op.lr0)) * R(op.nr - 1);
    const R v = (lt - R(op.lt0)) / (R(op.lt1) - R(op.lt0)) * R(op.nt - 1);
    int i = int(OMath<R>::floor_(u)), j = int(OMath<R>::floor_(v));
    i = i > op.nr - 2 ? op.nr - 2 : (i < 0 ? 0 : i);
    j = j > op.nt - 2 ? op.nt - 2 : (j < 0 ? 0 : j);
    const R wu = u - R(i), wv = v - R(j);
    // the cell's record: kappa_P, then kappa_R, at nodes (i, j), (i+1, j),
    // (i, j+1), (i+1, j+1)
    const float4 *rec = reinterpret_cast<const float4 *>(op.tab_cells) + 2 * (j * (op.nr - 1) + i);
    const float4 P = rec[0], Q = rec[1];
    const R w00 = (R(1) - wu) * (R(1) - wv), w10 = wu * (R(1) - wv);
    const R w01 = (R(1) - wu) * wv, w11 = wu * wv;
    lkP = w00 * R(P.x) + w10 * R(P.y) + w01 * R(P.z) + w11 * R(P.w);
    lkR = w00 * R(Q.x) + w10 * R(Q.y) + w01 * R(Q.z) + w11 * R(Q.w);
}

// kappa_P, kappa_R of the analytic models and the table (OPK != MLP).
template <typename R, int OPK>
__device__ __forceinline__ void opacity_analytic(const OpacityParams &op, R rho, R T, R &kP, R &kR)
{
    if (OPK == OPK_CONST) {
        kP = R(op.kP);
        kR = R(op.kR);
    } else if (OPK == OPK_POWERLAW) {
        const R k = R(op.k0) * OMath<R>::pow_(rho / R(op.rho0), R(op.alpha)) *
                    OMath<R>::pow_(T / R(op.T0), R(op.beta));
        kP = k;
        kR = k;
    } else {
        R lr, lt, a, b;
        table_coords<R>(op, rho, T, lr, lt);
        table_lookup<R>(op, lr, lt, a, b);
        kP = OMath<R>::exp10_(a);
        kR = OMath<R>::exp10_(b);
    }
}

} // namespace m1
