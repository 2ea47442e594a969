// transport.hip -- explicit M1 transport step on gfx950.
//
// One Euler stage of the hyperbolic part (Sect. 2.4-2.6): boundary values
// by index mapping in the loader (periodic wrap / outflow copy), PLM van
// Leer reconstruction of (E, F) on faces with the f-preserving fix, the
// Levermore closure and signal speeds of both face states, the HLL flux with
// the optical-depth limiter, and the conservative update with the geometric
// sources of the flux equation in cylindrical / spherical coordinates.
#include "m1_internal.h"
#include "m1_device.h"

namespace m1 {

template <typename R>
struct TArgs {
    const R *U[4];
    const R *tau;
    R *out[4];
    int n[3];
    int bc[3][2];
    int ign[3];
    Metric<R> m;
    R dt, c_hat, e_floor;
    unsigned long long *cnt;
};

// index along one direction after applying the boundary condition
__device__ __forceinline__ int map_index(int t, int n, int lo, int hi)
{
    if (t < 0) {
        if (lo == M1_BC_PERIODIC) { while (t < 0) t += n; return t; }
        return 0;
    }
    if (t >= n) {
        if (hi == M1_BC_PERIODIC) { while (t >= n) t -= n; return t; }
        return n - 1;
    }
    return t;
}

template <typename R>
__device__ __forceinline__ void load4(const TArgs<R> &a, int lin, R q[4])
{
    q[0] = a.U[0][lin];
    q[1] = a.U[1][lin];
    q[2] = a.U[2][lin];
    q[3] = a.U[3][lin];
}

// Contribution of direction D to the flux divergence of the cell at index t
// along D (row base `base`, stride `stride`): reconstruct cells t-1, t, t+1
// (stencil t-2 .. t+2), take HLL fluxes at both faces of cell t and add
// A_hi/V * Phi_hi - A_lo/V * Phi_lo to acc.
template <typename R, int D>
__device__ __forceinline__ void direction_div(const TArgs<R> &a, int base, int stride, int t,
                                              R tr, R acc[4])
{
    const int n = a.n[D], lo = a.bc[D][0], hi = a.bc[D][1];
    R q[5][4];
    int li[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        li[s] = base + map_index(t - 2 + s, n, lo, hi) * stride;
        load4(a, li[s], q[s]);
    }
    const R *winv = a.m.winv[D], *hp = a.m.hp[D], *hm = a.m.hm[D];
    // face states: cell t-1 upper, cell t lower and upper, cell t+1 lower
    R Lm[4], Rt[4], Lt[4], Rp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const R dA = (q[1][v] - q[0][v]) * winv[t + 1];
        const R dB = (q[2][v] - q[1][v]) * winv[t + 2];
        const R dC = (q[3][v] - q[2][v]) * winv[t + 3];
        const R dD = (q[4][v] - q[3][v]) * winv[t + 4];
        const R sm = vanleer(dA, dB), s0 = vanleer(dB, dC), sp = vanleer(dC, dD);
        Lm[v] = q[1][v] + sm * hp[t + 1];
        Rt[v] = q[2][v] - s0 * hm[t + 2];
        Lt[v] = q[2][v] + s0 * hp[t + 2];
        Rp[v] = q[3][v] - sp * hm[t + 3];
    }
    ffix(Lm, q[1]);
    ffix(Rt, q[2]);
    ffix(Lt, q[2]);
    ffix(Rp, q[3]);
    const R tm = a.tau[li[1]], t0 = a.tau[li[2]], tp = a.tau[li[3]];
    R flo[4], fhi[4];
    hll_flux<R, D>(Lm, Rt, R(0.5) * (tm + t0), a.c_hat, flo);
    hll_flux<R, D>(Lt, Rp, R(0.5) * (t0 + tp), a.c_hat, fhi);
    const R al = a.m.alo[D][t] * tr, ah = a.m.ahi[D][t] * tr;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += ah * fhi[v] - al * flo[v];
}

template <typename R, int D>
__device__ __forceinline__ void ignorable_div(const TArgs<R> &a, const R U[4], R tr, R acc[4])
{
    const Wave<R> w = closure_wave<R, D>(U[0], U[1], U[2], U[3]);
    const R dA = (a.m.ahi[D][0] - a.m.alo[D][0]) * tr * a.c_hat;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += dA * w.phi[v];
}

template <typename R, int NDIM, int GEOM>
__global__ void __launch_bounds__(256) k_transport(TArgs<R> a)
{
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int N = n0 * n1 * n2;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const int i = id % n0, j = (id / n0) % n1, k = id / (n0 * n1);
    R U[4];
    load4(a, id, U);
    R acc[4] = {R(0), R(0), R(0), R(0)};

    direction_div<R, 0>(a, id - i, 1, i, R(1), acc);
    if (NDIM >= 2) {
        const R tr = a.m.trA[1][i];
        direction_div<R, 1>(a, id - j * n0, n0, j, tr, acc);
    } else if (a.ign[1]) {
        ignorable_div<R, 1>(a, U, a.m.trA[1][i], acc);
    }
    if (NDIM >= 3) {
        const R tr = a.m.trA[2][i] * a.m.trB[2][j];
        direction_div<R, 2>(a, id - k * n0 * n1, n0 * n1, k, tr, acc);
    } else if (a.ign[2]) {
        ignorable_div<R, 2>(a, U, a.m.trA[2][i] * a.m.trB[2][j], acc);
    }

    R Us[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Us[v] = U[v] - a.dt * acc[v];

    if (GEOM != M1_CARTESIAN) {
        // geometric sources from the cell-centre pressure tensor P = D E
        const R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
        const R Fn = Num<R>::sqrt_(F2);
        R f = Fn / U[0];
        f = f > R(1) ? R(1) : f;
        const R s = Num<R>::sqrt_(R(4) - R(3) * f * f);
        const R xi = (R(3) + R(4) * f * f) / (R(5) + R(2) * s);
        const R inv = Fn > R(0) ? R(1) / Fn : R(0);
        const R n_[3] = {U[1] * inv, U[2] * inv, U[3] * inv};
        const R iso = R(0.5) * (R(1) - xi) * U[0];
        const R an = R(0.5) * (R(3) * xi - R(1)) * U[0];
        const R ir = a.m.inv_reff[i];
        const R k_ = a.dt * a.c_hat * ir;
        if (GEOM == M1_CYLINDRICAL) {           // (R, phi, z)
            const R Ppp = an * n_[1] * n_[1] + iso, PRp = an * n_[0] * n_[1];
            Us[1] += k_ * Ppp;
            Us[2] -= k_ * PRp;
        } else {                                 // (r, theta, phi)
            const R ct = a.m.cot_eff[j];
            const R Ptt = an * n_[1] * n_[1] + iso, Ppp = an * n_[2] * n_[2] + iso;
            const R Prt = an * n_[0] * n_[1], Prp = an * n_[0] * n_[2], Ptp = an * n_[1] * n_[2];
            Us[1] += k_ * (Ptt + Ppp);
            Us[2] += k_ * (ct * Ppp - Prt);
            Us[3] -= k_ * (Prp + ct * Ptp);
        }
    }

    // positivity floor on E, then f <= 1 at the cell centre
    if (Us[0] < a.e_floor) {
        Us[0] = a.e_floor;
        atomicAdd(&a.cnt[0], 1ull);
    }
    const R Fn = Num<R>::sqrt_(Us[1] * Us[1] + Us[2] * Us[2] + Us[3] * Us[3]);
    if (Fn > Us[0]) {
        const R sc = Us[0] / Fn;
        Us[1] *= sc;
        Us[2] *= sc;
        Us[3] *= sc;
        atomicAdd(&a.cnt[1], 1ull);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) a.out[v][id] = Us[v];
}

template <typename R>
static hipError_t launch_t(m1_ctx *c, double dt, const Metric<R> &met)
{
    TArgs<R> a;
    for (int v = 0; v < 4; ++v) a.out[v] = static_cast<R *>(c->star[v]);
    a.U[0] = static_cast<const R *>(c->f.E);
    a.U[1] = static_cast<const R *>(c->f.Fx);
    a.U[2] = static_cast<const R *>(c->f.Fy);
    a.U[3] = static_cast<const R *>(c->f.Fz);
    a.tau = static_cast<const R *>(c->tau);
    for (int d = 0; d < 3; ++d) {
        a.n[d] = c->n[d];
        a.bc[d][0] = c->bc[d][0];
        a.bc[d][1] = c->bc[d][1];
        a.ign[d] = c->ign[d];
    }
    a.m = met;
    a.dt = R(dt);
    a.c_hat = R(c->c_hat);
    a.e_floor = R(c->par.e_floor);
    a.cnt = c->cnt;
    const int N = c->n[0] * c->n[1] * c->n[2];
    dim3 block(256), grid((N + 255) / 256);
#define M1_LAUNCH(ND, G) \
    hipLaunchKernelGGL((k_transport<R, ND, G>), grid, block, 0, c->stream, a)
#define M1_GEOMS(ND)                                                      \
    switch (c->geom) {                                                    \
    case M1_CARTESIAN: M1_LAUNCH(ND, M1_CARTESIAN); break;                \
    case M1_CYLINDRICAL: M1_LAUNCH(ND, M1_CYLINDRICAL); break;            \
    default: M1_LAUNCH(ND, M1_SPHERICAL); break;                          \
    }
    switch (c->ndim) {
    case 1: M1_GEOMS(1); break;
    case 2: M1_GEOMS(2); break;
    default: M1_GEOMS(3); break;
    }
#undef M1_GEOMS
#undef M1_LAUNCH
    return hipGetLastError();
}

hipError_t launch_transport(m1_ctx *c, double dt)
{
    if (c->par.precision == M1_F32) return launch_t<float>(c, dt, c->met32);
    return launch_t<double>(c, dt, c->met64);
}

} // namespace m1
