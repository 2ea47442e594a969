/*
 * transport.c -- oracle: grid geometry, boundary ghosts, PLM + f-fix
 * reconstruction, HLL interface fluxes and the conservative update of one
 * explicit radiation transport step.  Test infrastructure only.
 *
 * One Euler stage of the paper's step list (Sect. 2.4): boundary values,
 * reconstruction on faces, f <= 1 on faces, wave speeds, Riemann fluxes,
 * flux divergence in each direction (all directions from the same state).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "m1_oracle.h"

/* ------------------------------------------------------------------------ */
/* grid                                                                     */
/* ------------------------------------------------------------------------ */

/* Geometry of cell (i, j, k):
 *   out[0]      volume V
 *   out[1..3]   area of the lower face normal to d = 0, 1, 2
 *   out[4..6]   area of the upper face normal to d = 0, 1, 2
 *   out[7]      1 / r_eff  (cylindrical: 1/R_eff, Cartesian: 0)
 *   out[8]      cot(theta)_eff (spherical only)
 *   out[9..11]  cell extent h_d used by the optical depth and the CFL rule
 * Cylindrical axes are (R, phi, z), spherical axes (r, theta, phi).  The
 * effective radius and cotangent are the ratios that make a static
 * isotropic radiation field an exact discrete equilibrium. */
void m1o_cell_geometry(const m1o_problem *p, int i, int j, int k, double out[12])
{
    const double *x0 = p->faces[0], *x1 = p->faces[1], *x2 = p->faces[2];
    double a0 = x0[i], b0 = x0[i + 1], a1 = x1[j], b1 = x1[j + 1], a2 = x2[k], b2 = x2[k + 1];
    double d0 = b0 - a0, d1 = b1 - a1, d2 = b2 - a2;
    memset(out, 0, 12 * sizeof(double));
    if (p->geometry == M1O_CARTESIAN) {
        out[0] = d0 * d1 * d2;
        out[1] = out[4] = d1 * d2;
        out[2] = out[5] = d0 * d2;
        out[3] = out[6] = d0 * d1;
        out[9] = d0; out[10] = d1; out[11] = d2;
    } else if (p->geometry == M1O_CYLINDRICAL) {
        double ring = 0.5 * (b0 * b0 - a0 * a0);
        out[0] = ring * d1 * d2;
        out[1] = a0 * d1 * d2;
        out[4] = b0 * d1 * d2;
        out[2] = out[5] = d0 * d2;
        out[3] = out[6] = ring * d1;
        out[7] = (out[4] - out[1]) / out[0];
        double Rc = 0.5 * (a0 + b0);
        out[9] = d0; out[10] = Rc * d1; out[11] = d2;
    } else {
        double dmu = cos(a1) - cos(b1);
        double shell = (b0 * b0 * b0 - a0 * a0 * a0) / 3.0;
        double ring = 0.5 * (b0 * b0 - a0 * a0);
        out[0] = shell * dmu * d2;
        out[1] = a0 * a0 * dmu * d2;
        out[4] = b0 * b0 * dmu * d2;
        out[2] = ring * sin(a1) * d2;
        out[5] = ring * sin(b1) * d2;
        out[3] = out[6] = ring * d1;
        out[7] = (out[4] - out[1]) / (2.0 * out[0]);
        out[8] = (sin(b1) - sin(a1)) / dmu;
        double rc = 0.5 * (a0 + b0), thc = 0.5 * (a1 + b1);
        out[9] = d0; out[10] = rc * d1; out[11] = rc * sin(thc) * d2;
    }
}

/* dt = cfl / max over cells of c_hat * sum_{d < ndim} 1/h_d. */
double m1o_max_dt(const m1o_problem *p, double cfl)
{
    double worst = 0.0, g[12];
    for (int k = 0; k < p->n[2]; ++k)
        for (int j = 0; j < p->n[1]; ++j)
            for (int i = 0; i < p->n[0]; ++i) {
                m1o_cell_geometry(p, i, j, k, g);
                double s = 0.0;
                for (int d = 0; d < p->ndim; ++d) s += 1.0 / g[9 + d];
                if (s > worst) worst = s;
            }
    return cfl / (p->c_hat * worst);
}

/* ------------------------------------------------------------------------ */
/* boundary ghosts                                                          */
/* ------------------------------------------------------------------------ */

/* Interior index that supplies ghost index t along d: periodic wrap, the
 * mirror image for a reflective side, or the nearest interior cell for
 * outflow (zero-gradient copy) and fixed sides (whose state is replaced, see
 * ghost_state; the optical depth is the nearest interior cell's). */
static int src_index(const m1o_problem *p, int d, int t)
{
    int n = p->n[d];
    if (t >= 0 && t < n) return t;
    int bc = p->bc[d][t < 0 ? 0 : 1];
    if (bc == M1O_PERIODIC) return ((t % n) + n) % n;
    if (bc == M1O_REFLECT) return t < 0 ? -1 - t : 2 * n - 1 - t;
    return t < 0 ? 0 : n - 1;
}

/* State (E, Fx, Fy, Fz) of cell c whose index along d is t (possibly a
 * ghost): a reflective ghost is the mirror cell with its F component normal
 * to the boundary reversed; a fixed ghost carries the side's given state. */
static void ghost_state(const m1o_problem *p, const double *const st[9], int d, const int c[3], int t,
                        double q[4])
{
    int n = p->n[d];
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] = src_index(p, d, t);
    long id = ((long)cc[2] * p->n[1] + cc[1]) * p->n[0] + cc[0];
    for (int v = 0; v < 4; ++v) q[v] = st[v][id];
    if (t >= 0 && t < n) return;
    int side = t < 0 ? 0 : 1, bc = p->bc[d][side];
    if (bc == M1O_REFLECT) q[1 + d] = -q[1 + d];
    if (bc == M1O_FIXED)
        for (int v = 0; v < 4; ++v) q[v] = p->bc_state[d][side][v];
}

/* Lower / upper face and centre coordinate of (possibly ghost) index t along d.
 * Periodic ghosts are shifted copies, reflective ghosts mirror images of the
 * interior cells; outflow and fixed ghosts repeat the edge width. */
static void coords(const m1o_problem *p, int d, int t, double *lo, double *c, double *hi)
{
    int n = p->n[d];
    const double *x = p->faces[d];
    int bc = (t >= 0 && t < n) ? -1 : p->bc[d][t < 0 ? 0 : 1];
    if (bc < 0) {
        *lo = x[t]; *hi = x[t + 1];
    } else if (bc == M1O_PERIODIC) {
        int w = src_index(p, d, t);
        double shift = (double)((t - w) / n) * (x[n] - x[0]);
        *lo = x[w] + shift; *hi = x[w + 1] + shift;
    } else if (bc == M1O_REFLECT) {
        int m = src_index(p, d, t);
        double wall = t < 0 ? x[0] : x[n];
        *lo = 2.0 * wall - x[m + 1]; *hi = 2.0 * wall - x[m];
    } else if (t < 0) {
        double h = x[1] - x[0];
        *lo = x[0] + t * h; *hi = *lo + h;
    } else {
        double h = x[n] - x[n - 1];
        *lo = x[n] + (t - n) * h; *hi = *lo + h;
    }
    *c = 0.5 * (*lo + *hi);
}

static long lin(const m1o_problem *p, const int c[3])
{
    return ((long)c[2] * p->n[1] + c[1]) * p->n[0] + c[0];
}

/* ------------------------------------------------------------------------ */
/* reconstruction                                                           */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea and Flood 2014): a counter-based
 * generator, so the value for a given key is the same in every thread. */
static unsigned long long splitmix64(unsigned long long x)
{
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform in [-1, 1) for the face value of field v of cell (c with index t
 * along d) on side `side`, under seed */
static double face_noise_unit(unsigned long long seed, int d, int side, int t, const int c[3], int v)
{
    unsigned long long k = splitmix64(seed);
    const long long parts[7] = {d, side, t + 2, c[0], c[1], c[2], v};
    for (int i = 0; i < 7; ++i) k = splitmix64(k ^ (unsigned long long)parts[i]);
    return (double)(k >> 11) * (1.0 / 4503599627370496.0) - 1.0;
}

/* Reconstruction of (E, Fx, Fy, Fz) of cell t along d on its upper face
 * (side = +1) or lower face (side = -1): piecewise linear with the van Leer
 * slope, or LimO3, whose slope depends on the face (the difference on the
 * face side is the near one); then the face treatment (f-preserving fix by
 * default) against that cell's centre values.  The slopes use divided
 * differences over centre spacings. */
static void face_state(const m1o_problem *p, const double *const st[9], int d, int cbase[3],
                       int t, int side, double U[4])
{
    int c[3] = {cbase[0], cbase[1], cbase[2]};
    double q[3][4], xc[3], lo, hi, xm;
    for (int s = -1; s <= 1; ++s) {
        ghost_state(p, st, d, c, t + s, q[s + 1]);
        coords(p, d, t + s, &lo, &xc[s + 1], &hi);
    }
    coords(p, d, t, &lo, &xm, &hi);
    double off = side > 0 ? (hi - xm) : -(xm - lo);
    for (int v = 0; v < 4; ++v) {
        double dl = (q[1][v] - q[0][v]) / (xc[1] - xc[0]);
        double dr = (q[2][v] - q[1][v]) / (xc[2] - xc[1]);
        double slope;
        if (p->limiter == M1O_LIMO3)
            slope = side > 0 ? m1o_limo3(dl, dr) : m1o_limo3(dr, dl);
        else
            slope = m1o_vanleer(dl, dr);
        U[v] = q[1][v] + slope * off;
        if (p->face_noise > 0.0)
            U[v] += p->face_noise * (fabs(q[1][v]) + fabs(slope * off)) *
                    face_noise_unit(p->noise_seed, d, side, t, c, v);
    }
    double Fc[3] = {q[1][1], q[1][2], q[1][3]};
    double Ff[3] = {U[1], U[2], U[3]};
    m1o_face_fix(p->recon, &U[0], Ff, q[1][0], Fc);
    U[1] = Ff[0]; U[2] = Ff[1]; U[3] = Ff[2];
}

/* ------------------------------------------------------------------------ */
/* per-cell optical depth at the start of the step                          */
/* ------------------------------------------------------------------------ */

static double gas_temperature(const m1o_problem *p, double rho, double mx, double my,
                              double mz, double Eg)
{
    double Cv = rho / (p->gamma - 1.0);
    return (Eg - 0.5 * (mx * mx + my * my + mz * mz) / rho) / Cv;
}

static void cell_tau(const m1o_problem *p, const double *const st[9], double *tau)
{
    long N = (long)p->n[0] * p->n[1] * p->n[2];
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int c[3] = {(int)(id % p->n[0]), (int)((id / p->n[0]) % p->n[1]),
                    (int)(id / ((long)p->n[0] * p->n[1]))};
        double g[12], kP, kR;
        double rho = st[4][id];
        double T = gas_temperature(p, rho, st[5][id], st[6][id], st[7][id], st[8][id]);
        m1o_opacity(p, rho, T, &kP, &kR);
        m1o_cell_geometry(p, c[0], c[1], c[2], g);
        double hmax = 0.0;
        for (int d = 0; d < p->ndim; ++d) if (g[9 + d] > hmax) hmax = g[9 + d];
        tau[id] = rho * (kR + p->sigma) * hmax;
    }
}

/* ------------------------------------------------------------------------ */
/* explicit step                                                            */
/* ------------------------------------------------------------------------ */

int m1o_explicit(const m1o_problem *p, double dt, const double *const st[9],
                 double *const out[4], long long cnt[M1O_NCNT])
{
    const int *n = p->n;
    long N = (long)n[0] * n[1] * n[2];
    double *tau = malloc(N * sizeof(double));
    double *flux[3] = {0, 0, 0};
    if (!tau) return -1;
    cell_tau(p, st, tau);

    /* interface fluxes: face f along d sits between cells f-1 and f */
    for (int d = 0; d < p->ndim; ++d) {
        int nf[3] = {n[0], n[1], n[2]};
        nf[d] += 1;
        long NF = (long)nf[0] * nf[1] * nf[2];
        flux[d] = malloc(NF * 4 * sizeof(double));
        if (!flux[d]) return -1;
#pragma omp parallel for schedule(static)
        for (long fid = 0; fid < NF; ++fid) {
            int c[3] = {(int)(fid % nf[0]), (int)((fid / nf[0]) % nf[1]),
                        (int)(fid / ((long)nf[0] * nf[1]))};
            int f = c[d];
            double UL[4], UR[4], out4[4];
            face_state(p, st, d, c, f - 1, +1, UL);
            face_state(p, st, d, c, f, -1, UR);
            int ca[3] = {c[0], c[1], c[2]}, cb[3] = {c[0], c[1], c[2]};
            ca[d] = src_index(p, d, f - 1);
            cb[d] = src_index(p, d, f);
            double tface = 0.5 * (tau[lin(p, ca)] + tau[lin(p, cb)]);
            if (p->riemann == M1O_LF)
                m1o_lf(UL, UR, d, tface, p->c_hat, out4);
            else
                m1o_hll(UL, UR, d, tface, p->c_hat, out4, NULL, NULL);
            for (int q = 0; q < 4; ++q) flux[d][fid * 4 + q] = out4[q];
        }
    }

    long long efl = 0, ffx = 0;
#pragma omp parallel for schedule(static) reduction(+ : efl, ffx)
    for (long id = 0; id < N; ++id) {
        int c[3] = {(int)(id % n[0]), (int)((id / n[0]) % n[1]), (int)(id / ((long)n[0] * n[1]))};
        double g[12];
        m1o_cell_geometry(p, c[0], c[1], c[2], g);
        double U[4] = {st[0][id], st[1][id], st[2][id], st[3][id]};
        double acc[4] = {0, 0, 0, 0};
        for (int d = 0; d < p->ndim; ++d) {
            int nf[3] = {n[0], n[1], n[2]};
            nf[d] += 1;
            int lo[3] = {c[0], c[1], c[2]}, hi[3] = {c[0], c[1], c[2]};
            hi[d] += 1;
            long flo = ((long)lo[2] * nf[1] + lo[1]) * nf[0] + lo[0];
            long fhi = ((long)hi[2] * nf[1] + hi[1]) * nf[0] + hi[0];
            for (int q = 0; q < 4; ++q)
                acc[q] += g[4 + d] * flux[d][fhi * 4 + q] - g[1 + d] * flux[d][flo * 4 + q];
        }
        /* an inactive (ignorable) direction has no variation: both of its
         * faces carry the physical flux of the cell's own state */
        for (int d = p->ndim; d < 3; ++d) {
            double phi[4];
            m1o_flux(U[0], U[1], U[2], U[3], d, phi);
            for (int q = 0; q < 4; ++q) acc[q] += (g[4 + d] - g[1 + d]) * p->c_hat * phi[q];
        }
        double Us[4];
        for (int q = 0; q < 4; ++q) Us[q] = U[q] - dt * acc[q] / g[0];

        /* geometric sources of the flux equation from the cell-centre
         * pressure tensor P = D E (divergence of a symmetric tensor in
         * orthonormal curvilinear components) */
        if (p->geometry != M1O_CARTESIAN) {
            double f, xi, D[9], P[9];
            m1o_eddington(U[0], U[1], U[2], U[3], &f, &xi, D);
            for (int a = 0; a < 9; ++a) P[a] = D[a] * U[0];
            double S[3] = {0, 0, 0};
            if (p->geometry == M1O_CYLINDRICAL) {       /* (R, phi, z) */
                S[0] = P[4] * g[7];
                S[1] = -P[1] * g[7];
            } else {                                     /* (r, theta, phi) */
                S[0] = (P[4] + P[8]) * g[7];
                S[1] = (g[8] * P[8] - P[1]) * g[7];
                S[2] = -(P[2] + g[8] * P[5]) * g[7];
            }
            for (int a = 0; a < 3; ++a) Us[1 + a] += dt * p->c_hat * S[a];
        }

        /* positivity floor on E, then f <= 1 at the cell centre */
        if (Us[0] < p->e_floor) { Us[0] = p->e_floor; ++efl; }
        double Fn = sqrt(Us[1] * Us[1] + Us[2] * Us[2] + Us[3] * Us[3]);
        if (Fn > Us[0]) {
            double s = Us[0] / Fn;
            Us[1] *= s; Us[2] *= s; Us[3] *= s;
            ++ffx;
        }
        for (int q = 0; q < 4; ++q) out[q][id] = Us[q];
    }
    cnt[M1O_CNT_EFLOOR] += efl;
    cnt[M1O_CNT_FFIX_TRANSPORT] += ffx;
    for (int d = 0; d < 3; ++d) free(flux[d]);
    free(tau);
    return 0;
}

/* One full step = explicit transport then the implicit source step; the
 * state arrays (E, Fx, Fy, Fz, rho, mx, my, mz, Eg) are updated in place. */
int m1o_run(const m1o_problem *p, double dt, int nsteps, double *const st[9],
            long long cnt[M1O_NCNT])
{
    long N = (long)p->n[0] * p->n[1] * p->n[2];
    double *buf = malloc(4 * N * sizeof(double));
    if (!buf) return -1;
    double *star[4] = {buf, buf + N, buf + 2 * N, buf + 3 * N};
    m1o_problem q = *p;
    for (int s = 0; s < nsteps; ++s) {
        q.noise_seed = p->noise_seed + (unsigned long long)s;
        if (m1o_explicit(&q, dt, (const double *const *)st, star, cnt)) { free(buf); return -1; }
        if (m1o_implicit(p, dt, (const double *const *)star, st, cnt)) { free(buf); return -1; }
    }
    free(buf);
    return 0;
}

/* Second-order Runge-Kutta stepping (Heun / SSP-RK2) with the split step as
 * the stage operator, as the integration scheme of Sect. 2.4 applies the
 * transport + source sequence to every sub-step:
 *   U1 = S(T(U^n)),  U2 = S(T(U1)),  U^{n+1} = (U^n + U2) / 2
 * for the radiation (E, F) and the gas (m, E_g); rho is frozen. */
int m1o_run_rk2(const m1o_problem *p, double dt, int nsteps, double *const st[9],
                long long cnt[M1O_NCNT])
{
    long N = (long)p->n[0] * p->n[1] * p->n[2];
    double *save = malloc(9 * N * sizeof(double));
    if (!save) return -1;
    for (int s = 0; s < nsteps; ++s) {
        for (int f = 0; f < 9; ++f) memcpy(save + f * N, st[f], N * sizeof(double));
        if (m1o_run(p, dt, 2, st, cnt)) { free(save); return -1; }
        for (int f = 0; f < 9; ++f) {
            if (f == 4) continue;
#pragma omp parallel for schedule(static)
            for (long id = 0; id < N; ++id) st[f][id] = 0.5 * (save[f * N + id] + st[f][id]);
        }
    }
    free(save);
    return 0;
}

