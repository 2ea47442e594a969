/*
 * multigroup.c -- oracle: multigroup M1 (Sect. 2.3 and 2.8: one gray M1
 * fluid per frequency group, coupled to the gas by an (m+1)^2 implicit
 * system).  Test infrastructure only.
 *
 * Groups g = 0 .. m-1 cover x = nu / T in [x_g, x_{g+1}) with x_0 = 0 and
 * x_m = infinity (nu in temperature units, h nu / k).  Each group is
 * transported as an independent gray fluid with constant opacities
 * (kappa_P,g, kappa_R,g).  In the implicit step group g emits the fraction
 * b_g(T^n) of a T^4, the Planck fraction of its band at the start-of-step
 * temperature; (T')^4 is linearised as in the gray system, b_g is frozen.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "m1_oracle.h"

/* Fraction of the Planck energy density below x = h nu / k T:
 * P(x) = (15 / pi^4) int_0^x t^3 / (e^t - 1) dt.
 * Small x: the Bernoulli series t / (e^t - 1) = sum B_k t^k / k!, integrated
 * term by term; large x: 1 minus the tail sum over n of
 * int_x^inf t^3 e^{-n t} dt = e^{-n x} (x^3/n + 3 x^2/n^2 + 6 x/n^3 + 6/n^4). */
double m1o_planck_cdf(double x)
{
    const double pi = 3.14159265358979323846;
    const double norm = 15.0 / (pi * pi * pi * pi);
    if (x <= 0.0) return 0.0;
    if (x < 1.0) {
        /* Bernoulli numbers B_0 .. B_20 (odd ones beyond B_1 vanish) */
        static const double B[21] = {1.0, -0.5, 1.0 / 6, 0, -1.0 / 30, 0, 1.0 / 42, 0, -1.0 / 30, 0,
                                     5.0 / 66, 0, -691.0 / 2730, 0, 7.0 / 6, 0, -3617.0 / 510, 0,
                                     43867.0 / 798, 0, -174611.0 / 330};
        double sum = 0.0, fact = 1.0, xp = x * x * x;
        for (int k = 0; k <= 20; ++k) {
            if (k > 0) fact *= k;
            if (B[k] != 0.0) sum += B[k] * xp / ((k + 3) * fact);
            xp *= x;
        }
        return norm * sum;
    }
    double tail = 0.0;
    for (int n = 1; n <= 64; ++n) {
        double e = exp(-n * x);
        if (e < 1e-300) break;
        double dn = n;
        tail += e * (x * x * x / dn + 3.0 * x * x / (dn * dn) + 6.0 * x / (dn * dn * dn) + 6.0 / (dn * dn * dn * dn));
    }
    return 1.0 - norm * tail;
}

/* b_g(T) for the m groups with interior edges x_1 .. x_{m-1} (in units of T). */
void m1o_group_fractions(int m, const double *edges, double T, double *b)
{
    double lo = 0.0;
    for (int g = 0; g < m; ++g) {
        double hi = g + 1 < m ? m1o_planck_cdf(edges[g] / T) : 1.0;
        b[g] = hi - lo;
        lo = hi;
    }
}

/* Solve A x = r (n x n, row-major, overwritten) by Gaussian elimination with
 * partial pivoting, in extended precision.  Returns 0, or -1 for a singular
 * matrix. */
static int gauss_solve(int n, long double *A, long double *r, long double *x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabsl(A[i * n + c]) > fabsl(A[piv * n + c])) piv = i;
        if (A[piv * n + c] == 0.0L) return -1;
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                long double t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t;
            }
            long double t = r[c]; r[c] = r[piv]; r[piv] = t;
        }
        for (int i = c + 1; i < n; ++i) {
            long double f = A[i * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[i * n + j] -= f * A[c * n + j];
            r[i] -= f * r[c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        long double s = r[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
        x[i] = s / A[i * n + i];
    }
    return 0;
}

/* One cell of the multigroup implicit step: the (m+1)^2 system
 *   (1 + gr_g) E'_g - 4 gr_g b_g a T^3 T'  = E*_g - 3 gr_g b_g a T^4      (g < m)
 *   -sum_g g_g E'_g + (C_v + 4 sum_g g_g b_g a T^3) T'
 *                                     = C_v T + 3 sum_g g_g b_g a T^4 + S
 * with gr_g = dt c_hat kappa_P,g rho, g_g = dt c kappa_P,g rho, assembled
 * literally and solved densely.  The right-hand sides cancel when the gas is
 * much hotter than the radiation, so assembly and elimination run in
 * extended precision (64-bit significand) and the result is rounded once.
 * out: E'_0 .. E'_{m-1}, T'. */
int m1o_mg_cell(int m, const double *Es, double Cv, double T, const double *kP, double rho, double dt,
                double c_hat, double c, double a, const double *b, double S, double *out)
{
    int n = m + 1;
    long double A[(M1O_MAX_GROUPS + 1) * (M1O_MAX_GROUPS + 1)], r[M1O_MAX_GROUPS + 1], x[M1O_MAX_GROUPS + 1];
    if (m < 1 || m > M1O_MAX_GROUPS) return -1;
    for (int i = 0; i < n * n; ++i) A[i] = 0.0L;
    long double aT3 = (long double)a * T * T * T, aT4 = aT3 * T;
    r[m] = (long double)Cv * T + S;
    A[m * n + m] = Cv;
    for (int g = 0; g < m; ++g) {
        long double gr = (long double)dt * c_hat * kP[g] * rho, gg = (long double)dt * c * kP[g] * rho;
        A[g * n + g] = 1.0L + gr;
        A[g * n + m] = -4.0L * gr * b[g] * aT3;
        r[g] = Es[g] - 3.0L * gr * b[g] * aT4;
        A[m * n + g] = -gg;
        A[m * n + m] += 4.0L * gg * b[g] * aT3;
        r[m] += 3.0L * gg * b[g] * aT4;
    }
    if (gauss_solve(n, A, r, x)) return -1;
    for (int i = 0; i < n; ++i) out[i] = (double)x[i];
    return 0;
}

/* Multigroup run: st_rad[4 m] = (E_g, Fx_g, Fy_g, Fz_g) for g = 0 .. m-1,
 * gas[5] = (rho, mx, my, mz, Eg).  Each step transports every group with the
 * gray scheme (constant group opacities), then solves the coupled implicit
 * system per cell; the flux of group g is damped by 1 + dt c_hat chi_g rho,
 * the gas takes the rescaled totals (Sect. 2.7). */
int m1o_run_mg(const m1o_problem *p, int m, const double *edges, const double *kPg, const double *kRg,
               double dt, int nsteps, double *const rad[], double *const gas[5], long long cnt[M1O_NCNT])
{
    if (m < 1 || m > M1O_MAX_GROUPS) return -1;
    long N = (long)p->n[0] * p->n[1] * p->n[2];
    double *star = malloc((size_t)4 * m * N * sizeof(double));
    if (!star) return -1;
    m1o_problem pg = *p;
    pg.opac_kind = M1O_CONST;
    for (int s = 0; s < nsteps; ++s) {
        for (int g = 0; g < m; ++g) {
            pg.kP = kPg[g];
            pg.kR = kRg[g];
            pg.noise_seed = p->noise_seed + (unsigned long long)s * 4096u + (unsigned long long)g;
            const double *in[9] = {rad[4 * g], rad[4 * g + 1], rad[4 * g + 2], rad[4 * g + 3],
                                   gas[0], gas[1], gas[2], gas[3], gas[4]};
            double *out[4] = {star + (4 * g) * N, star + (4 * g + 1) * N, star + (4 * g + 2) * N,
                              star + (4 * g + 3) * N};
            if (m1o_explicit(&pg, dt, in, out, cnt)) { free(star); return -1; }
        }
        long long ffx = 0, bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : ffx, bad)
        for (long id = 0; id < N; ++id) {
            double rho = gas[0][id], mx = gas[1][id], my = gas[2][id], mz = gas[3][id], Eg = gas[4][id];
            double Cv = rho / (p->gamma - 1.0);
            double T = (Eg - 0.5 * (mx * mx + my * my + mz * mz) / rho) / Cv;
            double b[M1O_MAX_GROUPS], Es[M1O_MAX_GROUPS], x[M1O_MAX_GROUPS + 1];
            m1o_group_fractions(m, edges, T, b);
            for (int g = 0; g < m; ++g) Es[g] = star[(4 * g) * N + id];
            double S = p->irr ? p->irr[id] * dt : 0.0;
            if (m1o_mg_cell(m, Es, Cv, T, kPg, rho, dt, p->c_hat, p->c, p->a_rad, b, S, x)) { ++bad; continue; }
            double dE = 0.0, dF[3] = {0, 0, 0};
            for (int g = 0; g < m; ++g) {
                /* absorption only (Sect. 3.3): no emission in any group */
                double E1 = p->absorb_only ? Es[g] / (1.0 + dt * p->c_hat * kPg[g] * rho) : x[g];
                double damp = 1.0 + dt * p->c_hat * (kRg[g] + p->sigma) * rho;
                double F1[3], Fs[3];
                for (int q = 0; q < 3; ++q) {
                    Fs[q] = star[(4 * g + 1 + q) * N + id];
                    F1[q] = Fs[q] / damp;
                }
                double Fn = sqrt(F1[0] * F1[0] + F1[1] * F1[1] + F1[2] * F1[2]);
                if (Fn > E1) {
                    double sc = E1 / Fn;
                    F1[0] *= sc; F1[1] *= sc; F1[2] *= sc;
                    ++ffx;
                }
                dE += E1 - Es[g];
                for (int q = 0; q < 3; ++q) dF[q] += F1[q] - Fs[q];
                rad[4 * g][id] = E1;
                for (int q = 0; q < 3; ++q) rad[4 * g + 1 + q][id] = F1[q];
            }
            gas[4][id] = Eg + S - (p->c / p->c_hat) * dE;
            gas[1][id] = mx - dF[0] / p->c_hat;
            gas[2][id] = my - dF[1] / p->c_hat;
            gas[3][id] = mz - dF[2] / p->c_hat;
        }
        cnt[M1O_CNT_FFIX_IMPLICIT] += ffx;
        if (bad) { free(star); return -1; }
    }
    free(star);
    return 0;
}

/* Second-order Runge-Kutta stepping of the multigroup system, the scheme of
 * the gray m1o_run_rk2 (Sect. 2.4: the transport + source sequence is the
 * operator of every sub-step):
 *   U1 = S(T(U^n)),  U2 = S(T(U1)),  U^{n+1} = (U^n + U2) / 2
 * for every group's (E, F) and the gas (m, E_g); rho is frozen. */
int m1o_run_mg_rk2(const m1o_problem *p, int m, const double *edges, const double *kPg, const double *kRg,
                   double dt, int nsteps, double *const rad[], double *const gas[5], long long cnt[M1O_NCNT])
{
    if (m < 1 || m > M1O_MAX_GROUPS) return -1;
    long N = (long)p->n[0] * p->n[1] * p->n[2];
    int nf = 4 * m + 4;
    double *save = malloc((size_t)nf * N * sizeof(double));
    if (!save) return -1;
    double *f[4 * M1O_MAX_GROUPS + 4];
    for (int q = 0; q < 4 * m; ++q) f[q] = rad[q];
    for (int q = 0; q < 4; ++q) f[4 * m + q] = gas[1 + q];     /* mx, my, mz, Eg */
    for (int s = 0; s < nsteps; ++s) {
        for (int q = 0; q < nf; ++q) memcpy(save + (long)q * N, f[q], N * sizeof(double));
        if (m1o_run_mg(p, m, edges, kPg, kRg, dt, 2, rad, gas, cnt)) { free(save); return -1; }
        for (int q = 0; q < nf; ++q) {
#pragma omp parallel for schedule(static)
            for (long id = 0; id < N; ++id) f[q][id] = 0.5 * (save[(long)q * N + id] + f[q][id]);
        }
    }
    free(save);
    return 0;
}
