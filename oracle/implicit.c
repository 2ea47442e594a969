/*
 * implicit.c -- oracle: opacity sources and the implicit radiation-matter
 * step (Sect. 2.8).  Test infrastructure only.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include "m1_oracle.h"

/* ------------------------------------------------------------------------ */
/* opacities                                                                */
/* ------------------------------------------------------------------------ */

/* Bilinear interpolation of a [nt][nr] table of log10 kappa on a uniform
 * node grid that includes both axis ends; coordinates are clamped to it. */
static double table_bilinear(const m1o_problem *p, const float *tab, double lr, double lt)
{
    if (lr < p->tab_lr0) lr = p->tab_lr0;
    if (lr > p->tab_lr1) lr = p->tab_lr1;
    if (lt < p->tab_lt0) lt = p->tab_lt0;
    if (lt > p->tab_lt1) lt = p->tab_lt1;
    double u = (lr - p->tab_lr0) / (p->tab_lr1 - p->tab_lr0) * (p->tab_nr - 1);
    double v = (lt - p->tab_lt0) / (p->tab_lt1 - p->tab_lt0) * (p->tab_nt - 1);
    int i = (int)floor(u), j = (int)floor(v);
    if (i > p->tab_nr - 2) i = p->tab_nr - 2;
    if (j > p->tab_nt - 2) j = p->tab_nt - 2;
    double wu = u - i, wv = v - j;
    double k00 = tab[(long)j * p->tab_nr + i], k10 = tab[(long)j * p->tab_nr + i + 1];
    double k01 = tab[(long)(j + 1) * p->tab_nr + i], k11 = tab[(long)(j + 1) * p->tab_nr + i + 1];
    return (1.0 - wu) * (1.0 - wv) * k00 + wu * (1.0 - wv) * k10
         + (1.0 - wu) * wv * k01 + wu * wv * k11;
}

/* Planck and Rosseland absorption opacities at (rho, T).  Scattering sigma is
 * added separately (chi = kappa_R + sigma, Sect. 2.1). */
void m1o_opacity(const m1o_problem *p, double rho, double T, double *kP, double *kR)
{
    switch (p->opac_kind) {
    case M1O_CONST:
        *kP = p->kP; *kR = p->kR;
        return;
    case M1O_POWERLAW: {
        double k = p->pl_k0 * pow(rho / p->pl_rho0, p->pl_alpha) * pow(T / p->pl_T0, p->pl_beta);
        *kP = k; *kR = k;
        return;
    }
    case M1O_TABLE: {
        double lr = log10(rho) + p->tab_lr_off, lt = log10(T) + p->tab_lt_off;
        *kP = pow(10.0, table_bilinear(p, p->tab_kP, lr, lt));
        *kR = pow(10.0, table_bilinear(p, p->tab_kR, lr, lt));
        return;
    }
    default: {
        double lr = log10(rho) + p->tab_lr_off, lt = log10(T) + p->tab_lt_off;
        if (lr < p->tab_lr0) lr = p->tab_lr0;
        if (lr > p->tab_lr1) lr = p->tab_lr1;
        if (lt < p->tab_lt0) lt = p->tab_lt0;
        if (lt > p->tab_lt1) lt = p->tab_lt1;
        double x[2] = {2.0 * (lr - p->tab_lr0) / (p->tab_lr1 - p->tab_lr0) - 1.0,
                       2.0 * (lt - p->tab_lt0) / (p->tab_lt1 - p->tab_lt0) - 1.0};
        double y[2];
        m1o_mlp_forward(p->mlp_theta, p->mlp_bf16, 1, x, y);
        *kP = pow(10.0, y[0] * p->mlp_norm[1] + p->mlp_norm[0]);
        *kR = pow(10.0, y[1] * p->mlp_norm[3] + p->mlp_norm[2]);
        return;
    }
    }
}

void m1o_opacity_many(const m1o_problem *p, long n, const double *rho, const double *T,
                      double *kP, double *kR)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) m1o_opacity(p, rho[i], T[i], &kP[i], &kR[i]);
}

/* ------------------------------------------------------------------------ */
/* implicit source step                                                     */
/* ------------------------------------------------------------------------ */

/* Backward-Euler radiation-matter exchange of one cell (Eq. implicit_matrix):
 *
 *   [ 1 + g_r        -4 g_r a T^3     ] [E']   [ E* - 3 g_r a T^4   ]
 *   [ -g             C_v + 4 g a T^3  ] [T'] = [ C_v T + 3 g a T^4  ]
 *
 * with g_r = dt c_hat kappa_P rho, g = dt c kappa_P rho and the linearised
 * (T')^4 = 4 T' T^3 - 3 T^4.  The determinant is C_v (1 + g_r) + 4 g a T^3.
 * out[0], out[1]: E', T' in a cancellation-free arrangement of Cramer's
 * rule; out[2], out[3]: the same from the literal Cramer numerators. */
void m1o_implicit_cell(double Es, double Cv, double T, double kP, double rho, double dt,
                       double c_hat, double c, double a, double S, double out[4])
{
    double gr = dt * c_hat * kP * rho;
    double g = dt * c * kP * rho;
    double aT3 = a * T * T * T, aT4 = aT3 * T;
    double det = Cv * (1.0 + gr) + 4.0 * g * aT3;
    out[0] = (Cv * (Es + gr * aT4) + 4.0 * aT3 * (g * Es + gr * S)) / det;
    out[1] = (Cv * T * (1.0 + gr) + 3.0 * g * aT4 + g * Es + (1.0 + gr) * S) / det;
    double b0 = Es - 3.0 * gr * aT4, b1 = Cv * T + 3.0 * g * aT4 + S;
    double m00 = 1.0 + gr, m01 = -4.0 * gr * aT3, m10 = -g, m11 = Cv + 4.0 * g * aT3;
    out[2] = (b0 * m11 - m01 * b1) / det;
    out[3] = (m00 * b1 - m10 * b0) / det;
}

int m1o_implicit(const m1o_problem *p, double dt, const double *const star[4],
                 double *const st[9], long long cnt[M1O_NCNT])
{
    long N = (long)p->n[0] * p->n[1] * p->n[2];
    long long ffx = 0, mism = 0;
#pragma omp parallel for schedule(static) reduction(+ : ffx, mism)
    for (long id = 0; id < N; ++id) {
        double rho = st[4][id], mx = st[5][id], my = st[6][id], mz = st[7][id], Eg = st[8][id];
        double Cv = rho / (p->gamma - 1.0);
        double T = (Eg - 0.5 * (mx * mx + my * my + mz * mz) / rho) / Cv;
        double kP, kR;
        m1o_opacity(p, rho, T, &kP, &kR);
        double chi = kR + p->sigma;
        double Es = star[0][id];
        double Fs[3] = {star[1][id], star[2][id], star[3][id]};
        /* irradiation heating deposited in this step (Sect. 2.9: -div F_irr dt
         * in the S_1 row and in the conserved total) */
        double S = p->irr ? p->irr[id] * dt : 0.0;
        double r[4];
        m1o_implicit_cell(Es, Cv, T, kP, rho, dt, p->c_hat, p->c, p->a_rad, S, r);
        /* both algebraic forms must agree within their rounding bound */
        if (!p->absorb_only) {
            double gr = dt * p->c_hat * kP * rho, g = dt * p->c * kP * rho;
            double aT3 = p->a_rad * T * T * T, aT4 = aT3 * T;
            double det = Cv * (1.0 + gr) + 4.0 * g * aT3;
            double b0 = Es - 3.0 * gr * aT4, b1 = Cv * T + 3.0 * g * aT4 + S;
            double scale = (fabs(b0 * (Cv + 4.0 * g * aT3)) + fabs(4.0 * gr * aT3 * b1)) / det;
            if (fabs(r[0] - r[2]) > 64.0 * DBL_EPSILON * scale + DBL_MIN) ++mism;
        }
        /* absorption only (shadow test of Sect. 3.3): no emission by the gas,
         * E' = E* / (1 + gamma_abs,red) */
        double E1 = p->absorb_only ? Es / (1.0 + dt * p->c_hat * kP * rho) : r[0];
        double damp = 1.0 + dt * p->c_hat * chi * rho;     /* Eq. source_discrete2 */
        double F1[3] = {Fs[0] / damp, Fs[1] / damp, Fs[2] / damp};
        double Fn = sqrt(F1[0] * F1[0] + F1[1] * F1[1] + F1[2] * F1[2]);
        if (Fn > E1) {
            double s = E1 / Fn;
            F1[0] *= s; F1[1] *= s; F1[2] *= s;
            ++ffx;
        }
        /* gas from the rescaled conservation laws E + (c/c_hat) E_r and
         * rho v + F_r / c_hat (Sect. 2.7) */
        st[8][id] = Eg + S - (p->c / p->c_hat) * (E1 - Es);
        st[5][id] = mx - (F1[0] - Fs[0]) / p->c_hat;
        st[6][id] = my - (F1[1] - Fs[1]) / p->c_hat;
        st[7][id] = mz - (F1[2] - Fs[2]) / p->c_hat;
        st[0][id] = E1;
        st[1][id] = F1[0]; st[2][id] = F1[1]; st[3][id] = F1[2];
    }
    cnt[M1O_CNT_FFIX_IMPLICIT] += ffx;
    cnt[M1O_CNT_FORM_MISMATCH] += mism;
    return 0;
}
