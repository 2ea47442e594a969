/*
 * closure.c -- oracle: M1 closure, signal speeds, physical fluxes, HLL,
 * van Leer slope and the f-preserving face fix.  Test infrastructure only.
 *
 * Notation: the radiation flux F carries the 1/c factor of the paper's
 * definition (Sect. 2.1), so the reduced flux f = |F|/E lies in [0, 1] and
 * speeds below are in units of the reduced speed of light c_hat.
 */
#include <math.h>
#include "m1_oracle.h"

/* Levermore Eddington factor xi(f) (Sect. 2.1, closure equations). */
double m1o_xi(double f)
{
    double s = sqrt(4.0 - 3.0 * f * f);
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * s);
}

/* Reduced flux f = min(|F|/E, 1) and direction n = F/|F| (n = 0 when F = 0). */
static void reduced_flux(double E, const double F[3], double *f, double n[3])
{
    double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    if (Fn > 0.0) {
        n[0] = F[0] / Fn; n[1] = F[1] / Fn; n[2] = F[2] / Fn;
    } else {
        n[0] = n[1] = n[2] = 0.0;
    }
    *f = Fn / E;
    if (*f > 1.0) *f = 1.0;
}

/* Eddington tensor D^{ij} = (1-xi)/2 delta^{ij} + (3 xi - 1)/2 n^i n^j
 * (Sect. 2.1); the pressure tensor is P = D E. */
void m1o_eddington(double E, double Fx, double Fy, double Fz, double *f, double *xi, double D[9])
{
    double F[3] = {Fx, Fy, Fz}, n[3];
    reduced_flux(E, F, f, n);
    *xi = m1o_xi(*f);
    double iso = 0.5 * (1.0 - *xi), aniso = 0.5 * (3.0 * *xi - 1.0);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            D[3 * a + b] = (a == b ? iso : 0.0) + aniso * n[a] * n[b];
}

/* Extreme eigenvalues lambda_{1,3} = (f cos(theta) -+ zeta) / sqrt(4 - 3 f^2)
 * of the M1 system along direction d (Sect. 2.6); cos(theta) = n_d. */
void m1o_speeds(double E, double Fx, double Fy, double Fz, int d, double *lm, double *lp)
{
    double F[3] = {Fx, Fy, Fz}, n[3], f;
    reduced_flux(E, F, &f, n);
    double mu = n[d];
    double s = sqrt(4.0 - 3.0 * f * f);
    double z2 = (2.0 / 3.0) * (4.0 - 3.0 * f * f - s) + 2.0 * mu * mu * (2.0 - f * f - s);
    if (z2 < 0.0) z2 = 0.0;
    double zeta = sqrt(z2);
    double a = (f * mu - zeta) / s, b = (f * mu + zeta) / s;
    *lm = a < b ? a : b;
    *lp = a < b ? b : a;
}

/* Physical flux of (E, F) through a face normal to d, divided by c_hat:
 * (F_d, P_{xd}, P_{yd}, P_{zd}) with P = D E (Eqs. rad1, rad2). */
void m1o_flux(double E, double Fx, double Fy, double Fz, int d, double phi[4])
{
    double f, xi, D[9];
    double F[3] = {Fx, Fy, Fz};
    m1o_eddington(E, Fx, Fy, Fz, &f, &xi, D);
    phi[0] = F[d];
    for (int a = 0; a < 3; ++a) phi[1 + a] = E * D[3 * a + d];
}

/* HLL flux (Sect. 2.5) with the Sect. 2.6 signal speeds and the optical-depth
 * limiter: lambda_L = min of the left-going speeds of both states, lambda_R =
 * max of the right-going ones, then clamped to -+4/(3 tau) when tau > 0.
 * Returns c_hat * Phi*. */
void m1o_hll(const double UL[4], const double UR[4], int d, double tau, double c_hat,
             double out[4], double *SLo, double *SRo)
{
    double lmL, lpL, lmR, lpR, phiL[4], phiR[4];
    m1o_speeds(UL[0], UL[1], UL[2], UL[3], d, &lmL, &lpL);
    m1o_speeds(UR[0], UR[1], UR[2], UR[3], d, &lmR, &lpR);
    m1o_flux(UL[0], UL[1], UL[2], UL[3], d, phiL);
    m1o_flux(UR[0], UR[1], UR[2], UR[3], d, phiR);
    double lamL = lmL < lmR ? lmL : lmR;
    double lamR = lpL > lpR ? lpL : lpR;
    if (tau > 0.0) {
        double lim = 4.0 / (3.0 * tau);
        if (lamL < -lim) lamL = -lim;
        if (lamR > lim) lamR = lim;
    }
    double SL = lamL < 0.0 ? lamL : 0.0;
    double SR = lamR > 0.0 ? lamR : 0.0;
    for (int q = 0; q < 4; ++q) {
        if (SR > SL)
            out[q] = c_hat * (SR * phiL[q] - SL * phiR[q] + SL * SR * (UR[q] - UL[q])) / (SR - SL);
        else
            out[q] = c_hat * 0.5 * (phiL[q] + phiR[q]);
    }
    if (SLo) *SLo = SL;
    if (SRo) *SRo = SR;
}

/* van Leer limited slope: harmonic mean of the one-sided divided differences
 * when they share a sign, zero otherwise (PLM, Sect. 2.5). */
double m1o_vanleer(double dl, double dr)
{
    if (dl * dr > 0.0) return 2.0 * dl * dr / (dl + dr);
    return 0.0;
}

/* LimO3, the compact third-order limited reconstruction that Sect. 2.5
 * names (Cada and Torrilhon 2009, "Compact third-order limiter functions for
 * finite volume methods", J. Comput. Phys. 228, 4118).  On a uniform grid the
 * face value of cell i towards its neighbour on the face side is
 *   u_i + phi(theta) (u_near - u_i) / 2,   theta = (u_i - u_far) / (u_near - u_i),
 * with the third-order reconstruction phi3(theta) = (2 + theta) / 3 limited as
 *   phi = max(0, min(phi3, max(-theta/2, min(2 theta, phi3, 3/2)))).
 * In slope form, as the PLM slopes: dfar and dnear are the divided
 * differences on the far side and on the face side of the cell; the
 * returned slope phi(dfar / dnear) dnear (0 when dnear = 0) times the
 * signed centre-to-face distance gives the face value. */
double m1o_limo3(double dfar, double dnear)
{
    if (dnear == 0.0) return 0.0;
    double th = dfar / dnear;
    double p3 = (2.0 + th) / 3.0;
    double inner = fmin(fmin(2.0 * th, p3), 1.5);
    double phi = fmax(0.0, fmin(p3, fmax(-0.5 * th, inner)));
    return phi * dnear;
}

/* f-preserving face fix (Eq. f_reconstruct): keep the reconstructed face flux
 * only if the face reduced flux is <= 1 and strictly larger than the donor
 * cell's; otherwise scale the cell-centred flux by E_face / E_cell.  A face
 * energy <= 0 (not covered by the paper) falls back to the cell state.
 * Returns 0 = kept, 1 = rescaled, 2 = flat fallback. */
int m1o_ffix(double *Ef, double Ff[3], double Ec, const double Fc[3])
{
    if (*Ef > 0.0) {
        double ff = sqrt(Ff[0] * Ff[0] + Ff[1] * Ff[1] + Ff[2] * Ff[2]) / *Ef;
        double fc = sqrt(Fc[0] * Fc[0] + Fc[1] * Fc[1] + Fc[2] * Fc[2]) / Ec;
        if (ff <= 1.0 && ff > fc) return 0;
        for (int a = 0; a < 3; ++a) Ff[a] = Fc[a] * (*Ef / Ec);
        return 1;
    }
    *Ef = Ec;
    for (int a = 0; a < 3; ++a) Ff[a] = Fc[a];
    return 2;
}

/* Face treatments compared in the paper (Sect. 2.5 and the beam test of
 * Sect. 3.2).  PLUTO: flat state (E_c, F_c) whenever |R(F)| > R(E).  Clip:
 * F_f = R(F) R(E) / |R(F)| whenever |R(F)| > R(E).  Both keep the face state
 * otherwise; a face energy <= 0 falls back to the flat state.  The default
 * is the f-preserving fix (m1o_ffix).  Returns 0 = kept, 1 = changed,
 * 2 = flat. */
int m1o_face_fix(int recon, double *Ef, double Ff[3], double Ec, const double Fc[3])
{
    if (recon == M1O_RECON_FPRESERVE) return m1o_ffix(Ef, Ff, Ec, Fc);
    double Fn = sqrt(Ff[0] * Ff[0] + Ff[1] * Ff[1] + Ff[2] * Ff[2]);
    if (*Ef > 0.0 && Fn <= *Ef) return 0;
    if (recon == M1O_RECON_CLIP && *Ef > 0.0) {
        for (int a = 0; a < 3; ++a) Ff[a] = Ff[a] * (*Ef / Fn);
        return 1;
    }
    *Ef = Ec;
    for (int a = 0; a < 3; ++a) Ff[a] = Fc[a];
    return 2;
}

/* Lax-Friedrichs-Rusanov flux (Sect. 2.5): the average flux minus the jump
 * times the largest signal speed magnitude a = max(|lambda_L|, |lambda_R|),
 * with the speeds of m1o_hll (including the optical-depth limiter). */
void m1o_lf(const double UL[4], const double UR[4], int d, double tau, double c_hat, double out[4])
{
    double lmL, lpL, lmR, lpR, phiL[4], phiR[4];
    m1o_speeds(UL[0], UL[1], UL[2], UL[3], d, &lmL, &lpL);
    m1o_speeds(UR[0], UR[1], UR[2], UR[3], d, &lmR, &lpR);
    m1o_flux(UL[0], UL[1], UL[2], UL[3], d, phiL);
    m1o_flux(UR[0], UR[1], UR[2], UR[3], d, phiR);
    double lamL = lmL < lmR ? lmL : lmR;
    double lamR = lpL > lpR ? lpL : lpR;
    if (tau > 0.0) {
        double lim = 4.0 / (3.0 * tau);
        if (lamL < -lim) lamL = -lim;
        if (lamR > lim) lamR = lim;
    }
    double a = fabs(lamL) > fabs(lamR) ? fabs(lamL) : fabs(lamR);
    for (int q = 0; q < 4; ++q)
        out[q] = c_hat * (0.5 * (phiL[q] + phiR[q]) - 0.5 * a * (UR[q] - UL[q]));
}

