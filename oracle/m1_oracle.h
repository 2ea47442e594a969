/*
 * m1_oracle.h -- slow, plain FP64 CPU oracle of the gray M1 radiation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the HIP path.
 *
 * It computes, in double precision and in the order the method states it,
 * one explicit transport step (Sect. 2.5 reconstruction + f-preserving face
 * fix, Sect. 2.6 signal speeds + optical-depth limiter, HLL fluxes,
 * conservative update in Cartesian / cylindrical / spherical coordinates)
 * and one implicit radiation-matter step (Sect. 2.8, Eq. implicit_matrix),
 * plus the opacity sources (constant, power law, bilinear table, MLP).
 *
 * Array layout: cell (i, j, k) along (d0, d1, d2) lives at ((k*n1)+j)*n0+i.
 * F components are in the local orthonormal basis of the grid.
 *
 * Parity unpinned: the optical depth of a curvilinear cell in the signal-
 * speed limiter, tau = rho chi max_d h_d with h_d the cell's metric extent
 * (cell_tau in transport.c).  The method gives tau per cell without saying
 * which length a cylindrical or spherical cell takes; the extents are a
 * reading, and no value the paper fixes checks them (the same extents in
 * the time-step rule are pinned by hand-worked values).
 */
#ifndef M1_ORACLE_H
#define M1_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { M1O_CARTESIAN = 0, M1O_CYLINDRICAL = 1, M1O_SPHERICAL = 2 };
/* boundaries: periodic wrap, outflow (zero-gradient copy), reflective
 * (mirror image with the normal flux component reversed), fixed (a given
 * ghost state, e.g. an injected beam) */
enum { M1O_PERIODIC = 0, M1O_OUTFLOW = 1, M1O_REFLECT = 2, M1O_FIXED = 3 };
enum { M1O_CONST = 0, M1O_POWERLAW = 1, M1O_TABLE = 2, M1O_MLP = 3 };
/* face treatment after reconstruction (Sect. 2.5, 3.2) and Riemann solver */
enum { M1O_RECON_FPRESERVE = 0, M1O_RECON_PLUTO = 1, M1O_RECON_CLIP = 2 };
enum { M1O_HLL = 0, M1O_LF = 1 };
/* reconstruction: PLM with the van Leer slope, or LimO3 (Sect. 2.5) */
enum { M1O_PLM = 0, M1O_LIMO3 = 1 };

/* counters returned by the step routines */
enum { M1O_CNT_EFLOOR = 0, M1O_CNT_FFIX_TRANSPORT = 1, M1O_CNT_FFIX_IMPLICIT = 2,
       M1O_CNT_FORM_MISMATCH = 3, M1O_NCNT = 4 };

typedef struct {
    int geometry, ndim;
    int n[3];
    const double *faces[3];
    int bc[3][2];
    double c_hat, c, a_rad, gamma, e_floor;
    int opac_kind;
    double kP, kR, sigma;
    double pl_k0, pl_rho0, pl_alpha, pl_T0, pl_beta;
    int tab_nr, tab_nt;
    double tab_lr0, tab_lr1, tab_lt0, tab_lt1, tab_lr_off, tab_lt_off;
    const float *tab_kP, *tab_kR;
    const double *mlp_theta;  /* flat parameters, order W1 b1 W2 b2 W3 b3 Ws */
    double mlp_norm[4];       /* mean_P, std_P, mean_R, std_R of log10 kappa */
    int mlp_bf16;             /* 1: round layer-2 operands like the GPU */
    int recon;                /* M1O_RECON_* */
    int riemann;              /* M1O_HLL or M1O_LF */
    double bc_state[3][2][4]; /* ghost (E, Fx, Fy, Fz) of M1O_FIXED sides */
    const double *irr;        /* per-cell irradiation heating -div F_irr, or NULL */
    int absorb_only;          /* 1: radiation is absorbed, never emitted */
    int limiter;              /* M1O_PLM or M1O_LIMO3 */
    /* test use only: random perturbation of every reconstructed face value
     * by face_noise x (|u_cell| + |slope x offset|) x w, w uniform in
     * [-1, 1) from a counter-based hash of noise_seed and the face (0 = off);
     * models the rounding of face values computed in lower precision */
    double face_noise;
    unsigned long long noise_seed;
} m1o_problem;

/* --- closure, speeds, fluxes (Sect. 2.1, 2.5, 2.6) ------------------------ */
double m1o_xi(double f);
void m1o_eddington(double E, double Fx, double Fy, double Fz, double *f, double *xi, double D[9]);
void m1o_speeds(double E, double Fx, double Fy, double Fz, int d, double *lm, double *lp);
void m1o_flux(double E, double Fx, double Fy, double Fz, int d, double phi[4]);
void m1o_hll(const double UL[4], const double UR[4], int d, double tau, double c_hat,
             double out[4], double *SL, double *SR);
double m1o_vanleer(double dl, double dr);
double m1o_limo3(double dfar, double dnear);
int m1o_ffix(double *Ef, double Ff[3], double Ec, const double Fc[3]);
int m1o_face_fix(int recon, double *Ef, double Ff[3], double Ec, const double Fc[3]);
void m1o_lf(const double UL[4], const double UR[4], int d, double tau, double c_hat, double out[4]);

/* --- grid ----------------------------------------------------------------- */
void m1o_cell_geometry(const m1o_problem *p, int i, int j, int k, double out[12]);
double m1o_max_dt(const m1o_problem *p, double cfl);

/* --- steps ---------------------------------------------------------------- */
int m1o_explicit(const m1o_problem *p, double dt, const double *const in[9],
                 double *const out[4], long long cnt[M1O_NCNT]);
int m1o_implicit(const m1o_problem *p, double dt, const double *const star[4],
                 double *const st[9], long long cnt[M1O_NCNT]);
int m1o_run(const m1o_problem *p, double dt, int nsteps, double *const st[9],
            long long cnt[M1O_NCNT]);
int m1o_run_rk2(const m1o_problem *p, double dt, int nsteps, double *const st[9],
                long long cnt[M1O_NCNT]);

/* --- multigroup (one gray fluid per group, (m+1)^2 implicit system) ------- */
#define M1O_MAX_GROUPS 32
double m1o_planck_cdf(double x);
void m1o_group_fractions(int m, const double *edges, double T, double *b);
int m1o_mg_cell(int m, const double *Es, double Cv, double T, const double *kP, double rho, double dt,
                double c_hat, double c, double a, const double *b, double S, double *out);
int m1o_run_mg(const m1o_problem *p, int m, const double *edges, const double *kPg, const double *kRg,
               double dt, int nsteps, double *const rad[], double *const gas[5], long long cnt[M1O_NCNT]);
int m1o_run_mg_rk2(const m1o_problem *p, int m, const double *edges, const double *kPg, const double *kRg,
                   double dt, int nsteps, double *const rad[], double *const gas[5], long long cnt[M1O_NCNT]);

/* --- single-cell implicit solve (both algebraic forms) -------------------- */
void m1o_implicit_cell(double Es, double Cv, double T, double kP, double rho, double dt,
                       double c_hat, double c, double a, double S, double out[4]);

/* --- opacity -------------------------------------------------------------- */
void m1o_opacity(const m1o_problem *p, double rho, double T, double *kP, double *kR);
void m1o_opacity_many(const m1o_problem *p, long n, const double *rho, const double *T,
                      double *kP, double *kR);

/* --- MLP surrogate (2 -> 64 -> 64 -> 2, tanh, linear shortcut) ------------ */
int m1o_mlp_nparam(void);
void m1o_mlp_forward(const double *theta, int bf16, long n, const double *x, double *y);
double m1o_mlp_loss_grad(const double *theta, int bf16, long n, const double *x,
                         const double *t, double *grad);
void m1o_adam(long np, double *theta, const double *g, double *m, double *v, long step,
              double lr, double b1, double b2, double eps);
double m1o_bf16_round(double x);

#ifdef __cplusplus
}
#endif
#endif
