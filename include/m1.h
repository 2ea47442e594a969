/*
 * m1.h -- C ABI of the MI355X (gfx950) gray M1 radiation step library.
 *
 * The library advances the radiation moments (E_r, F_r) of the gray M1
 * scheme coupled to a static gas: one step is
 *
 *   m1_step_explicit   transport of (E, F): PLM van Leer reconstruction with
 *                      the f-preserving face fix, Levermore closure, HLL
 *                      fluxes with the optical-depth speed limiter, at the
 *                      reduced speed of light c_hat, conservative update in
 *                      Cartesian, cylindrical or spherical coordinates
 *                      (paper Sect. 2.4-2.7);
 *   m1_step_implicit   per-cell backward-Euler radiation-matter exchange,
 *                      the 2x2 system of Eq. implicit_matrix, flux damping of
 *                      Eq. source_discrete2 and the gas update from the
 *                      rescaled conservation laws (Sect. 2.7, 2.8).
 *
 * Conventions
 *   - F is the paper's radiation flux that carries the 1/c factor
 *     (Sect. 2.1), so the reduced flux f = |F|/E lies in [0, 1].
 *   - Cells are stored as contiguous structure-of-arrays, one array per
 *     field, index ((k*n1)+j)*n0+i with i along d = 0 (x / R / r), j along
 *     d = 1 (y / phi / theta), k along d = 2 (z / z / phi).  Vector
 *     components are in the local orthonormal basis of the grid.
 *   - Device pointers are HIP device memory owned by the caller, 256-byte
 *     aligned.  Radiation arrays (E, Fx, Fy, Fz) are double (M1_P64) or
 *     float (M1_F32); gas arrays (rho, mx, my, mz, Eg) are always double.
 *   - All work is enqueued asynchronously on the stream given by
 *     m1_set_stream (default: the null stream); no call synchronises except
 *     m1_sync, m1_diagnostics, m1_mlp_train and m1_mlp_get.
 *   - Every function returns an m1_status; a negative value is an error
 *     whose text m1_last_error() returns.  No call allocates device memory
 *     after m1_bind_state except m1_set_opacity_table, m1_set_opacity_mlp
 *     and m1_mlp_train (which own their buffers until m1_destroy).
 */
#ifndef M1_H
#define M1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    M1_OK = 0,
    M1_EINVAL = -1,   /* bad argument: dimensions, pointers, ranges */
    M1_ENOMEM = -2,   /* device or host allocation failed */
    M1_EDEVICE = -3,  /* HIP runtime error (launch or deferred kernel error) */
    M1_ESTATE = -4,   /* call out of order (e.g. implicit before explicit) */
    M1_ENOTSUP = -5   /* valid request the library does not implement */
} m1_status;

typedef enum { M1_CARTESIAN = 0, M1_CYLINDRICAL = 1, M1_SPHERICAL = 2 } m1_geometry;
/* boundaries: periodic wrap (paired), outflow (zero-gradient copy of the
 * edge cell), reflective (mirror image of the interior with the flux
 * component normal to the boundary reversed: the wall of the shadow test,
 * Sect. 3.3) and fixed (a ghost state given by m1_set_boundary_state, e.g.
 * a beam injected through the boundary, Sect. 3.3) */
typedef enum { M1_BC_PERIODIC = 0, M1_BC_OUTFLOW = 1, M1_BC_REFLECT = 2, M1_BC_FIXED = 3 } m1_bc;
typedef enum { M1_P64 = 0, M1_F32 = 1 } m1_precision;
typedef enum { M1_OPAC_CONSTANT = 0, M1_OPAC_POWERLAW = 1 } m1_opacity_model;
/* face treatment after reconstruction (Sect. 2.5; compared in Sect. 3.2) */
typedef enum { M1_RECON_FPRESERVE = 0, M1_RECON_PLUTO = 1, M1_RECON_CLIP = 2 } m1_recon;
typedef enum { M1_RIEMANN_HLL = 0, M1_RIEMANN_LF = 1 } m1_riemann;
/* reconstruction of the face states (Sect. 2.5): piecewise linear with the
 * van Leer slope (PLM), or the compact third-order LimO3 of Cada and
 * Torrilhon (2009) */
typedef enum { M1_LIMITER_PLM = 0, M1_LIMITER_LIMO3 = 1 } m1_limiter;

/* Grid: ndim active directions (1..3); n[d] interior cells (n[d] = 1 for an
 * inactive direction); faces[d] = n[d]+1 strictly increasing coordinates
 * (host memory, copied).  Spherical: r >= 0 and 0 <= theta <= pi;
 * cylindrical: R >= 0.  bc[d][0|1] = lower/upper boundary of direction d. */
typedef struct {
    int ndim;
    int n[3];
    const double *faces[3];
    int bc[3][2];
} m1_grid;

/* Physical and numerical parameters (m1_params_default fills them):
 * c       true speed of light (default: c_hat), enters the gas energy
 *         exchange (Eq. internal) and the rescaled energy total (Sect. 2.7)
 * a_rad   radiation constant a_R (default 1)
 * gamma   adiabatic index; C_v = rho / (gamma - 1) per volume (default 5/3)
 * precision  M1_P64 (all FP64) or M1_F32 (FP32 radiation storage and
 *         transport, FP64 implicit solve and gas).  The closure works with
 *         squared norms, so E and |F| should stay within about 1e-19..1e19
 *         in M1_F32 (1e-154..1e154 in M1_P64); a flux whose squared norm is
 *         below the normal range counts as zero
 * e_floor lower bound enforced on E after transport (default 1e-30)
 * recon   face treatment: M1_RECON_FPRESERVE (default, Eq. f_reconstruct),
 *         M1_RECON_PLUTO (flat face state whenever |R(F)| > R(E)) or
 *         M1_RECON_CLIP (F_f = R(F) R(E)/|R(F)| whenever |R(F)| > R(E))
 * riemann M1_RIEMANN_HLL (default) or M1_RIEMANN_LF (Lax-Friedrichs-Rusanov
 *         with the largest limited signal speed)
 * absorb_only  0 (default): the full radiation-matter system of
 *         Eq. implicit_matrix; 1: absorption without emission,
 *         E' = E* / (1 + dt c_hat kappa_P rho) (shadow test, Sect. 3.3), the
 *         absorbed energy going to the gas
 * second_order  0 (default) or 1: m1_bind_state also allocates the buffer
 *         of m1_step_rk2 (the first-stage state, 4 m + 4 fields), so that no
 *         step call allocates
 * limiter M1_LIMITER_PLM (default) or M1_LIMITER_LIMO3: phi(theta) of
 *         theta = (far-side difference) / (face-side difference),
 *         phi = max(0, min(p3, max(-theta/2, min(2 theta, p3, 3/2)))),
 *         p3 = (2 + theta)/3, the face value u + phi (face-side divided
 *         difference) (x_face - x_cell); each face of a cell has its own
 *         slope.  The face treatment (recon) applies to either.
 * stream_reads  how the implicit step reads its inputs (each once per
 *         step): M1_STREAM_AUTO (default) with a nontemporal hint, which
 *         streams them past the caches and leaves the last-level cache to
 *         the step's outputs, when a step moves at least 384 MiB, else as
 *         plain loads; M1_STREAM_ON always; M1_STREAM_OFF never.  Results are
 *         bit-identical; only the speed differs (execution tuning, no
 *         passage of the paper). */
typedef enum { M1_STREAM_AUTO = 0, M1_STREAM_ON = 1, M1_STREAM_OFF = 2 } m1_stream_reads;
typedef struct {
    double c;
    double a_rad;
    double gamma;
    int precision;
    double e_floor;
    int recon;
    int riemann;
    int absorb_only;
    int second_order;
    int limiter;
    int stream_reads;
} m1_params;

/* Caller-owned device state bound to a context (see conventions). */
typedef struct {
    void *E, *Fx, *Fy, *Fz;
    const double *rho;
    double *mx, *my, *mz, *Eg;
} m1_fields;

/* Conserved totals and extrema of the bound state (m1_diagnostics):
 * rad_energy = sum V E;  total_energy = sum V (E_g + (c/c_hat) E)
 * momentum[3] = sum V (m + F / c_hat) (meaningful for Cartesian grids)
 * min_E, max_f over cells; counters of fix-ups since m1_bind_state:
 * [0] E floor after transport, [1] f <= 1 rescale after transport,
 * [2] f <= 1 rescale after the implicit step. */
typedef struct {
    double rad_energy;
    double total_energy;
    double momentum[3];
    double min_E;
    double max_f;
    long long counters[4];
} m1_diag;

/* MLP opacity surrogate: 2 -> 64 -> 64 -> 2 tanh network with a linear
 * 2 -> 2 shortcut, inputs x = 2 (l - l_min)/(l_max - l_min) - 1 of the table
 * coordinates (log10 rho + off_rho, log10 T + off_T) clamped to the bound
 * table's axes, outputs y with log10 kappa_{P,R} = y * std + mean.
 * theta: 4486 float32 parameters in the order W1[64][2] b1[64] W2[64][64]
 * b2[64] W3[2][64] b3[2] Ws[2][2] (host memory, copied). */
#define M1_MLP_NPARAM 4486
typedef struct {
    const float *theta;
    double norm[4]; /* mean_P, std_P, mean_R, std_R */
} m1_mlp;

/* Training of the surrogate on the GPU by the library's own kernels against
 * bilinear lookups of the bound table.  samples: device float32 [n][2] table
 * coordinates (log10 rho + off, log10 T + off), the first n_train for
 * training, the remaining n_eval held out.  theta_init: host float32
 * initial parameters (M1_MLP_NPARAM). */
typedef struct {
    const float *samples;
    long n_train;
    long n_eval;
    const float *theta_init;
    int batch;        /* samples per Adam step (multiple of 64, <= 4096) */
    long steps;       /* Adam steps */
    double lr;        /* peak learning rate */
    double lr_final;  /* learning rate at the last step (cosine decay) */
    double beta1, beta2, eps;
    int keep_init;    /* 0: the linear shortcut (Ws, b3) of theta_init is
                         replaced by the least-squares plane through the
                         table (default); 1: training starts from theta_init
                         unchanged (resuming a trained network) */
} m1_train_cfg;

typedef struct {
    double final_loss;      /* mean over the last 100 steps */
    double max_rel_err_P;   /* max |kappa_mlp / kappa_table - 1| on held-out */
    double max_rel_err_R;
    double seconds;         /* device time of the training loop */
} m1_train_report;

typedef struct m1_ctx m1_ctx;

/* Fill *p with defaults for reduced speed of light c_hat: c = c_hat (the
 * reduced-c factor of Sect. 2.7 off), a_rad = 1, gamma = 5/3, FP64, the
 * f-preserving face fix with HLL (Sect. 2.5), PLM, Euler steps.  Host only. */
m1_status m1_params_default(double c_hat, m1_params *p);

/* Create a context for grid g (copied) in geometry geom with reduced speed
 * of light c_hat (> 0; Sect. 2.7).  The finite-volume solver of Sect. 2.5
 * runs on Cartesian, cylindrical and spherical grids (the Sect. 3.4 pulses
 * use Cartesian and spherical coordinates, Sect. 3.7 a spherical grid).  p may be NULL (defaults).  Uploads the separable
 * metric arrays of the grid.  Errors: M1_EINVAL (ndim outside 1..3,
 * n[d] < 1, n[d] != 1 for d >= ndim, more than 2^31 - 2^16 cells,
 * non-increasing faces, negative radius, theta outside [0, pi],
 * c_hat <= 0, unknown enum), M1_ENOMEM, M1_EDEVICE. */
m1_status m1_create(const m1_grid *g, m1_geometry geom, double c_hat, const m1_params *p,
                    m1_ctx **out);

/* Free the context and every library-owned buffer; never the caller's.
 * (Resource management: no passage of the paper.) */
m1_status m1_destroy(m1_ctx *ctx);

/* Enqueue all further work on hipStream_t `stream` (NULL: null stream).
 * (Execution plumbing: no passage of the paper.) */
m1_status m1_set_stream(m1_ctx *ctx, void *stream);

/* Bind the state of Sect. 2.1 and 2.8 (radiation E_r, F_r; gas density,
 * momentum and total energy) as caller-owned device arrays (must outlive
 * the binding) and allocate
 * the library's scratch (transported E*, F*, opacity caches, reduction
 * buffers).  Evaluates the opacity cache from the current gas state.
 * M1_EINVAL on a NULL or non-256-byte-aligned pointer.  M1_ENOMEM when an
 * allocation fails: the new buffers are allocated before the old ones are
 * released, so a failed (re)binding leaves any previous binding, its
 * arrays and its buffers, in force and usable. */
m1_status m1_bind_state(m1_ctx *ctx, const m1_fields *f);

/* Opacity model (Sect. 2.1 source terms; chi = kappa_R + sigma):
 * M1_OPAC_CONSTANT  params = {kappa_P, kappa_R, sigma}
 * M1_OPAC_POWERLAW  params = {k0, rho0, alpha, T0, beta, sigma}:
 *                   kappa_P = kappa_R = k0 (rho/rho0)^alpha (T/T0)^beta
 * Re-evaluates the opacity cache when a state is bound. */
m1_status m1_set_opacity_model(m1_ctx *ctx, int kind, const double *params);

/* Tabulated Planck and Rosseland mean opacities (kappa_P, kappa_R of
 * Sect. 2.1; tables computed beforehand and interpolated, as in Sect. 3.7).
 * Bilinear table of log10 kappa (Planck and Rosseland) on nr x nt nodes that
 * include both axis ends: node (i, j) at (lr_min + i h_r, lt_min + j h_t),
 * host float32 arrays [nt][nr] (copied).  Looked up at
 * (log10 rho + lr_off, log10 T + lt_off), clamped to the axes.  nr, nt >= 2.
 * The library keeps the tables and, for the lookup, one 32-byte record per
 * table cell with its four node values of both (device memory of about
 * 40 nr nt bytes, and as much host memory while the call runs).
 * On M1_ENOMEM or an upload error the previous opacity source is kept. */
m1_status m1_set_opacity_table(m1_ctx *ctx, int nr, int nt, double lr_min, double lr_max,
                               double lt_min, double lt_max, double lr_off, double lt_off,
                               const float *log10_kP, const float *log10_kR, double sigma);

/* Use the MLP surrogate in place of the table (the table must be set: its
 * axes and offsets define the network's input scaling).  The surrogate is
 * not part of the paper's method: it stands in for the tabulated mean
 * opacities kappa_P, kappa_R (Sect. 2.1, Sect. 3.7), and the table it was
 * trained on stays the reference for its error. */
m1_status m1_set_opacity_mlp(m1_ctx *ctx, const m1_mlp *w);

/* Train the surrogate on the GPU (see m1_train_cfg) against the bound
 * table (Sect. 3.7 tabulated opacities; the surrogate itself is an
 * addition, see m1_set_opacity_mlp); on success the trained network
 * becomes the context's opacity source.  Synchronous. */
m1_status m1_mlp_train(m1_ctx *ctx, const m1_train_cfg *cfg, m1_train_report *rep);

/* Copy the current network parameters to host theta (M1_MLP_NPARAM floats)
 * and norm[4].  Synchronous.  (Surrogate bookkeeping, see
 * m1_set_opacity_mlp.) */
m1_status m1_mlp_get(m1_ctx *ctx, float *theta, double *norm);

/* Loss and gradient of the surrogate (parameters theta, host float32
 * [M1_MLP_NPARAM]) on n device samples (float32 [n][2] table coordinates, n
 * a positive multiple of 64) against the bound table, computed by the
 * training kernels: grad (host, M1_MLP_NPARAM floats), *loss.  theta
 * becomes the context's network; the normalisation is the one set by
 * m1_set_opacity_mlp or m1_mlp_train.  Synchronous.  (The surrogate's
 * training gradient, checked against the oracle; see m1_set_opacity_mlp.) */
m1_status m1_mlp_gradient(m1_ctx *ctx, const float *samples, long n, const float *theta, float *grad,
                          double *loss);

/* Evaluate the active opacity source on n device points: rho, T (double) ->
 * kP, kR (double), the Planck and Rosseland means of Sect. 2.1.  n = 0 is
 * a no-op.  Asynchronous. */
m1_status m1_opacity_eval(m1_ctx *ctx, long n, const double *rho, const double *T, double *kP,
                          double *kR);

/* The time-step update that closes the step list of Sect. 2.4, at a
 * Courant number such as the 0.4 of Sect. 3.1.
 * Largest stable step for Courant number cfl: cfl / max_cells(c_hat
 * sum_{d < ndim} 1/h_d) with h = (dr, r dtheta, r sin(theta) dphi) in
 * spherical and (dR, R dphi, dz) in cylindrical grids (host computation). */
m1_status m1_max_dt(const m1_ctx *ctx, double cfl, double *dt);

/* Items 1-7 of the Euler step list of Sect. 2.4: boundary values,
 * reconstruction (Sect. 2.5) with the f <= 1 face treatment of
 * Eq. f_reconstruct, wave speeds with the optical-depth limiter (Sect. 2.6),
 * Riemann fluxes (Sect. 2.5) and the flux divergence, at c_hat (Sect. 2.7).
 * Explicit transport step of length dt (> 0) from the bound (E, F) into the
 * library's transported state (E*, F*).  Asynchronous.  M1_ESTATE if no
 * state is bound. */
m1_status m1_step_explicit(m1_ctx *ctx, double dt);

/* Item 8 of the Sect. 2.4 list: the local source terms, solved implicitly
 * as Eqs. source_discrete1, source_discrete2 and implicit_matrix of
 * Sect. 2.8, with the gas update from the rescaled totals of Sect. 2.7.
 * Implicit source step of length dt from (E*, F*) and the gas: writes E, F,
 * m, E_g of the bound arrays and refreshes the opacity cache at the new
 * temperature.  Asynchronous.  M1_ESTATE unless the previous step call was
 * m1_step_explicit. */
m1_status m1_step_implicit(m1_ctx *ctx, double dt);

/* Multigroup M1 (Sect. 2.3, 2.8): m frequency groups, each transported as
 * an independent gray M1 fluid, coupled to the gas by the (m+1)^2 implicit
 * system in which group g emits the Planck fraction b_g(T^n) of a T^4
 * (fraction of int B_nu over its band at the start-of-step temperature).
 * edges: m-1 increasing interior group boundaries x_g = h nu_g / k, in the
 * temperature unit (> 0; NULL for m = 1); kP, kR: m constant Planck and
 * Rosseland opacities per group (>= 0); sigma: scattering (>= 0).  All host
 * memory, copied.  Call before m1_bind_state; afterwards the bound E, Fx,
 * Fy, Fz hold m n0 n1 n2 values each, group-major (group g starts at
 * g n0 n1 n2).  The group opacities replace the gray opacity model.  m = 1
 * returns to the gray model.  1 <= m <= M1_MAX_GROUPS.  M1_ESTATE once a
 * state is bound; m1_opacity_eval returns M1_ENOTSUP while m > 1. */
#define M1_MAX_GROUPS 32
m1_status m1_set_groups(m1_ctx *ctx, int m, const double *edges, const double *kP, const double *kR,
                        double sigma);

/* Ghost state of a M1_BC_FIXED side (the injected beam of the shadow test,
 * Sect. 3.3): dir 0..2, side 0 (lower) or 1 (upper),
 * state = (E, Fx, Fy, Fz) in the grid's local basis (host memory, copied),
 * E > 0 and |F| <= E.  Every fixed side needs its state before the first
 * m1_step_explicit (M1_ESTATE otherwise).  The optical depth of a fixed
 * ghost is that of the adjacent interior cell.  M1_EINVAL for a side that
 * is not fixed or an invalid state. */
m1_status m1_set_boundary_state(m1_ctx *ctx, int dir, int side, const double state[4]);

/* Irradiation heating (Sect. 2.9): q = -div F_irr per cell (device FP64,
 * n0 n1 n2 values in the state layout, caller-owned, must stay valid while
 * set), energy per unit volume and time.  Each implicit step deposits q dt:
 * it enters the S_1 row of Eq. implicit_matrix and the conserved total
 * E_g + (c/c_hat) E.  NULL switches irradiation off.  The caller updates
 * the array between steps as the paper's user function does. */
m1_status m1_set_irradiation(m1_ctx *ctx, const double *q);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one Euler step, the work of m1_step_explicit then
 * m1_step_implicit, of the gray state in the caller's arrays f (layout and
 * precision as for m1_bind_state; caller-owned, 256-byte aligned, updated
 * in place), with the step's buffers (transported state, opacity cache,
 * fix-up counters) in a static device array of M1_NOALLOC_MAX_BYTES that
 * the library holds on each device it runs on until the process ends and
 * that every context on that device shares.  The opacity cache is
 * evaluated from the gas state at the start of the call, so the result is
 * that of m1_bind_state(f) followed by one explicit and one implicit step.
 * The context needs no bound state and its own binding is left as it was.
 * A grid of N cells needs 6 ceil256(N s) + 32768 bytes (s = 4 in M1_F32, 8
 * in M1_P64): up to about 5.5e6 cells in M1_F32 and 2.7e6 in M1_P64; larger
 * grids return M1_EINVAL.  Nothing carries over from one call to the next
 * (the counters are cleared by a kernel, not a memset); calls that overlap
 * on one device (several streams or host threads) race on the shared array.
 * Asynchronous on the context's stream.  M1_ENOTSUP for multigroup
 * contexts, M1_ESTATE when a fixed boundary has no state.  The library
 * allocates nothing here; the FP64 LimO3 transport kernel keeps a few
 * registers in per-lane scratch, whose backing the HIP runtime sets up at
 * that kernel's first launch on a stream, so a caller that must not see
 * even that runs one step before the allocation-free section. */
#define M1_NOALLOC_MAX_BYTES (128u << 20)
m1_status m1_step_noalloc(m1_ctx *ctx, const m1_fields *f, double dt);

/* Second-order Runge-Kutta step of length dt built from the split step as in
 * Sect. 2.4 (every sub-step is transport then sources): U1 = S(T(U^n)),
 * U2 = S(T(U1)), U^{n+1} = (U^n + U2) / 2 for E, F (every group), m and
 * E_g (rho is frozen); the opacity cache ends at the averaged gas state.
 * U1 lives in a library buffer (4 m + 4 fields) that m1_bind_state
 * allocates when the context was created with m1_params.second_order = 1;
 * the second stage writes the average directly into the bound arrays.
 * Asynchronous.  M1_ESTATE if no state is bound or the context was created
 * without second_order. */
m1_status m1_step_rk2(m1_ctx *ctx, double dt);

/* Device pointers of the library's transported state E*, Fx*, Fy*, Fz*
 * (the state between the explicit and the implicit part of the Sect. 2.4
 * step list; valid after m1_step_explicit; owned by the library).  Gray states only
 * (M1_ENOTSUP with groups). */
m1_status m1_transported(m1_ctx *ctx, void **E, void **Fx, void **Fy, void **Fz);

/* Re-evaluate the opacity cache (rho kappa_P and the optical depth of the
 * Sect. 2.6 limiter) from the bound gas state (call after the caller
 * changes rho, m or E_g outside the library). */
m1_status m1_refresh_opacity(m1_ctx *ctx);

/* Wait for the stream; reports a deferred device error as M1_EDEVICE.
 * (Execution plumbing: no passage of the paper.) */
m1_status m1_sync(m1_ctx *ctx);

/* Synchronous reduction of the bound state (see m1_diag): the conserved
 * totals E + (c/c_hat) E_r and rho v + F_r / c_hat of Sect. 2.7, and the
 * counters of the positivity and f <= 1 fix-ups (Sect. 3.1, Sect. 2.1). */
m1_status m1_diagnostics(m1_ctx *ctx, m1_diag *out);

/* Text of the last error raised on the calling thread ("" if none).
 * (Error reporting: no passage of the paper.) */
const char *m1_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
