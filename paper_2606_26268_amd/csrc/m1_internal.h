// m1_internal.h -- library-internal context, metric layout and kernel
// launchers shared by the host API and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/m1.h"

namespace m1 {

// Separable metric of the grid, one set of 1D arrays per direction, in the
// working precision R.  Reconstruction arrays are padded with two ghost
// entries on each side (index t + 2 for t in [-2, n+1]).
template <typename R>
struct Metric {
    const R *winv[3];  // 1 / (x_t - x_{t-1}) between centres, t in [-1, n+1]
    const R *hp[3];    // x_{t+1/2} - x_t
    const R *hm[3];    // x_t - x_{t-1/2}
    // face area over cell volume for direction d:
    //   A_lo/V = alo[d][t] * trA[d][i] * trB[d][j], A_hi/V likewise with ahi
    const R *alo[3], *ahi[3], *trA[3], *trB[3];
    // extent of cell (i,j,k) along d: hd[d][t] * hI[d][i] * hJ[d][j]
    const R *hd[3], *hI[3], *hJ[3];
    const R *inv_reff;  // 1 / r_eff (per i), 0 for Cartesian
    const R *cot_eff;   // cot(theta)_eff (per j), spherical only
};

// Unsigned division by a divisor fixed for the launch, with one multiply-high
// instead of the vector ALU's long division sequence (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994,
// Sect. 4): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(x, m) and x / d = (t + ((x - t) >> min(l, 1))) >> max(l - 1, 0),
// exact for every 32-bit x and d >= 1.
struct FastDiv {
    unsigned d, m, s1, s2;
    void set(unsigned dv)
    {
        unsigned l = 0;
        while (l < 32 && (1ull << l) < dv) ++l;
        d = dv;
        m = unsigned(((1ull << 32) * ((1ull << l) - dv)) / dv + 1);
        s1 = l ? 1 : 0;
        s2 = l ? l - 1 : 0;
    }
    __device__ __forceinline__ unsigned div(unsigned x) const
    {
        const unsigned t = __umulhi(x, m);
        return (t + ((x - t) >> s1)) >> s2;
    }
};

// (i, j, k) of the cell with linear index id = (k n1 + j) n0 + i
struct CellIndex {
    FastDiv d0, d1;
    void set(int n0, int n1)
    {
        d0.set(unsigned(n0));
        d1.set(unsigned(n1));
    }
    __device__ __forceinline__ void split(int id, int &i, int &j, int &k) const
    {
        const unsigned q = d0.div(unsigned(id));
        i = int(unsigned(id) - q * d0.d);
        const unsigned kk = d1.div(q);
        j = int(q - kk * d1.d);
        k = int(kk);
    }
};

enum OpacKind { OPK_CONST = 0, OPK_POWERLAW = 1, OPK_TABLE = 2, OPK_MLP = 3 };

struct OpacityParams {
    int kind;
    double kP, kR, sigma;                       // constant
    double k0, rho0, alpha, T0, beta;           // power law
    int nr, nt;                                 // table
    double lr0, lr1, lt0, lt1, lr_off, lt_off;
    double lr_inv, lt_inv;                      // 1 / (lr1 - lr0), 1 / (lt1 - lt0)
    const float *tab_kP, *tab_kR;               // device, [nt][nr] each
    // device, per table cell (i, j) of [nt - 1][nr - 1]: kappa_P at its
    // nodes (i, j), (i+1, j), (i, j+1), (i+1, j+1), then kappa_R likewise
    // (two 16-byte words: one lookup reads 32 contiguous bytes)
    const float *tab_cells;
    const float *mlp;                           // device, packed (see mlp.hip)
    double norm[4];
    // FP32 copies of the table axes and sigma for the network's FP32
    // arithmetic (rounded once on the host instead of per wavefront)
    struct {
        float lr0, lr1, lt0, lt1, lr_off, lt_off, lr_inv, lt_inv, sigma;
    } f32;
};

// refresh OpacityParams::f32 from the FP64 fields
inline void opacity_f32(OpacityParams &o)
{
    o.f32.lr0 = float(o.lr0);
    o.f32.lr1 = float(o.lr1);
    o.f32.lt0 = float(o.lt0);
    o.f32.lt1 = float(o.lt1);
    o.f32.lr_off = float(o.lr_off);
    o.f32.lt_off = float(o.lt_off);
    o.f32.lr_inv = float(o.lr_inv);
    o.f32.lt_inv = float(o.lt_inv);
    o.f32.sigma = float(o.sigma);
}

// multigroup parameters (constant group opacities, interior band edges)
struct GroupParams {
    int m;
    double edges[M1_MAX_GROUPS];
    double kP[M1_MAX_GROUPS], kR[M1_MAX_GROUPS];
    double sigma;
};

struct ImplicitConsts {
    double dt, c_hat, c, a, gamma;
    double gm1, inv_gm1;        // gamma - 1 and its reciprocal
    double dt_ch, dt_c;         // dt c_hat, dt c
    double inv_ch, c_ratio;     // 1 / c_hat, c / c_hat
};

} // namespace m1

// Fix-up counters: each of the 4 is spread over CNT_SLOTS slots, one per
// 128-byte line (slot s of counter c at cnt[(c * CNT_SLOTS + s) * CNT_STRIDE]);
// a wavefront adds to the slot of its index, the host sums the slots.  A
// single address per counter serialised the atomics of every wavefront.
constexpr int CNT_SLOTS = 64, CNT_STRIDE = 16;
constexpr size_t CNT_BYTES = size_t(4) * CNT_SLOTS * CNT_STRIDE * sizeof(unsigned long long);

struct m1_ctx {
    int ndim = 1;
    int n[3] = {1, 1, 1};
    int bc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int geom = 0;
    double c_hat = 1.0;
    m1_params par{};
    std::vector<double> faces[3];
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 256;            // compute units of the device (pairing of transport blocks)

    // metric arrays (one allocation) in both precisions
    void *metric_buf = nullptr;
    m1::Metric<double> met64{};
    m1::Metric<float> met32{};
    double *vol_dev[3] = {nullptr, nullptr, nullptr};  // volume factors (double)
    int ign[3] = {0, 0, 0};   // inactive direction with unequal face areas
    double bc_state[3][2][4] = {};         // ghost state of fixed sides
    bool bc_state_set[3][2] = {};
    const double *irr = nullptr;           // irradiation heating per cell (caller's)
    m1::GroupParams grp{1, {}, {}, {}, 0.0};   // m > 1: multigroup
    size_t plane_bytes = 0;                // per-field stride of the scratch arrays

    // bound state
    bool bound = false;
    m1_fields f{};
    void *scratch = nullptr;  // E*, Fx*, Fy*, Fz*, tau, rkp (form precision)
    void *star[4] = {nullptr, nullptr, nullptr, nullptr};
    void *tau = nullptr, *rkp = nullptr;
    unsigned long long *cnt = nullptr;     // 4 fix-up counters, CNT_SLOTS slots each
    double *partials = nullptr;            // reduction scratch
    int npartial = 0;
    bool transported = false;
    void *rk2_save = nullptr;              // first-stage state U1 of m1_step_rk2
    size_t rk2_rad_bytes = 0;              // its per-field radiation stride (all groups)

    // opacity
    m1::OpacityParams op{};
    float *table_dev = nullptr;            // [2][nt][nr], then the cell records
    float *mlp_dev = nullptr;              // packed network
    std::vector<float> mlp_theta;          // host copy of the float32 master
};

namespace m1 {
// Device allocation that leaves no error behind: a failed hipMalloc also
// sets the thread's last HIP error, which the next launch check (the
// library's or the caller's, e.g. torch's) would report as its own; it is
// read back and cleared here, the failure being returned instead.
inline hipError_t device_alloc(void **p, size_t bytes)
{
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
    }
    return e;
}

// kernel launchers (defined in the .hip translation units)
hipError_t launch_transport(m1_ctx *c, double dt);
hipError_t launch_implicit(m1_ctx *c, double dt);
hipError_t launch_opacity_init(m1_ctx *c);
hipError_t launch_opacity_eval(m1_ctx *c, long n, const double *rho, const double *T, double *kP,
                               double *kR);
hipError_t launch_diag(m1_ctx *c, double out[8]);
hipError_t launch_implicit_rk2(m1_ctx *c, double dt, int stage);
hipError_t launch_transport_from(m1_ctx *c, double dt, const void *const rad[4]);
int mlp_pack(m1_ctx *c, const float *theta, const double *norm);
int mlp_train(m1_ctx *c, const m1_train_cfg *cfg, m1_train_report *rep);
int mlp_gradient(m1_ctx *c, const float *samples, long n, const float *theta, float *grad, double *loss);
void set_error(const std::string &msg);
void set_error(const char *msg);
hipError_t launch_zero_words(unsigned long long *p, size_t n, hipStream_t s);
} // namespace m1
