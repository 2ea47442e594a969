// diag.hip -- deterministic reductions of the bound state: sum V E,
// sum V (E_g + (c/c_hat) E), sum V (m + F / c_hat), min E, max f (E and F
// summed over the frequency groups; min E and max f over every group).
// Two passes with a fixed summation order (block partials, then one block),
// so repeated calls on the same state give bit-identical results.
#include "m1_internal.h"

namespace m1 {

constexpr int DIAG_VALUES = 7;   // 5 sums, min E, max f
constexpr int DIAG_BLOCKS = 1024;

template <typename R>
struct DArgs {
    const R *E, *Fx, *Fy, *Fz;
    const double *mx, *my, *mz, *Eg;
    const double *vol[3];
    int n[3];
    int groups;                // radiation arrays hold `groups` consecutive fields
    double ratio, inv_ch;
    double *partials;
};

template <typename R>
__global__ void __launch_bounds__(256) k_diag_partial(DArgs<R> a)
{
    __shared__ double sh[DIAG_VALUES][256];
    const int n0 = a.n[0], n1 = a.n[1];
    const long N = long(n0) * n1 * a.n[2];
    double acc[5] = {0, 0, 0, 0, 0};
    double mn = 1.0e300, mx = 0.0;
    // 64-bit stride: the index past the last cell may exceed 2^31
    for (long id = long(blockIdx.x) * 256 + threadIdx.x; id < N; id += long(gridDim.x) * 256) {
        const int i = int(id % n0), j = int((id / n0) % n1), k = int(id / (long(n0) * n1));
        const double V = a.vol[0][i] * a.vol[1][j] * a.vol[2][k];
        double Et = 0.0, Ft[3] = {0.0, 0.0, 0.0};
        for (int g = 0; g < a.groups; ++g) {
            const long gid = long(g) * N + id;
            const double E = double(a.E[gid]);
            const double Fx = double(a.Fx[gid]), Fy = double(a.Fy[gid]), Fz = double(a.Fz[gid]);
            Et += E;
            Ft[0] += Fx;
            Ft[1] += Fy;
            Ft[2] += Fz;
            mn = E < mn ? E : mn;
            const double f = sqrt(Fx * Fx + Fy * Fy + Fz * Fz) / E;
            mx = f > mx ? f : mx;
        }
        acc[0] += V * Et;
        acc[1] += V * (a.Eg[id] + a.ratio * Et);
        acc[2] += V * (a.mx[id] + Ft[0] * a.inv_ch);
        acc[3] += V * (a.my[id] + Ft[1] * a.inv_ch);
        acc[4] += V * (a.mz[id] + Ft[2] * a.inv_ch);
    }
    for (int v = 0; v < 5; ++v) sh[v][threadIdx.x] = acc[v];
    sh[5][threadIdx.x] = mn;
    sh[6][threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int v = 0; v < 5; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
            sh[5][threadIdx.x] = fmin(sh[5][threadIdx.x], sh[5][threadIdx.x + s]);
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < DIAG_VALUES) a.partials[blockIdx.x * DIAG_VALUES + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_diag_final(double *partials, int nblk)
{
    __shared__ double sh[DIAG_VALUES][256];
    double acc[5] = {0, 0, 0, 0, 0};
    double mn = 1.0e300, mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        for (int v = 0; v < 5; ++v) acc[v] += partials[b * DIAG_VALUES + v];
        mn = fmin(mn, partials[b * DIAG_VALUES + 5]);
        mx = fmax(mx, partials[b * DIAG_VALUES + 6]);
    }
    for (int v = 0; v < 5; ++v) sh[v][threadIdx.x] = acc[v];
    sh[5][threadIdx.x] = mn;
    sh[6][threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int v = 0; v < 5; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
            sh[5][threadIdx.x] = fmin(sh[5][threadIdx.x], sh[5][threadIdx.x + s]);
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    // result lands after the partials of the largest grid
    if (threadIdx.x < DIAG_VALUES) partials[DIAG_BLOCKS * DIAG_VALUES + threadIdx.x] = sh[threadIdx.x][0];
}

template <typename R>
static hipError_t launch_d(m1_ctx *c, double out[8])
{
    DArgs<R> a;
    a.E = static_cast<const R *>(c->f.E);
    a.Fx = static_cast<const R *>(c->f.Fx);
    a.Fy = static_cast<const R *>(c->f.Fy);
    a.Fz = static_cast<const R *>(c->f.Fz);
    a.mx = c->f.mx;
    a.my = c->f.my;
    a.mz = c->f.mz;
    a.Eg = c->f.Eg;
    for (int d = 0; d < 3; ++d) {
        a.vol[d] = c->vol_dev[d];
        a.n[d] = c->n[d];
    }
    a.groups = c->grp.m;
    a.ratio = c->par.c / c->c_hat;
    a.inv_ch = 1.0 / c->c_hat;
    a.partials = c->partials;
    const int N = c->n[0] * c->n[1] * c->n[2];
    int nblk = (N + 255) / 256;
    nblk = nblk > DIAG_BLOCKS ? DIAG_BLOCKS : nblk;
    hipLaunchKernelGGL((k_diag_partial<R>), dim3(nblk), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, c->stream, c->partials, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(out, c->partials + DIAG_BLOCKS * DIAG_VALUES, DIAG_VALUES * sizeof(double),
                       hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

// zero n 64-bit words with a kernel (a memset node is not recorded for
// callers that capture the stream into a graph)
__global__ void __launch_bounds__(256) k_zero_words(unsigned long long *p, size_t n)
{
    const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_words(unsigned long long *p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_diag(m1_ctx *c, double out[8])
{
    if (c->par.precision == M1_F32) return launch_d<float>(c, out);
    return launch_d<double>(c, out);
}

} // namespace m1
