// mlp.hip -- training and packing of the opacity surrogate on gfx950.
//
// Training minimises L = (1/B) sum_b sum_o (y_bo - t_bo)^2 / 2 over
// mini-batches of table coordinates, targets t = (log10 kappa_table - mean)
// / std from bilinear lookups of the bound table.  One wavefront handles 64
// samples: forward as in inference, back-propagation with the two 64x64
// products (dL/dh1 = W2^T dz2 and dL/dW2 = sum_s dz2 h1^T) on the bfloat16
// matrix cores with split (hi + lo) operands and FP32 accumulation, the
// small layers on the vector ALU.  Per-wave gradients go to a partial buffer
// that one kernel reduces in a fixed order before the Adam update (Kingma &
// Ba 2015), so training is deterministic.
#include <cmath>
#include <cstring>
#include <vector>

#include "m1_internal.h"
#include "mlp_device.h"

namespace m1 {

constexpr int NP = M1_MLP_NPARAM;
// parameter offsets in the flat vector (W1 b1 W2 b2 W3 b3 Ws)
constexpr int P_W1 = 0, P_B1 = 128, P_W2 = 192, P_B2 = 4288, P_W3 = 4352, P_B3 = 4480, P_WS = 4482;
// transposed W2 fragments for back-propagation, after the inference pack
constexpr int MLP_OFF_W2THI = MLP_PACK_FLOATS, MLP_OFF_W2TLO = MLP_PACK_FLOATS + 2048;
// then a copy of the flat parameters, from which the inference entries are derived
constexpr int MLP_OFF_THETA = MLP_PACK_FLOATS + 4096;
constexpr int MLP_TRAIN_PACK = MLP_OFF_THETA + NP;
constexpr int LDS_STRIDE = 65;

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------

// Fragment slot of A-operand element (m, k) of a 64x64 matrix for
// v_mfma_f32_32x32x16_bf16: tile mt = m / 32, k-step ks = k / 16, lane =
// 32 ((k % 16) / 8) + m % 32, element e = k % 8.
__host__ __device__ __forceinline__ int frag_slot(int m, int k)
{
    const int mt = m >> 5, ks = k >> 4, lane = ((k & 15) >> 3) * 32 + (m & 31), e = k & 7;
    return ((mt * 4 + ks) * 64 + lane) * 8 + e;
}

static inline unsigned short host_bf16_bits(float v)
{
    unsigned int u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

static inline float host_bf16_value(unsigned short b)
{
    unsigned int u = (unsigned int)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// The inference form's LDS image in the packed network, from the flat
// parameters: the split fragments of A2 = s W2 (s = MLP_TANH_SCALE), one W2
// element per thread, and the layer-1, bias and output entries
// (mlp_image_entry).  16 blocks of 256 threads.
__global__ void __launch_bounds__(256) k_mlp_pack_infer(const float *theta, float *pk)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int u = t >> 6, k = t & 63;
    MlpShared &img = *reinterpret_cast<MlpShared *>(pk + MLP_OFF_IMG);
    const float v = MLP_TANH_SCALE * theta[P_W2 + t];
    const __bf16 h = to_bf16(v);
    const __bf16 l = to_bf16(v - float(h));
    reinterpret_cast<unsigned short *>(&img.w2[0][0][0][0])[frag_slot(u, k)] = __builtin_bit_cast(unsigned short, h);
    reinterpret_cast<unsigned short *>(&img.w2[1][0][0][0])[frag_slot(u, k)] = __builtin_bit_cast(unsigned short, l);
    mlp_image_entry(theta + P_W1, theta + P_B1, theta + P_B2, theta + P_W3, img, t);
}

static void host_pack(const float *th, const double *norm, std::vector<float> &pk)
{
    pk.assign(MLP_TRAIN_PACK, 0.0f);
    for (int i = 0; i < NP; ++i) pk[MLP_OFF_THETA + i] = th[i];
    for (int i = 0; i < 128; ++i) pk[MLP_OFF_W1 + i] = th[P_W1 + i];
    for (int i = 0; i < 64; ++i) pk[MLP_OFF_B1 + i] = th[P_B1 + i];
    for (int i = 0; i < 64; ++i) pk[MLP_OFF_B2 + i] = th[P_B2 + i];
    for (int i = 0; i < 128; ++i) pk[MLP_OFF_W3 + i] = th[P_W3 + i];
    for (int i = 0; i < 2; ++i) pk[MLP_OFF_B3 + i] = th[P_B3 + i];
    for (int i = 0; i < 4; ++i) pk[MLP_OFF_WS + i] = th[P_WS + i];
    for (int i = 0; i < 4; ++i) pk[MLP_OFF_NORM + i] = float(norm[i]);
    unsigned short *hi = reinterpret_cast<unsigned short *>(&pk[MLP_OFF_W2HI]);
    unsigned short *lo = reinterpret_cast<unsigned short *>(&pk[MLP_OFF_W2LO]);
    unsigned short *thi = reinterpret_cast<unsigned short *>(&pk[MLP_OFF_W2THI]);
    unsigned short *tlo = reinterpret_cast<unsigned short *>(&pk[MLP_OFF_W2TLO]);
    for (int u = 0; u < 64; ++u)
        for (int k = 0; k < 64; ++k) {
            const float w = th[P_W2 + u * 64 + k];
            const unsigned short h = host_bf16_bits(w);
            const unsigned short l = host_bf16_bits(w - host_bf16_value(h));
            hi[frag_slot(u, k)] = h;
            lo[frag_slot(u, k)] = l;
            thi[frag_slot(k, u)] = h;
            tlo[frag_slot(k, u)] = l;
        }
}

int mlp_pack(m1_ctx *c, const float *theta, const double *norm)
{
    std::vector<float> pk;
    host_pack(theta, norm, pk);
    if (!c->mlp_dev) {
        if (device_alloc(reinterpret_cast<void **>(&c->mlp_dev), MLP_TRAIN_PACK * sizeof(float)) != hipSuccess) {
            set_error("MLP buffer allocation failed");
            return -2;
        }
    }
    hipError_t e = hipMemcpy(c->mlp_dev, pk.data(), MLP_TRAIN_PACK * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mlp_pack_infer, dim3(16), dim3(256), 0, c->stream, c->mlp_dev + MLP_OFF_THETA,
                           c->mlp_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        set_error(std::string("MLP upload: ") + hipGetErrorString(e));
        return -3;
    }
    c->mlp_theta.assign(theta, theta + NP);
    for (int i = 0; i < 4; ++i) c->op.norm[i] = norm[i];
    c->op.mlp = c->mlp_dev;
    return 0;
}

// ---------------------------------------------------------------------------
// forward + backward of one 64-sample wavefront
// ---------------------------------------------------------------------------

struct TrainArgs {
    const float *pk;       // packed current network (inference + transposed frags)
    const float *samples;  // [n][2] table coordinates
    long n_train;
    long offset;
    float inv_batch;
    OpacityParams op;      // table (targets) and axes
    float *partial;        // [nblk][NP]
    float *loss_part;      // [nblk]
};

__device__ __forceinline__ void split8(const float v[8], bf16x8 &h, bf16x8 &l)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 b = to_bf16(v[e]);
        h[e] = b;
        l[e] = to_bf16(v[e] - float(b));
    }
}

__device__ __forceinline__ f32x16 mfma3(const bf16x8 &ah, const bf16x8 &al, const bf16x8 &bh, const bf16x8 &bl,
                                        f32x16 acc)
{
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    return acc;
}

__global__ void __launch_bounds__(64) k_mlp_fwd_bwd(TrainArgs a)
{
    __shared__ float H1[64 * LDS_STRIDE];
    __shared__ float DZ2[64 * LDS_STRIDE];
    __shared__ float H2[64 * LDS_STRIDE];   // later reused for dz1
    __shared__ float XS[64][2];
    __shared__ float DY[64][2];
    const int lane = threadIdx.x, g = lane >> 5, l32 = lane & 31;
    const float *p = a.pk;

    const long sidx = (a.offset + (long)blockIdx.x * 64 + lane) % a.n_train;
    const float lr = a.samples[2 * sidx], lt = a.samples[2 * sidx + 1];
    const float x0 = 2.0f * (lr - float(a.op.lr0)) / float(a.op.lr1 - a.op.lr0) - 1.0f;
    const float x1 = 2.0f * (lt - float(a.op.lt0)) / float(a.op.lt1 - a.op.lt0) - 1.0f;
    double tP, tR;
    table_lookup<double>(a.op, double(lr), double(lt), tP, tR);
    const float t0 = float((tP - a.op.norm[0]) / a.op.norm[1]);
    const float t1 = float((tR - a.op.norm[2]) / a.op.norm[3]);

    MlpWave net;
    net.load(p, lane);
    float h1[64];
    net.layer1(x0, x1, h1);
#pragma unroll
    for (int u = 0; u < 64; ++u) H1[lane * LDS_STRIDE + u] = h1[u];
    f32x16 acc[2][2];
    net.layer2(h1, lane, acc);
    float h2[2][2][16];
    float part[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int u = MlpWave::unit(mt, i, g);
                const float h = fast_tanh(acc[mt][nt][i] + p[MLP_OFF_B2 + u]);
                h2[mt][nt][i] = h;
                H2[(32 * nt + l32) * LDS_STRIDE + u] = h;
                part[nt][0] += p[MLP_OFF_W3 + u] * h;
                part[nt][1] += p[MLP_OFF_W3 + 64 + u] * h;
            }
    const float s0 = g ? part[0][0] : part[1][0], s1 = g ? part[0][1] : part[1][1];
    const float r0 = __shfl_xor(s0, 32), r1 = __shfl_xor(s1, 32);
    const float y0 = (g ? part[1][0] : part[0][0]) + r0 + p[MLP_OFF_B3] + p[MLP_OFF_WS] * x0 + p[MLP_OFF_WS + 1] * x1;
    const float y1 = (g ? part[1][1] : part[0][1]) + r1 + p[MLP_OFF_B3 + 1] + p[MLP_OFF_WS + 2] * x0 +
                     p[MLP_OFF_WS + 3] * x1;
    const float e0 = y0 - t0, e1 = y1 - t1;
    float lossl = 0.5f * (e0 * e0 + e1 * e1) * a.inv_batch;
    XS[lane][0] = x0;
    XS[lane][1] = x1;
    DY[lane][0] = e0 * a.inv_batch;
    DY[lane][1] = e1 * a.inv_batch;
    __syncthreads();

    // dz2 = (W3^T dy) * (1 - h2^2), in the matrix-core output layout
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int s = 32 * nt + l32;
            const float d0 = DY[s][0], d1 = DY[s][1];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int u = MlpWave::unit(mt, i, g);
                const float h = h2[mt][nt][i];
                DZ2[s * LDS_STRIDE + u] = (p[MLP_OFF_W3 + u] * d0 + p[MLP_OFF_W3 + 64 + u] * d1) * (1.0f - h * h);
            }
        }
    __syncthreads();

    float *out = a.partial + (long)blockIdx.x * NP;
    // dL/dW3[o][u] = sum_s dy_o h2[s][u]; lane = u
    {
        float g0 = 0.f, g1 = 0.f;
        for (int s = 0; s < 64; ++s) {
            const float h = H2[s * LDS_STRIDE + lane];
            g0 += DY[s][0] * h;
            g1 += DY[s][1] * h;
        }
        out[P_W3 + lane] = g0;
        out[P_W3 + 64 + lane] = g1;
        float b2 = 0.f;
        for (int s = 0; s < 64; ++s) b2 += DZ2[s * LDS_STRIDE + lane];
        out[P_B2 + lane] = b2;
    }
    if (lane < 6) {
        const int o = lane / 3, w = lane % 3;
        float acc1 = 0.f;
        for (int s = 0; s < 64; ++s) acc1 += DY[s][o] * (w == 0 ? 1.0f : XS[s][w - 1]);
        if (w == 0) out[P_B3 + o] = acc1;
        else out[P_WS + o * 2 + (w - 1)] = acc1;
    }

    // dL/dh1^T = W2^T dz2^T on the matrix cores: A = W2^T, B[k = u][n = s]
    const bf16x8 *thi = reinterpret_cast<const bf16x8 *>(p + MLP_OFF_W2THI);
    const bf16x8 *tlo = reinterpret_cast<const bf16x8 *>(p + MLP_OFF_W2TLO);
    f32x16 dh[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) dh[mt][nt][i] = 0.f;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x8 bh[2], bl[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            float v[8];
            const int s = 32 * nt + l32;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = DZ2[s * LDS_STRIDE + 16 * ks + 8 * g + e];
            split8(v, bh[nt], bl[nt]);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const bf16x8 ah = thi[(mt * 4 + ks) * 64 + lane], al = tlo[(mt * 4 + ks) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) dh[mt][nt] = mfma3(ah, al, bh[nt], bl[nt], dh[mt][nt]);
        }
    }
    __syncthreads();   // every lane is done reading H2 (dW3) before dz1 overwrites it
    float *DZ1 = H2;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int s = 32 * nt + l32;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int k = MlpWave::unit(mt, i, g);
                const float h = H1[s * LDS_STRIDE + k];
                DZ1[s * LDS_STRIDE + k] = dh[mt][nt][i] * (1.0f - h * h);
            }
        }

    // dL/dW2 = dz2^T h1 with K = samples: A[m = u][k = s], B[k = s][n = k_in]
    f32x16 gw[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) gw[mt][nt][i] = 0.f;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            float va[8], vb[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int s = 16 * ks + 8 * g + e;
                va[e] = DZ2[s * LDS_STRIDE + 32 * t + l32];
                vb[e] = H1[s * LDS_STRIDE + 32 * t + l32];
            }
            split8(va, ah[t], al[t]);
            split8(vb, bh[t], bl[t]);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) gw[mt][nt] = mfma3(ah[mt], al[mt], bh[nt], bl[nt], gw[mt][nt]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int u = MlpWave::unit(mt, i, g);
                out[P_W2 + u * 64 + 32 * nt + l32] = gw[mt][nt][i];
            }
    __syncthreads();   // dz1 complete
    {
        float gw0 = 0.f, gw1 = 0.f, gb = 0.f;
        for (int s = 0; s < 64; ++s) {
            const float d = DZ1[s * LDS_STRIDE + lane];
            gw0 += d * XS[s][0];
            gw1 += d * XS[s][1];
            gb += d;
        }
        out[P_W1 + 2 * lane] = gw0;
        out[P_W1 + 2 * lane + 1] = gw1;
        out[P_B1 + lane] = gb;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lossl += __shfl_xor(lossl, o);
    if (lane == 0) a.loss_part[blockIdx.x] = lossl;
}

// ---------------------------------------------------------------------------
// gradient reduction (fixed order), Adam, repacking
// ---------------------------------------------------------------------------

struct AdamArgs {
    float *theta, *m, *v;
    const float *partial;
    int nblk;
    float lr, b1, b2, eps, c1, c2;
    float *pk;
    const float *loss_part;
    float *loss_hist;
    long step;
};

__device__ __forceinline__ unsigned short dev_bf16_bits(float v)
{
    const __bf16 b = to_bf16(v);
    return __builtin_bit_cast(unsigned short, b);
}

// Sum of the nblk per-wavefront partial gradients of parameter i, in a
// fixed order shared by the Adam and gradient kernels (so both produce the
// same bits): a 256-thread block owns 64 consecutive parameters (one per
// lane); wavefront w adds the partials of the contiguous quarter
// [w q, w q + q) of the waves in order, and the first wavefront adds the
// four quarter sums in order w = 0..3.  Returns the sum in the threads of
// the first wavefront (i < NP); the other threads return 0.
constexpr int RED_PARAMS = 64;

__device__ __forceinline__ float reduce_partials(const float *partial, int nblk, int i, float (&sh)[4][64])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = (nblk + 3) >> 2;
    const int b0 = w * q, b1 = b0 + q < nblk ? b0 + q : nblk;
    float g = 0.f;
    if (i < NP)
        for (int b = b0; b < b1; ++b) g += partial[(long)b * NP + i];
    sh[w][lane] = g;
    __syncthreads();
    if (w != 0) return 0.f;
    return ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

__global__ void __launch_bounds__(256) k_mlp_adam(AdamArgs a)
{
    __shared__ float sh[4][64];
    const int i = blockIdx.x * RED_PARAMS + (threadIdx.x & 63);
    if (blockIdx.x == 0 && threadIdx.x == 64) {
        float L = 0.f;
        for (int b = 0; b < a.nblk; ++b) L += a.loss_part[b];
        a.loss_hist[a.step] = L;
    }
    const float g = reduce_partials(a.partial, a.nblk, i, sh);
    if (threadIdx.x >= 64 || i >= NP) return;
    const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float w = a.theta[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.theta[i] = w;
    // refresh the packed network used by the next forward pass
    float *pk = a.pk;
    if (i < P_B1) pk[MLP_OFF_W1 + i] = w;
    else if (i < P_W2) pk[MLP_OFF_B1 + (i - P_B1)] = w;
    else if (i < P_B2) {
        const int u = (i - P_W2) >> 6, k = (i - P_W2) & 63;
        const __bf16 h = to_bf16(w);
        const unsigned short hb = __builtin_bit_cast(unsigned short, h);
        const unsigned short lb = dev_bf16_bits(w - float(h));
        unsigned short *hi = reinterpret_cast<unsigned short *>(pk + MLP_OFF_W2HI);
        unsigned short *lo = reinterpret_cast<unsigned short *>(pk + MLP_OFF_W2LO);
        unsigned short *thi = reinterpret_cast<unsigned short *>(pk + MLP_OFF_W2THI);
        unsigned short *tlo = reinterpret_cast<unsigned short *>(pk + MLP_OFF_W2TLO);
        hi[frag_slot(u, k)] = hb;
        lo[frag_slot(u, k)] = lb;
        thi[frag_slot(k, u)] = hb;
        tlo[frag_slot(k, u)] = lb;
    } else if (i < P_W3) pk[MLP_OFF_B2 + (i - P_B2)] = w;
    else if (i < P_B3) pk[MLP_OFF_W3 + (i - P_W3)] = w;
    else if (i < P_WS) pk[MLP_OFF_B3 + (i - P_B3)] = w;
    else pk[MLP_OFF_WS + (i - P_WS)] = w;
}

__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, int nblk, const float *loss_part,
                                                    float *grad, float *loss)
{
    __shared__ float sh[4][64];
    const int i = blockIdx.x * RED_PARAMS + (threadIdx.x & 63);
    if (blockIdx.x == 0 && threadIdx.x == 64) {
        float L = 0.f;
        for (int b = 0; b < nblk; ++b) L += loss_part[b];
        *loss = L;
    }
    const float g = reduce_partials(partial, nblk, i, sh);
    if (threadIdx.x < 64 && i < NP) grad[i] = g;
}

// ---------------------------------------------------------------------------
// held-out error against the table
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_mlp_eval(const float *pk, const float *samples, long n, OpacityParams op,
                                                  float *blockmax)
{
    __shared__ float sh[2][256];
    __shared__ MlpShared w;
    mlp_stage(pk, w, threadIdx.x, blockDim.x);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const long id = blockIdx.x * 256L + threadIdx.x;
    const long idc = id < n ? id : n - 1;
    const float lr = samples[2 * idc], lt = samples[2 * idc + 1];
    const float x0 = 2.0f * (lr - float(op.lr0)) / float(op.lr1 - op.lr0) - 1.0f;
    const float x1 = 2.0f * (lt - float(op.lt0)) / float(op.lt1 - op.lt0) - 1.0f;
    float y0, y1;
    mlp_forward_shared(pk, w, x0, x1, lane, y0, y1);
    double tP, tR;
    table_lookup<double>(op, double(lr), double(lt), tP, tR);
    const double dP = double(y0 * pk[MLP_OFF_NORM + 1] + pk[MLP_OFF_NORM + 0]) - tP;
    const double dR = double(y1 * pk[MLP_OFF_NORM + 3] + pk[MLP_OFF_NORM + 2]) - tR;
    float mP = 0.f, mR = 0.f;
    if (id < n) {
        mP = float(fabs(exp10(dP) - 1.0));
        mR = float(fabs(exp10(dR) - 1.0));
    }
    sh[0][threadIdx.x] = mP;
    sh[1][threadIdx.x] = mR;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[0][threadIdx.x] = fmaxf(sh[0][threadIdx.x], sh[0][threadIdx.x + s]);
            sh[1][threadIdx.x] = fmaxf(sh[1][threadIdx.x], sh[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        blockmax[2 * blockIdx.x] = sh[0][0];
        blockmax[2 * blockIdx.x + 1] = sh[1][0];
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

// mean / std of each table and the least-squares plane t = b + w0 x0 + w1 x1
// (normalised units) used to initialise the linear shortcut
static void table_stats(const m1_ctx *c, const std::vector<float> &tab, double norm[4], float lin[2][3])
{
    const int nr = c->op.nr, nt = c->op.nt;
    const long n = (long)nr * nt;
    for (int o = 0; o < 2; ++o) {
        const float *T = tab.data() + o * n;
        double s = 0, s2 = 0;
        for (long q = 0; q < n; ++q) { s += T[q]; s2 += double(T[q]) * T[q]; }
        const double mean = s / n, var = s2 / n - mean * mean;
        norm[2 * o] = mean;
        norm[2 * o + 1] = var > 0 ? std::sqrt(var) : 1.0;
        // normal equations of the plane fit on the node grid
        double A[3][3] = {{0}}, b[3] = {0};
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < nr; ++i) {
                const double f[3] = {1.0, 2.0 * i / (nr - 1) - 1.0, 2.0 * j / (nt - 1) - 1.0};
                const double t = (T[(long)j * nr + i] - norm[2 * o]) / norm[2 * o + 1];
                for (int r = 0; r < 3; ++r) {
                    b[r] += f[r] * t;
                    for (int q = 0; q < 3; ++q) A[r][q] += f[r] * f[q];
                }
            }
        for (int piv = 0; piv < 3; ++piv)          // Gaussian elimination (SPD, no pivoting)
            for (int r = piv + 1; r < 3; ++r) {
                const double m = A[r][piv] / A[piv][piv];
                for (int q = piv; q < 3; ++q) A[r][q] -= m * A[piv][q];
                b[r] -= m * b[piv];
            }
        double x[3];
        for (int r = 2; r >= 0; --r) {
            double s3 = b[r];
            for (int q = r + 1; q < 3; ++q) s3 -= A[r][q] * x[q];
            x[r] = s3 / A[r][r];
        }
        lin[o][0] = float(x[0]);
        lin[o][1] = float(x[1]);
        lin[o][2] = float(x[2]);
    }
}

int mlp_train(m1_ctx *c, const m1_train_cfg *cfg, m1_train_report *rep)
{
    const long n = (long)c->op.nr * c->op.nt;
    std::vector<float> tab(2 * n);
    if (hipMemcpy(tab.data(), c->table_dev, 2 * n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("m1_mlp_train: table download failed");
        return int(M1_EDEVICE);
    }
    double norm[4];
    float lin[2][3];
    table_stats(c, tab, norm, lin);
    std::vector<float> th(cfg->theta_init, cfg->theta_init + NP);
    if (!cfg->keep_init)
        for (int o = 0; o < 2; ++o) {
            th[P_B3 + o] = lin[o][0];
            th[P_WS + 2 * o] = lin[o][1];
            th[P_WS + 2 * o + 1] = lin[o][2];
        }
    int rc = mlp_pack(c, th.data(), norm);
    if (rc) return int(M1_EDEVICE);

    const int nblk = cfg->batch / 64;
    const long n_eval_blocks = (cfg->n_eval + 255) / 256;
    // host buffers first: a failed host allocation then leaves no device
    // buffer behind
    std::vector<float> hist(cfg->steps), em(2 * n_eval_blocks);
    float *buf = nullptr;
    const size_t nbuf = 3 * size_t(NP) + size_t(nblk) * NP + nblk + cfg->steps + 2 * n_eval_blocks;
    if (device_alloc(reinterpret_cast<void **>(&buf), nbuf * sizeof(float)) != hipSuccess) {
        set_error("m1_mlp_train: allocation failed");
        return int(M1_ENOMEM);
    }
    float *theta = buf, *mom = buf + NP, *vel = buf + 2 * NP, *partial = buf + 3 * NP;
    float *loss_part = partial + size_t(nblk) * NP, *loss_hist = loss_part + nblk;
    float *evmax = loss_hist + cfg->steps;
    hipError_t e = hipMemcpyAsync(theta, th.data(), NP * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(mom, 0, 2 * NP * sizeof(float), c->stream);
    hipEvent_t ev0, ev1;
    hipEventCreate(&ev0);
    hipEventCreate(&ev1);
    hipEventRecord(ev0, c->stream);
    TrainArgs ta;
    ta.pk = c->mlp_dev;
    ta.samples = cfg->samples;
    ta.n_train = cfg->n_train;
    ta.inv_batch = 1.0f / float(cfg->batch);
    ta.op = c->op;
    ta.partial = partial;
    ta.loss_part = loss_part;
    AdamArgs aa;
    aa.theta = theta;
    aa.m = mom;
    aa.v = vel;
    aa.partial = partial;
    aa.nblk = nblk;
    aa.b1 = float(cfg->beta1);
    aa.b2 = float(cfg->beta2);
    aa.eps = float(cfg->eps);
    aa.pk = c->mlp_dev;
    aa.loss_part = loss_part;
    aa.loss_hist = loss_hist;
    for (long s = 0; s < cfg->steps && e == hipSuccess; ++s) {
        ta.offset = (s * (long)cfg->batch) % cfg->n_train;
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(nblk), dim3(64), 0, c->stream, ta);
        const double frac = cfg->steps > 1 ? double(s) / double(cfg->steps - 1) : 1.0;
        aa.lr = float(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(M_PI * frac)));
        aa.c1 = float(1.0 - std::pow(cfg->beta1, double(s + 1)));
        aa.c2 = float(1.0 - std::pow(cfg->beta2, double(s + 1)));
        aa.step = s;
        hipLaunchKernelGGL(k_mlp_adam, dim3((NP + RED_PARAMS - 1) / RED_PARAMS), dim3(256), 0, c->stream, aa);
        e = hipGetLastError();
    }
    hipEventRecord(ev1, c->stream);
    if (e == hipSuccess) {
        // the inference entries of the trained network
        hipLaunchKernelGGL(k_mlp_pack_infer, dim3(16), dim3(256), 0, c->stream, theta, c->mlp_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mlp_eval, dim3((unsigned)n_eval_blocks), dim3(256), 0, c->stream, c->mlp_dev,
                           cfg->samples + 2 * cfg->n_train, cfg->n_eval, c->op, evmax);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(th.data(), theta, NP * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hist.data(), loss_hist, cfg->steps * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(em.data(), evmax, 2 * n_eval_blocks * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float ms = 0.f;
    hipEventElapsedTime(&ms, ev0, ev1);
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    hipFree(buf);
    if (e != hipSuccess) {
        set_error(std::string("m1_mlp_train: ") + hipGetErrorString(e));
        return int(M1_EDEVICE);
    }
    double L = 0;
    const long tail = std::min<long>(100, cfg->steps);
    for (long s = cfg->steps - tail; s < cfg->steps; ++s) L += hist[s];
    rep->final_loss = L / tail;
    rep->max_rel_err_P = 0;
    rep->max_rel_err_R = 0;
    for (long b = 0; b < n_eval_blocks; ++b) {
        rep->max_rel_err_P = std::max<double>(rep->max_rel_err_P, em[2 * b]);
        rep->max_rel_err_R = std::max<double>(rep->max_rel_err_R, em[2 * b + 1]);
    }
    rep->seconds = ms * 1e-3;
    c->mlp_theta = th;   // packed device copy already holds the trained network
    return 0;
}

int mlp_gradient(m1_ctx *c, const float *samples, long n, const float *theta, float *grad, double *loss)
{
    if (mlp_pack(c, theta, c->op.norm) != 0) return int(M1_EDEVICE);
    const int nblk = int(n / 64);
    float *buf = nullptr;
    const size_t nbuf = size_t(nblk) * NP + nblk + NP + 1;
    if (device_alloc(reinterpret_cast<void **>(&buf), nbuf * sizeof(float)) != hipSuccess) {
        set_error("m1_mlp_gradient: allocation failed");
        return int(M1_ENOMEM);
    }
    float *partial = buf, *loss_part = buf + size_t(nblk) * NP, *g = loss_part + nblk, *L = g + NP;
    TrainArgs ta;
    ta.pk = c->mlp_dev;
    ta.samples = samples;
    ta.n_train = n;
    ta.offset = 0;
    ta.inv_batch = 1.0f / float(n);
    ta.op = c->op;
    ta.partial = partial;
    ta.loss_part = loss_part;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(nblk), dim3(64), 0, c->stream, ta);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + RED_PARAMS - 1) / RED_PARAMS), dim3(256), 0, c->stream, partial, nblk,
                       loss_part, g, L);
    float Lh = 0.f;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(grad, g, NP * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&Lh, L, sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    hipFree(buf);
    if (e != hipSuccess) {
        set_error(std::string("m1_mlp_gradient: ") + hipGetErrorString(e));
        return int(M1_EDEVICE);
    }
    *loss = Lh;
    return 0;
}

} // namespace m1
