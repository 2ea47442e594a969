// mlp_device.h -- wavefront-cooperative evaluation of the opacity surrogate
//   x (2) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
//         -> y = W3 h2 + b3 + Ws x (2),  log10 kappa = y * std + mean
// for 64 inputs at once (one per lane).  Layers 1 and 3 run on the vector
// ALU in FP32; the 64x64 layer runs on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with each operand split into
// a bfloat16 high part and a bfloat16 remainder, keeping hi*hi + hi*lo +
// lo*hi (about 16 significant bits per product).
//
// Matrix-core operand layout used (32x32x16): lane l, g = l / 32, holds
//   A[m = l % 32][k = 8 g + e], B[k = 8 g + e][n = l % 32], e = 0..7,
//   D[row = 8 (i / 4) + 4 g + (i % 4)][col = l % 32], i = 0..15.
// The product is computed as Z2^T = W2 * H1^T: A = W2 (rows: output units),
// B = H1^T (columns: samples).
#pragma once
#include <hip/hip_runtime.h>

#include "m1_internal.h"
#include "opacity_device.h"

namespace m1 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// LDS image of the inference form (see the inference section below); the
// packed network holds it at MLP_OFF_IMG, 16-byte words copied as they are
struct MlpShared {
    bf16x8 w2[2][2][4][64];   // A2 fragments [hi, lo][mt][ks][lane], 16 KiB
    bf16x8 w1[2][64];         // layer-1 A operand: [mt][lane]
    bf16x8 c2[2][64];         // s b2 as an A operand [mt][lane]: K slots 0..2 its three bfloat16 pieces
    float2 ep[2][2][16];      // [g][mt][i]: -2 W3[0], -2 W3[1] of the slot's unit
    float w3sum[2];           // sum over units of W3[0], W3[1]
    float pad[2];             // to a whole number of 16-byte words
};
static_assert(sizeof(MlpShared) % 16 == 0, "MlpShared is staged in 16-byte words");

// Packed network (float words):
//   [0, 128)      W1[64][2]
//   [128, 192)    b1[64]
//   [192, 256)    b2[64]
//   [256, 384)    W3[2][64]
//   [384, 386)    b3[2]
//   [386, 390)    Ws[2][2]
//   [390, 394)    norm: mean_P, std_P, mean_R, std_R
//   [512, 2560)   W2 hi fragments: bf16 [mt 2][ks 4][lane 64][8]
//   [2560, 4608)  W2 lo fragments, same order
//   [4608, 9860)  the inference form's LDS image (MlpShared below), staged
//                 by every block as it is: A2 hi and lo fragments
//                 (A2 = s W2, s = MLP_TANH_SCALE, same order as W2), the
//                 layer-1 and bias operands and the output weights
// (the image serves the inference form below, whose second layer delivers
// the scaled pre-activation s (W2 h1 + b2) = A2 h1 + s b2 directly; it is
// derived on the device from the flat parameters whenever they change)
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 128, MLP_OFF_B2 = 192, MLP_OFF_W3 = 256;
constexpr int MLP_OFF_B3 = 384, MLP_OFF_WS = 386, MLP_OFF_NORM = 390;
constexpr int MLP_OFF_W2HI = 512, MLP_OFF_W2LO = 2560;
constexpr int MLP_OFF_IMG = 4608;
constexpr float MLP_TANH_SCALE = 2.8853900817779268f;   // 2 / ln 2
constexpr int MLP_PACK_FLOATS = MLP_OFF_IMG + int(sizeof(MlpShared) / 4);
static_assert(MLP_OFF_IMG % 4 == 0 && MLP_PACK_FLOATS == 9860, "packed network layout");

__device__ __forceinline__ float fast_tanh(float x)
{
    // tanh x = sign(x) (1 - e) / (1 + e), e = exp(-2 |x|), exp via exp2
    const float ax = __builtin_fabsf(x);
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * ax);
    const float t = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    return __builtin_copysignf(t, x);
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

// kappa = 10^(y std + mean) from the normalised network output y, as
// 2^((y std + mean) log2 10) on the hardware exp2 (the FP32 rounding of the
// exponent dominates either way)
__device__ __forceinline__ float net_kappa(float y, float sd, float mean)
{
    return __builtin_amdgcn_exp2f((y * sd + mean) * 3.3219280948873623f);
}

struct MlpWave {
    const float *p;
    bf16x8 w2h[2][4], w2l[2][4];

    __device__ __forceinline__ void load(const float *packed, int lane)
    {
        p = packed;
        const bf16x8 *hi = reinterpret_cast<const bf16x8 *>(packed + MLP_OFF_W2HI);
        const bf16x8 *lo = reinterpret_cast<const bf16x8 *>(packed + MLP_OFF_W2LO);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                w2h[mt][ks] = hi[(mt * 4 + ks) * 64 + lane];
                w2l[mt][ks] = lo[(mt * 4 + ks) * 64 + lane];
            }
    }

    // Layer 1 for the lane's own input: h1[0..63].
    __device__ __forceinline__ void layer1(float x0, float x1, float h1[64]) const
    {
#pragma unroll
        for (int u = 0; u < 64; ++u)
            h1[u] = fast_tanh(p[MLP_OFF_W1 + 2 * u] * x0 + p[MLP_OFF_W1 + 2 * u + 1] * x1 +
                              p[MLP_OFF_B1 + u]);
    }

    // Layer 2 pre-activations Z2^T tiles acc[mt][nt]: lane holds samples
    // 32 nt + l % 32, output units 32 mt + 8 (i / 4) + 4 g + (i % 4).
    __device__ __forceinline__ void layer2(const float h1[64], int lane, f32x16 acc[2][2]) const
    {
        const int g = lane >> 5;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[mt][nt][i] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            // own values of chunk g and the partner's (lane ^ 32) of chunk g
            bf16x8 own_h, own_l, oth_h, oth_l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float mine = g ? h1[16 * ks + 8 + e] : h1[16 * ks + e];
                const float send = g ? h1[16 * ks + e] : h1[16 * ks + 8 + e];
                const float recv = __shfl_xor(send, 32);
                const __bf16 mh = to_bf16(mine), rh = to_bf16(recv);
                own_h[e] = mh;
                own_l[e] = to_bf16(mine - float(mh));
                oth_h[e] = rh;
                oth_l[e] = to_bf16(recv - float(rh));
            }
            // tile nt: lanes of group nt supply their own sample
            const bf16x8 b0h = g == 0 ? own_h : oth_h, b0l = g == 0 ? own_l : oth_l;
            const bf16x8 b1h = g == 1 ? own_h : oth_h, b1l = g == 1 ? own_l : oth_l;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2h[mt][ks], b0h, acc[mt][0], 0, 0, 0);
                acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2h[mt][ks], b0l, acc[mt][0], 0, 0, 0);
                acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2l[mt][ks], b0h, acc[mt][0], 0, 0, 0);
                acc[mt][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2h[mt][ks], b1h, acc[mt][1], 0, 0, 0);
                acc[mt][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2h[mt][ks], b1l, acc[mt][1], 0, 0, 0);
                acc[mt][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2l[mt][ks], b1h, acc[mt][1], 0, 0, 0);
            }
        }
    }

    // Output unit held in slot i of tile mt by lane group g.
    static __device__ __forceinline__ int unit(int mt, int i, int g)
    {
        return 32 * mt + 8 * (i >> 2) + 4 * g + (i & 3);
    }

    // Full forward for the lane's own input x -> y (normalised outputs).
    __device__ __forceinline__ void forward(float x0, float x1, int lane, float &y0, float &y1) const
    {
        float h1[64];
        layer1(x0, x1, h1);
        f32x16 acc[2][2];
        layer2(h1, lane, acc);
        const int g = lane >> 5;
        float part[2][2] = {{0.f, 0.f}, {0.f, 0.f}};  // [nt][output]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int u = unit(mt, i, g);
                    const float h2 = fast_tanh(acc[mt][nt][i] + p[MLP_OFF_B2 + u]);
                    part[nt][0] += p[MLP_OFF_W3 + u] * h2;
                    part[nt][1] += p[MLP_OFF_W3 + 64 + u] * h2;
                }
        // the partner lane holds the other 32 units of the same samples
        const float s0 = g ? part[0][0] : part[1][0];
        const float s1 = g ? part[0][1] : part[1][1];
        const float r0 = __shfl_xor(s0, 32), r1 = __shfl_xor(s1, 32);
        const float m0 = g ? part[1][0] : part[0][0];
        const float m1 = g ? part[1][1] : part[0][1];
        y0 = m0 + r0 + p[MLP_OFF_B3] + p[MLP_OFF_WS] * x0 + p[MLP_OFF_WS + 1] * x1;
        y1 = m1 + r1 + p[MLP_OFF_B3 + 1] + p[MLP_OFF_WS + 2] * x0 + p[MLP_OFF_WS + 3] * x1;
    }

    // Network inputs from (rho, T) through the table axes and offsets.
    static __device__ __forceinline__ void inputs(const OpacityParams &op, float rho, float T, float &x0,
                                                  float &x1)
    {
        // log10 through the hardware log2 (the network inputs carry FP32
        // rounding in any case), clamped to the table axes
        constexpr float LOG10_2 = 0.30102999566398120f;
        const auto &q = op.f32;
        float lr = __builtin_amdgcn_logf(rho) * LOG10_2 + q.lr_off;
        float lt = __builtin_amdgcn_logf(T) * LOG10_2 + q.lt_off;
        lr = __builtin_fminf(__builtin_fmaxf(lr, q.lr0), q.lr1);
        lt = __builtin_fminf(__builtin_fmaxf(lt, q.lt0), q.lt1);
        x0 = 2.0f * (lr - q.lr0) * q.lr_inv - 1.0f;
        x1 = 2.0f * (lt - q.lt0) * q.lt_inv - 1.0f;
    }

    __device__ __forceinline__ void opacity(const OpacityParams &op, float rho, float T, int lane, float &kP,
                                            float &kR) const
    {
        float x0, x1, y0, y1;
        inputs(op, rho, T, x0, x1);
        forward(x0, x1, lane, y0, y1);
        kP = net_kappa(y0, p[MLP_OFF_NORM + 1], p[MLP_OFF_NORM + 0]);
        kR = net_kappa(y1, p[MLP_OFF_NORM + 3], p[MLP_OFF_NORM + 2]);
    }
};


// ---------------------------------------------------------------------------
// Inference form.  A wavefront evaluates 64 inputs as two 32-sample column
// tiles of the matrix-core products, both hidden layers on the matrix cores.
//
// Layer 1 (K = 16 per 32-unit tile): inputs and weights are split exactly
// into three bfloat16 pieces (h + m + l, 24 significant bits), and the six
// cross terms hh, hm, mh, hl, lh, mm of each weight-input product plus the
// three bias pieces fill the K slots, so the pre-activation carries
// single-precision accuracy (the dropped terms are below 2^-24 relative).
// The rows of W1 are permuted (bits 2 and 3 of the row index swapped) so
// that each lane's accumulator slots 8 hs .. 8 hs + 7 are exactly the units
// 16 ks + 8 g + e (ks = 2 mt + hs) that layer 2 wants from the lane as its
// B operand: no hidden value changes lanes.
//
// tanh is evaluated as 1 - 2 r with r = 1 / (1 + 2^z), z = 2 log2(e) x =
// s x.  The factor s is folded into the staged first-layer weights and into
// the second layer: its weights are A2 = s W2 (split hi + lo, packed with
// the network) and its accumulator starts at s b2 (one more matrix product,
// s b2 in three exact bfloat16 pieces against a column of ones), so the
// matrix cores deliver z2 = s (W2 h1 + b2) directly; the output layer takes
// h2 = 1 - 2 r2 as sum W3 - 2 sum W3 r2.  (Folding h1 = 1 - 2 r1 into the
// second layer as well would save one more operation per unit, but the
// products would then carry the split error of r1 ~ 1/2 where h1 is small:
// measured, 3.4e-5 against 6-8e-6 in log10 kappa from the exact network on
// random weights, five times the error.)
// ---------------------------------------------------------------------------

// tanh(z / MLP_TANH_SCALE); saturates to -1 and +1 for large |z|
__device__ __forceinline__ float tanh_scaled(float z)
{
    return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z)), 1.0f);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Split two floats into packed bfloat16 high parts (round to nearest even)
// and packed bfloat16 remainders: a = hi_a + lo_a + O(2^-18 |a|).
__device__ __forceinline__ void split_bf16x2(float a, float b, unsigned &hi, unsigned &lo)
{
    const bf16x2_t h = {to_bf16(a), to_bf16(b)};
    hi = __builtin_bit_cast(unsigned, h);
    // a's high part moved to the upper half by a byte permutation of the
    // packed word (bytes 1, 0 to 3, 2; zeros below): written as a shift,
    // the compiler re-derives it from a with one more conversion
    const float ha = __uint_as_float(__builtin_amdgcn_perm(0u, hi, 0x01000c0cu));
    const float hb = __uint_as_float(hi & 0xffff0000u);
    const bf16x2_t l = {to_bf16(a - ha), to_bf16(b - hb)};
    lo = __builtin_bit_cast(unsigned, l);
}

// Exact three-piece split v = h + m + l (bfloat16 each), returned packed as
// (h, m) and (h, l).
__device__ __forceinline__ void split3_bf16(float v, unsigned &hm, unsigned &hl)
{
    const float h = __uint_as_float(__builtin_bit_cast(unsigned short, to_bf16(v)) << 16);
    const float r = v - h;
    const bf16x2_t p0 = {to_bf16(v), to_bf16(r)};
    hm = __builtin_bit_cast(unsigned, p0);
    const float r2 = r - __uint_as_float(hm & 0xffff0000u);
    const bf16x2_t p1 = {to_bf16(v), to_bf16(r2)};
    hl = __builtin_bit_cast(unsigned, p1);
}

// row of a 32-row layer-1 tile -> hidden unit it computes (bits 2, 3 swapped)
__host__ __device__ constexpr int mlp_l1_unit(int mt, int r)
{
    return 32 * mt + (r & 0x13) + ((r & 4) << 1) + ((r & 8) >> 1);
}

// Entries of the LDS image derived from the flat parameters (W1 [64][2],
// b1 [64], b2 [64], W3 [2][64] of the flat vector), for thread t of a
// 4096-thread pack grid (the A2 fragments are written elsewhere): t < 128
// the layer-1 operand, 128 <= t < 256 the bias operand, 256 <= t < 320 the
// output weights, and the wavefront 320 <= t < 384 (which runs this branch
// whole) the sums of W3 in a fixed order.
__device__ __forceinline__ void mlp_image_entry(const float *W1, const float *b1, const float *b2, const float *W3,
                                                MlpShared &img, int t)
{
    if (t < 128) {
        // layer-1 A operand of lane l in tile mt: row l % 32, K = 8 (l / 32) + e
        const int mt = t >> 6, l = t & 63, g = l >> 5;
        const int u = mlp_l1_unit(mt, l & 31);
        const float w = MLP_TANH_SCALE * W1[2 * u + g];
        const float bias = MLP_TANH_SCALE * b1[u];
        unsigned whm, whl, bhm, bhl;
        split3_bf16(w, whm, whl);
        split3_bf16(bias, bhm, bhl);
        const unsigned wh = whm & 0xffffu, wm = whm >> 16, wl = whl >> 16;
        const unsigned bh = bhm & 0xffffu, bm = bhm >> 16, bl = bhl >> 16;
        // K slots: Wh Wh Wm Wh Wl Wm | bias (g = 0: bh bm; g = 1: bl 0)
        uint4 v;
        v.x = wh | (wh << 16);
        v.y = wm | (wh << 16);
        v.z = wl | (wm << 16);
        v.w = g ? bl : (bh | (bm << 16));
        img.w1[mt][l] = __builtin_bit_cast(bf16x8, v);
    } else if (t < 256) {
        // the accumulator's start s b2 enters through one more product, A =
        // s b2 in K slots 0..2 (exact three-piece split) against B = 1 there
        const int q = t - 128, mt = q >> 6, l = q & 63;
        unsigned hm, hl;
        split3_bf16(MLP_TANH_SCALE * b2[32 * mt + (l & 31)], hm, hl);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (l < 32) {
            v.x = hm;              // K 0, 1: c2 hi, c2 mid
            v.y = hl >> 16;        // K 2: c2 lo
        }
        img.c2[mt][l] = __builtin_bit_cast(bf16x8, v);
    } else if (t < 320) {
        // the output layer takes h2 = 1 - 2 r (r = 1 / (1 + 2^z)) as
        // sum W3 - 2 sum W3 r: weights -2 W3 per unit, the sum once per output
        const int q = t - 256, g = q >> 5, mt = (q >> 4) & 1, i = q & 15;
        const int u = MlpWave::unit(mt, i, g);
        img.ep[g][mt][i] = make_float2(-2.0f * W3[u], -2.0f * W3[64 + u]);
    } else if (t < 384) {
        const int lane = t - 320;
        float s0 = W3[lane], s1 = W3[64 + lane];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            s0 += __shfl_xor(s0, o);
            s1 += __shfl_xor(s1, o);
        }
        if (lane == 0) {
            img.w3sum[0] = s0;
            img.w3sum[1] = s1;
            img.pad[0] = img.pad[1] = 0.0f;
        }
    }
}

// Stage the inference form's LDS image: a copy of 16-byte words.
__device__ __forceinline__ void mlp_stage(const float *packed, MlpShared &sh, int tid, int nthreads)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(packed + MLP_OFF_IMG);
    uint4 *dst = reinterpret_cast<uint4 *>(&sh);
    for (int q = tid; q < int(sizeof(MlpShared) / 16); q += nthreads) dst[q] = src[q];
}

__device__ __forceinline__ void mlp_forward_shared(const float *p, const MlpShared &sh, float x0, float x1, int lane,
                                                   float &y0, float &y1)
{
    const int g = lane >> 5;
    // layer-1 B operand: lanes of group 0 supply input 0, group 1 input 1, of
    // sample l % 32 (tile 0) and 32 + l % 32 (tile 1)
    const float mine = g ? x1 : x0;
    const float recv = __shfl_xor(g ? x0 : x1, 32);
    const float xin[2] = {g ? recv : mine, g ? mine : recv};
    bf16x8 b1op[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        unsigned hm, hl;
        split3_bf16(xin[nt], hm, hl);
        // K slots: xh xm xh xl xh xm | 1 1 (group 0) or 1 0 (group 1)
        uint4 v;
        v.x = hm;
        v.y = hl;
        v.z = hm;
        v.w = g ? 0x00003f80u : 0x3f803f80u;
        b1op[nt] = __builtin_bit_cast(bf16x8, v);
    }
    // B operand of the bias product: 1 in K slots 0..2 (lanes of group 0)
    const bf16x8 ones = __builtin_bit_cast(bf16x8, g ? make_uint4(0u, 0u, 0u, 0u)
                                                    : make_uint4(0x3f803f80u, 0x3f80u, 0u, 0u));
    f32x16 acc[2][2];
#pragma unroll
    for (int m1 = 0; m1 < 2; ++m1) {
        const bf16x8 a1 = sh.w1[m1][lane];
        f32x16 z1[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) z1[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1op[nt], f32x16{}, 0, 0, 0);
#pragma unroll
        for (int hs = 0; hs < 2; ++hs) {
            const int ks = 2 * m1 + hs;
            bf16x8 bh[2], bl[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                float h[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) h[e] = tanh_scaled(z1[nt][8 * hs + e]);
                uint4 ph, pl;
                split_bf16x2(h[0], h[1], ph.x, pl.x);
                split_bf16x2(h[2], h[3], ph.y, pl.y);
                split_bf16x2(h[4], h[5], ph.z, pl.z);
                split_bf16x2(h[6], h[7], ph.w, pl.w);
                bh[nt] = __builtin_bit_cast(bf16x8, ph);
                bl[nt] = __builtin_bit_cast(bf16x8, pl);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const bf16x8 ah = sh.w2[0][mt][ks][lane], al = sh.w2[1][mt][ks][lane];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const f32x16 c0 = ks == 0 ? __builtin_amdgcn_mfma_f32_32x32x16_bf16(sh.c2[mt][lane], ones,
                                                                                         f32x16{}, 0, 0, 0)
                                              : acc[mt][nt];
                    f32x16 t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[nt], c0, 0, 0, 0);
                    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[nt], t, 0, 0, 0);
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[nt], t, 0, 0, 0);
                }
            }
        }
    }
    float part[2][2] = {{0.f, 0.f}, {0.f, 0.f}};   // [nt][output]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float2 w = sh.ep[g][mt][i];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const float r = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(acc[mt][nt][i]));
                part[nt][0] = __builtin_fmaf(w.x, r, part[nt][0]);
                part[nt][1] = __builtin_fmaf(w.y, r, part[nt][1]);
            }
        }
    // the partner lane holds the other 32 units of the same samples
    const float s0 = g ? part[0][0] : part[1][0];
    const float s1 = g ? part[0][1] : part[1][1];
    const float r0 = __shfl_xor(s0, 32), r1 = __shfl_xor(s1, 32);
    const float m0 = g ? part[1][0] : part[0][0];
    const float m1 = g ? part[1][1] : part[0][1];
    y0 = m0 + r0 + (p[MLP_OFF_B3] + sh.w3sum[0]) + p[MLP_OFF_WS] * x0 + p[MLP_OFF_WS + 1] * x1;
    y1 = m1 + r1 + (p[MLP_OFF_B3 + 1] + sh.w3sum[1]) + p[MLP_OFF_WS + 2] * x0 + p[MLP_OFF_WS + 3] * x1;
}

__device__ __forceinline__ void mlp_opacity_shared(const OpacityParams &op, const MlpShared &sh, float rho, float T,
                                                   int lane, float &kP, float &kR)
{
    const float *p = op.mlp;
    float x0, x1, y0, y1;
    MlpWave::inputs(op, rho, T, x0, x1);
    mlp_forward_shared(p, sh, x0, x1, lane, y0, y1);
    kP = net_kappa(y0, p[MLP_OFF_NORM + 1], p[MLP_OFF_NORM + 0]);
    kR = net_kappa(y1, p[MLP_OFF_NORM + 3], p[MLP_OFF_NORM + 2]);
}

} // namespace m1
