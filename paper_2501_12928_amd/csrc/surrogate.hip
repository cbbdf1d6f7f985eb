// Learned surrogate of logL(theta): an ensemble of small fully connected
// networks n_in -> H -> H -> 1 with GELU after each hidden layer, in FP32,
// trained on exact evaluations by these kernels (forward, hand-derived
// backward, Adam) and used to gate sampler proposals, with the exact FP64
// likelihood as the fallback and as the arbiter of every accepted point.
//
// Layout per member (flat FP32, row-major matrices):
//   W1 [H x n_in], b1 [H], W2 [H x H], b2 [H], W3 [H], b3 [1]
// (P numbers). On the device member z starts at z * PP, PP = P rounded up
// to 64 floats, so that with H % 4 == 0 every row of W2 is 16-byte aligned;
// the API copies in and out of the packed [members x P] layout.
// Inputs are theta mapped from the prior box to [-1, 1]; targets are logL
// standardised by the training mean and standard deviation.
//
// One training step is two kernels:
//  - mlp_kernel<CT, 8, 1, true>: one workgroup per 16 samples of one member
//    gathers its inputs, runs both hidden layers, the output, the loss and
//    the backward pass down to dZ1 with the activations in LDS and
//    registers (FP32 MFMA 16x16x4), writes H1^T and dZ2^T (the operands of
//    the W2 gradient) and its samples' share of every other gradient;
//  - mlp_update_kernel: the W2 gradient as a sum over the minibatch on MFMA
//    (32 x 32 tile per workgroup) and the fixed-order sum of the per-block
//    shares of the other parameters, each followed by the Adam update of the
//    same parameters.
// Inference is mlp_kernel without the backward pass, 32 samples per
// workgroup. Every reduction has a fixed order, so training is
// deterministic for a given seed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "common.h"

// Fixed device scratch of eor_surrogate_gate_noalloc (see kGateScratchFloats).
static __device__ __align__(256) float scratch[(int64_t)1 << 22];

namespace {

using eor::f4;

constexpr int NI_MAX = 64;       // network inputs
constexpr int XS = NI_MAX + 4;   // LDS row stride of the inputs
constexpr int H_MAX = 512;       // hidden units (a multiple of 4)
constexpr int ST = 16;           // samples per MFMA row tile

__device__ inline f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Adam with bias-corrected moments, c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__device__ inline void adam_update(float *p, float g, float *m, float *v, float lr, float b1, float b2, float eps,
                                   float c1, float c2) {
    const float me = b1 * *m + (1.0f - b1) * g;
    const float ve = b2 * *v + (1.0f - b2) * g * g;
    *m = me;
    *v = ve;
    *p -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

__device__ inline void adam_factors(const int64_t *step, int64_t add, float b1, float b2, float *c1, float *c2) {
    const double t = (double)(*step + add + 1);
    *c1 = (float)(1.0 - pow((double)b1, t));
    *c2 = (float)(1.0 - pow((double)b2, t));
}

struct MlpArgs {
    // input row of sample s of member z: r = idx ? idx[z idxz + s] : s; its
    // features are theta[r] mapped to [-1, 1] (when theta is set, shared by
    // all members) or X[z xz + r n_in ...]; its target Y[z yz + r]
    const float *X;
    int64_t xz;
    const double *theta, *lo, *hi;
    const int32_t *idx;
    int64_t idxz;
    const float *Y;
    int64_t yz;
    int nb;  // samples (the loss is their mean)
    const float *params;
    int64_t PP, offb1, offW2, offb2, offW3, offb3;
    int n_in, H;
    // forward only: f[z fz + s] = network output, minus the target when Y is set
    float *f;
    int64_t fz;
    // backward: H1T, dZ2T [z][padded width][nbp]; part [z][block][PS]
    float *H1T, *dZ2T;
    int64_t nbp;
    float *part;
    int64_t PS;
};

// Shares of one block of samples, in part[z][block][...]: gW1 [H x n_in],
// gb1 [H], gb2 [H], gW3 [H], gb3, and the block's sum of squared residuals.
__host__ __device__ inline int64_t share_count(int H, int n_in) { return (int64_t)H * n_in + 3 * (int64_t)H + 2; }

// One workgroup of NW waves per RT * 16 samples of member blockIdx.y; wave
// w owns hidden units [16 CT w, 16 CT (w + 1)) of both layers (the hidden
// width is padded to 16 CT NW; padded units carry zero weights and stay
// exactly zero). In an MFMA step t, lane group q = lane / 16 supplies the
// operand pair of reduction index 4 q + t within a group of 16, for A and
// B alike, so that each lane loads four consecutive k with one 16-byte read.
template <int CT, int NW, int RT, bool BWD>
__global__ __launch_bounds__(64 * NW) void mlp_kernel(MlpArgs a) {
    static_assert(!BWD || RT == 1, "the backward pass takes 16 samples per workgroup");
    constexpr int FS = ST * RT;       // samples per workgroup
    constexpr int HP = 16 * CT * NW;
    constexpr int HS = HP + 4;        // LDS row stride of the hidden activations
    __shared__ __align__(16) float xs[FS * XS];
    __shared__ __align__(16) float hs[FS * HS];
    __shared__ float fpart[NW * FS];
    __shared__ float dfs[FS];
    __shared__ float r2s[FS];
    const int z = blockIdx.y, s0 = blockIdx.x * FS;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    // HK: the reduction length over hidden units, H rounded up to 32 (the
    // LDS rows are zero from H to 16 CT NW)
    const int H = a.H, n_in = a.n_in, nip = (n_in + 15) & ~15, HK = (H + 31) & ~31;
    const float *P = a.params + (int64_t)z * a.PP;
    const float *W2 = P + a.offW2;

    for (int e = tid; e < FS * nip; e += 64 * NW) {
        const int s = e / nip, k = e - s * nip, gs = s0 + s;
        float v = 0.0f;
        if (k < n_in && gs < a.nb) {
            const int64_t r = a.idx ? (int64_t)a.idx[z * a.idxz + gs] : (int64_t)gs;
            if (a.theta)
                v = (float)(2.0 * (a.theta[r * n_in + k] - a.lo[k]) / (a.hi[k] - a.lo[k]) - 1.0);
            else
                v = a.X[z * a.xz + r * n_in + k];
        }
        xs[s * XS + k] = v;
    }
    __syncthreads();

    const int hb = 16 * CT * w;
    f4 acc[RT][CT];
    // layer 1: Z1[s][h] = sum_k x[s][k] W1[h][k] + b1[h]
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[rt][c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int g = 0; g < nip; g += 16) {
        float wv[CT][4];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int h = hb + 16 * c + l16;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = g + 4 * q + t;
                wv[c][t] = (h < H && k < n_in) ? P[h * n_in + k] : 0.0f;
            }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const f4 xv = *reinterpret_cast<const f4 *>(&xs[(ST * rt + l16) * XS + g + 4 * q]);
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[rt][c] = mfma32(xv[t], wv[c][t], acc[rt][c]);
        }
    }
    // lane holds Z1[16 rt + 4 q + r][hb + 16 c + l16]
    f4 g1[BWD ? CT : 1];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int h = hb + 16 * c + l16;
        const float b = h < H ? P[a.offb1 + h] : 0.0f;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            f4 hv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float zz = acc[rt][c][r] + b;
                hv[r] = gelu_f(zz);
                if constexpr (BWD) g1[c][r] = gelu_grad_f(zz);
                hs[(ST * rt + 4 * q + r) * HS + h] = hv[r];
            }
            if constexpr (BWD) *reinterpret_cast<f4 *>(&a.H1T[((int64_t)z * HP + h) * a.nbp + s0 + 4 * q]) = hv;
        }
    }
    __syncthreads();

    // layer 2: Z2[s][o] = sum_k H1[s][k] W2[o][k] + b2[o]
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[rt][c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    // W2 reads run one group of 16 k ahead of the MFMAs that use them
    f4 wv[CT];
    auto load_w2 = [&](int g, f4 *dst) {
        const bool kin = g + 4 * q < H;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int o = hb + 16 * c + l16;
            dst[c] = (o < H && kin) ? *reinterpret_cast<const f4 *>(&W2[(int64_t)o * H + g + 4 * q])
                                    : f4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    // two groups of 16 k in flight: group g + 32 is read while g is multiplied
    f4 wb[CT];
    load_w2(0, wv);
    load_w2(16, wb);
    auto step2 = [&](int g, const f4 *w) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const f4 hv = *reinterpret_cast<const f4 *>(&hs[(ST * rt + l16) * HS + g + 4 * q]);
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[rt][c] = mfma32(hv[t], w[c][t], acc[rt][c]);
        }
    };
    for (int g = 0; g < HK; g += 32) {
        step2(g, wv);
        load_w2(g + 32, wv);
        step2(g + 16, wb);
        load_w2(g + 48, wb);
    }
    // output f[s] = sum_o GELU(Z2[s][o]) W3[o] + b3: this wave's units, then
    // the 16 lanes of a group (fixed xor tree), then the waves in order
    f4 h2[BWD ? CT : 1], gw[BWD ? CT : 1];
    float fp[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) fp[rt][r] = 0.0f;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int o = hb + 16 * c + l16;
        const float b = o < H ? P[a.offb2 + o] : 0.0f;
        const float w3 = o < H ? P[a.offW3 + o] : 0.0f;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float zz = acc[rt][c][r] + b;
                const float hv = gelu_f(zz);
                fp[rt][r] += hv * w3;
                if constexpr (BWD) {
                    h2[c][r] = hv;
                    gw[c][r] = w3 * gelu_grad_f(zz);
                }
            }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v = fp[rt][r];
            v += __shfl_xor(v, 8);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 1);
            if (l16 == 0) fpart[w * FS + ST * rt + 4 * q + r] = v;
        }
    __syncthreads();
    if (tid < FS) {
        const int s = tid, gs = s0 + s;
        float f = fpart[s];
#pragma unroll
        for (int v = 1; v < NW; ++v) f += fpart[v * FS + s];
        f += P[a.offb3];
        const bool valid = gs < a.nb;
        float res = 0.0f;
        if (valid && a.Y) {
            const int64_t r = a.idx ? (int64_t)a.idx[z * a.idxz + gs] : (int64_t)gs;
            res = f - a.Y[z * a.yz + r];
        }
        if constexpr (BWD) {
            dfs[s] = valid ? 2.0f * res / (float)a.nb : 0.0f;
            r2s[s] = res * res;
        } else {
            if (valid) a.f[z * a.fz + gs] = a.Y ? res : f;
        }
    }
    if constexpr (BWD) {
        float *part = a.part + ((int64_t)z * gridDim.x + blockIdx.x) * a.PS;
        const int64_t pW1 = 0, pb1 = (int64_t)H * n_in, pb2 = pb1 + H, pW3 = pb2 + H, pb3 = pW3 + H;
        __syncthreads();
        // dZ2 = dF W3 GELU'(Z2): into LDS (the A operand of dH1) and dZ2^T
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int o = hb + 16 * c + l16;
            f4 d;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                d[r] = dfs[4 * q + r] * gw[c][r];
                hs[(4 * q + r) * HS + o] = d[r];
            }
            *reinterpret_cast<f4 *>(&a.dZ2T[((int64_t)z * HP + o) * a.nbp + s0 + 4 * q]) = d;
            float sb = ((d[0] + d[1]) + d[2]) + d[3];
            float sw = dfs[4 * q] * h2[c][0];
            sw += dfs[4 * q + 1] * h2[c][1];
            sw += dfs[4 * q + 2] * h2[c][2];
            sw += dfs[4 * q + 3] * h2[c][3];
            sb += __shfl_xor(sb, 16);
            sb += __shfl_xor(sb, 32);
            sw += __shfl_xor(sw, 16);
            sw += __shfl_xor(sw, 32);
            if (q == 0 && o < H) {
                part[pb2 + o] = sb;
                part[pW3 + o] = sw;
            }
        }
        if (tid == 0) {
            float sb = 0.0f, sl = 0.0f;
            for (int s = 0; s < ST; ++s) {
                sb += dfs[s];
                sl += r2s[s];
            }
            part[pb3] = sb;
            part[pb3 + 1] = sl;
        }
        __syncthreads();
        // dH1[s][i] = sum_o dZ2[s][o] W2[o][i]
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[0][c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        float wt[4][CT];
        auto load_w2t = [&](int g, float (*dst)[CT]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int o = g + 4 * q + t;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const int i = hb + 16 * c + l16;
                    dst[t][c] = (o < H && i < H) ? W2[(int64_t)o * H + i] : 0.0f;
                }
            }
        };
        float wtb[4][CT];
        load_w2t(0, wt);
        load_w2t(16, wtb);
        auto step6 = [&](int g, float (*w)[CT]) {
            const f4 dv = *reinterpret_cast<const f4 *>(&hs[l16 * HS + g + 4 * q]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int c = 0; c < CT; ++c) acc[0][c] = mfma32(dv[t], w[t][c], acc[0][c]);
        };
        for (int g = 0; g < HK; g += 32) {
            step6(g, wt);
            load_w2t(g + 32, wt);
            step6(g + 16, wtb);
            load_w2t(g + 48, wtb);
        }
        // dZ1 = dH1 GELU'(Z1); shares of gb1 and of gW1 = dZ1^T x (the lane's
        // dZ1 values are the A operand of that product as they stand)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int h = hb + 16 * c + l16;
            f4 d1;
#pragma unroll
            for (int r = 0; r < 4; ++r) d1[r] = acc[0][c][r] * g1[c][r];
            float sb = ((d1[0] + d1[1]) + d1[2]) + d1[3];
            sb += __shfl_xor(sb, 16);
            sb += __shfl_xor(sb, 32);
            if (q == 0 && h < H) part[pb1 + h] = sb;
            for (int g = 0; g < nip; g += 16) {
                f4 ga = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int t = 0; t < 4; ++t) ga = mfma32(d1[t], xs[(4 * q + t) * XS + g + l16], ga);
                // lane holds gW1[hb + 16 c + 4 q + r][g + l16]
                const int k = g + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int hh = hb + 16 * c + 4 * q + r;
                    if (hh < H && k < n_in) part[pW1 + (int64_t)hh * n_in + k] = ga[r];
                }
            }
        }
    }
}

struct UpdArgs {
    const float *H1T, *dZ2T;  // [z][HP][nbp]
    int64_t nbp;
    int HP;
    const float *part;        // [z][nblk][PS]
    int64_t PS;
    int nblk;
    int H, n_in, nb;
    int64_t PP, offb1, offW2, offb2, offW3, offb3;
    float *grad;              // [z][PP], written when set
    float *loss;              // [z], written when set
    float *params, *mom, *vel;  // Adam when params is set
    float lr, b1, b2, eps;
    const int64_t *step;      // Adam step t = *step + step_add + 1
    int64_t step_add;
};

// Workgroups [0, (HP/32)^2) of member blockIdx.y: a 32 x 32 tile of
// gW2[o][i] = sum_s dZ2[s][o] H1[s][i] over the padded batch (whose padding
// holds dZ2 = 0); each wave sums every fourth group of 16 samples into all
// four 16 x 16 sub-tiles, then the four partial tiles are added in wave
// order. The other workgroups: 256 consecutive shares each, summed over the
// blocks in order.
__global__ __launch_bounds__(256) void mlp_update_kernel(UpdArgs a) {
    const int z = blockIdx.y, tid = threadIdx.x;
    const int tt = a.HP / 32, ntile = tt * tt;
    const int64_t zp = (int64_t)z * a.PP;
    float c1 = 1.0f, c2 = 1.0f;
    if (a.params) adam_factors(a.step, a.step_add, a.b1, a.b2, &c1, &c2);
    if ((int)blockIdx.x < ntile) {
        __shared__ f4 red[4][4][64];  // [wave][16 x 16 sub-tile][lane]
        const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
        const int o0 = 32 * ((int)blockIdx.x / tt), i0 = 32 * ((int)blockIdx.x % tt);
        const float *A0 = a.dZ2T + ((int64_t)z * a.HP + o0 + l16) * a.nbp + 4 * q;
        const float *A1 = A0 + 16 * a.nbp;
        const float *B0 = a.H1T + ((int64_t)z * a.HP + i0 + l16) * a.nbp + 4 * q;
        const float *B1 = B0 + 16 * a.nbp;
        // sub-tile j = 2 oh + ih covers rows o0 + 16 oh, columns i0 + 16 ih
        f4 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        // wave w takes the groups of 16 samples g = w, w + 4, ..., four in flight
        const int ng = (int)(a.nbp / 16);
        int g = w;
        for (; g + 12 < ng; g += 16) {
            f4 av[4][2], bv[4][2];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t k = 16 * (int64_t)(g + 4 * u);
                av[u][0] = *reinterpret_cast<const f4 *>(A0 + k);
                av[u][1] = *reinterpret_cast<const f4 *>(A1 + k);
                bv[u][0] = *reinterpret_cast<const f4 *>(B0 + k);
                bv[u][1] = *reinterpret_cast<const f4 *>(B1 + k);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[j] = mfma32(av[u][j >> 1][t], bv[u][j & 1][t], acc[j]);
        }
        for (; g < ng; g += 4) {
            const int64_t k = 16 * (int64_t)g;
            const f4 av0 = *reinterpret_cast<const f4 *>(A0 + k), av1 = *reinterpret_cast<const f4 *>(A1 + k);
            const f4 bv0 = *reinterpret_cast<const f4 *>(B0 + k), bv1 = *reinterpret_cast<const f4 *>(B1 + k);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                acc[0] = mfma32(av0[t], bv0[t], acc[0]);
                acc[1] = mfma32(av0[t], bv1[t], acc[1]);
                acc[2] = mfma32(av1[t], bv0[t], acc[2]);
                acc[3] = mfma32(av1[t], bv1[t], acc[3]);
            }
        }
        // fixed-order sum over the waves; wave w finishes sub-tile w
#pragma unroll
        for (int j = 0; j < 4; ++j) red[w][j][lane] = acc[j];
        __syncthreads();
        f4 sum = red[0][w][lane];
        sum += red[1][w][lane];
        sum += red[2][w][lane];
        sum += red[3][w][lane];
        // lane holds gW2[o0 + 16 (w >> 1) + 4 q + r][i0 + 16 (w & 1) + l16]
        const int i = i0 + 16 * (w & 1) + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = o0 + 16 * (w >> 1) + 4 * q + r;
            if (o < a.H && i < a.H) {
                const int64_t e = zp + a.offW2 + (int64_t)o * a.H + i;
                if (a.grad) a.grad[e] = sum[r];
                if (a.params) adam_update(&a.params[e], sum[r], &a.mom[e], &a.vel[e], a.lr, a.b1, a.b2, a.eps, c1, c2);
            }
        }
        return;
    }
    const int64_t e = (int64_t)((int)blockIdx.x - ntile) * 256 + tid;
    const int64_t ns = a.PS - 1;  // the last share is the squared residuals
    if (e > ns) return;
    const float *pp = a.part + (int64_t)z * a.nblk * a.PS + e;
    float g = 0.0f;
    int b = 0;
    for (; b + 8 <= a.nblk; b += 8) {  // eight reads in flight, added in block order
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pp[(int64_t)(b + u) * a.PS];
#pragma unroll
        for (int u = 0; u < 8; ++u) g += v[u];
    }
    for (; b < a.nblk; ++b) g += pp[(int64_t)b * a.PS];
    if (e == ns) {
        if (a.loss) a.loss[z] = g / (float)a.nb;
        return;
    }
    const int64_t HW1 = (int64_t)a.H * a.n_in;
    int64_t off;
    if (e < HW1) off = e;
    else if (e < HW1 + a.H) off = a.offb1 + (e - HW1);
    else if (e < HW1 + 2 * a.H) off = a.offb2 + (e - HW1 - a.H);
    else if (e < HW1 + 3 * a.H) off = a.offW3 + (e - HW1 - 2 * a.H);
    else off = a.offb3;
    const int64_t pe = zp + off;
    if (a.grad) a.grad[pe] = g;
    if (a.params) adam_update(&a.params[pe], g, &a.mom[pe], &a.vel[pe], a.lr, a.b1, a.b2, a.eps, c1, c2);
}

// loss[z] = mean over s < n of r[z][s]^2 (one workgroup per member, fixed order).
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ r, int n, float *__restrict__ loss) {
    __shared__ float red[256];
    const int z = blockIdx.x;
    float acc = 0.0f;
    for (int s = threadIdx.x; s < n; s += 256) {
        const float v = r[(int64_t)z * n + s];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[z] = red[0] / (float)n;
}

// Adam on all n parameters from the stored gradient; the step count lives in
// device memory.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            const int64_t *__restrict__ step) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float c1, c2;
    adam_factors(step, 0, b1, b2, &c1, &c2);
    adam_update(&p[e], g[e], &m[e], &v[e], lr, b1, b2, eps, c1, c2);
}

__global__ void tick_kernel(int64_t *step, int64_t add) { *step += add; }

// x = 2 (theta - lo) / (hi - lo) - 1 (FP32) and, if logL is given,
// y = (logL - mean) / std (FP32).
__global__ void scale_kernel(const double *__restrict__ theta, const double *__restrict__ logL, int64_t N,
                             int n_in, const double *__restrict__ lo, const double *__restrict__ hi, double ymean,
                             double ystd, float *__restrict__ X, float *__restrict__ Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < N * n_in) {
        const int k = (int)(e % n_in);
        X[e] = (float)(2.0 * (theta[e] - lo[k]) / (hi[k] - lo[k]) - 1.0);
    }
    if (logL && e < N) Y[e] = (float)((logL[e] - ymean) / ystd);
}

// Ensemble statistics in logL units (FP64): mean and population spread of
// y_mean + y_std f_m over the members; with a gate, decision 1 = evaluate
// exactly, 0 = reject without an exact call (spread <= tau and mean < L_min).
__global__ void ensemble_kernel(const float *__restrict__ f, int M, int64_t nb, double ymean, double ystd,
                                double *__restrict__ mean, double *__restrict__ spread, int gate, double L_min,
                                double tau, int32_t *__restrict__ decision) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    double mu = 0.0;
    for (int z = 0; z < M; ++z) mu += ymean + ystd * (double)f[z * nb + s];
    mu /= (double)M;
    double var = 0.0;
    for (int z = 0; z < M; ++z) {
        const double d = ymean + ystd * (double)f[z * nb + s] - mu;
        var += d * d;
    }
    const double sd = sqrt(var / (double)M);
    if (mean) mean[s] = mu;
    if (spread) spread[s] = sd;
    if (gate) decision[s] = (sd <= tau && mu < L_min) ? 0 : 1;
}

// Stable compaction of the rows with keep[s] != 0, in three passes:
// per-block counts, an exclusive scan of the counts (one workgroup), and a
// scatter that scans inside each block.
constexpr int CB = 256;

__global__ __launch_bounds__(CB) void count_kernel(const int32_t *__restrict__ keep, int64_t n,
                                                   int32_t *__restrict__ counts) {
    __shared__ int red[CB];
    const int64_t s = (int64_t)blockIdx.x * CB + threadIdx.x;
    red[threadIdx.x] = (s < n && keep[s] != 0) ? 1 : 0;
    __syncthreads();
    for (int h = CB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void scan_kernel(int32_t *__restrict__ counts, int64_t nblocks,
                                                    int32_t *__restrict__ total) {
    __shared__ int carry;
    __shared__ int buf[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblocks; base += 1024) {
        const int64_t b = base + threadIdx.x;
        const int v = b < nblocks ? counts[b] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
            const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < nblocks) counts[b] = carry + buf[threadIdx.x] - v;  // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(CB) void scatter_kernel(const int32_t *__restrict__ keep, int64_t n, int n_cols,
                                                     const double *__restrict__ rows,
                                                     const int32_t *__restrict__ offsets,
                                                     double *__restrict__ rows_out, int32_t *__restrict__ index_out) {
    __shared__ int buf[CB];
    const int64_t s = (int64_t)blockIdx.x * CB + threadIdx.x;
    const int k = (s < n && keep[s] != 0) ? 1 : 0;
    buf[threadIdx.x] = k;
    __syncthreads();
    for (int off = 1; off < CB; off <<= 1) {
        const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    if (k) {
        const int64_t dst = offsets[blockIdx.x] + buf[threadIdx.x] - 1;
        if (index_out) index_out[dst] = (int32_t)s;
        if (rows_out)
            for (int c = 0; c < n_cols; ++c) rows_out[dst * n_cols + c] = rows[s * n_cols + c];
    }
}

}  // namespace

struct eor_surrogate {
    int device = 0;
    int n_in = 0, M = 0, H = 0;
    int NT = 0;   // forward: four waves of NT 16-unit tiles (width 64 NT)
    int CTB = 0;  // backward: eight waves of CTB tiles (width 128 CTB)
    int64_t P = 0;                  // parameters per member (packed layout of the API)
    int64_t PP = 0;                 // device stride of a member, P rounded up to 64
    int64_t offW1 = 0, offb1 = 0, offW2 = 0, offb2 = 0, offW3 = 0, offb3 = 0;
    double *d_lo = nullptr, *d_hi = nullptr;   // prior box
    std::vector<double> lo, hi;
    double ymean = 0.0, ystd = 1.0;
    bool trained = false;
    float *params = nullptr, *best = nullptr, *grad = nullptr, *mom = nullptr, *vel = nullptr;
    float *loss = nullptr;
    // backward-pass buffers for batches of up to cap samples
    int64_t cap = 0;
    float *H1T = nullptr, *dZ2T = nullptr, *part = nullptr;
    // forward outputs for up to f_cap samples per member
    int64_t f_cap = 0;
    float *f = nullptr;
    // training data (scaled) and indices
    int64_t data_cap = 0;
    float *X = nullptr, *Y = nullptr;
    int32_t *idx = nullptr;
    int64_t idx_cap = 0;
    uint64_t seed = 0;
    int64_t *d_step = nullptr;      // Adam step count (device)
    hipGraphExec_t epoch_exec = nullptr;  // one captured training epoch
    hipGraph_t epoch_graph = nullptr;
    int64_t epoch_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // what it was captured for
    hipStream_t cap_stream = nullptr;
    int epochs_run = 0;
    std::vector<double> best_val;
    eor::StreamOrder order;  // the last call's work on its stream
};

namespace {

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_epoch_graph(eor_surrogate &s) {
    if (s.epoch_exec) (void)hipGraphExecDestroy(s.epoch_exec);
    if (s.epoch_graph) (void)hipGraphDestroy(s.epoch_graph);
    s.epoch_exec = nullptr;
    s.epoch_graph = nullptr;
    std::memset(s.epoch_key, 0, sizeof(s.epoch_key));
}

int64_t pad16(int64_t n) { return (n + ST - 1) / ST * ST; }

// (Re)allocating any buffer a captured epoch refers to drops that graph; work
// queued by the previous call (on any stream) may still use the old buffer.
hipError_t ensure_bwd(eor_surrogate &s, int64_t nb) {
    if (s.cap >= nb) return hipSuccess;
    const hipError_t ed = s.order.drain();
    if (ed != hipSuccess) return ed;
    drop_epoch_graph(s);
    dfree(s.H1T); dfree(s.dZ2T); dfree(s.part);
    s.cap = 0;
    const int64_t nbp = pad16(nb), HP = 128 * (int64_t)s.CTB;
    const size_t hb = (size_t)s.M * HP * nbp * sizeof(float);
    hipError_t e = hipMalloc(&s.H1T, hb);
    if (e == hipSuccess) e = hipMalloc(&s.dZ2T, hb);
    if (e == hipSuccess) e = hipMalloc(&s.part, (size_t)s.M * (nbp / ST) * share_count(s.H, s.n_in) * sizeof(float));
    if (e == hipSuccess) s.cap = nb;
    return e;
}

hipError_t ensure_f(eor_surrogate &s, int64_t n) {
    if (s.f_cap >= n) return hipSuccess;
    const hipError_t ed = s.order.drain();
    if (ed != hipSuccess) return ed;
    drop_epoch_graph(s);
    dfree(s.f);
    s.f_cap = 0;
    hipError_t e = hipMalloc(&s.f, (size_t)s.M * n * sizeof(float));
    if (e == hipSuccess) s.f_cap = n;
    return e;
}

MlpArgs net_args(const eor_surrogate &s) {
    MlpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = s.params;
    a.PP = s.PP;
    a.offb1 = s.offb1;
    a.offW2 = s.offW2;
    a.offb2 = s.offb2;
    a.offW3 = s.offW3;
    a.offb3 = s.offb3;
    a.n_in = s.n_in;
    a.H = s.H;
    return a;
}

template <int NW, int RT, bool BWD>
void launch_mlp(const MlpArgs &a, int CT, int members, hipStream_t st) {
    const dim3 grid((unsigned)((a.nb + ST * RT - 1) / (ST * RT)), (unsigned)members), block(64 * NW);
    if constexpr (NW == 8) {  // widths up to 512 in tiles of 128
        switch (CT) {
        case 1: hipLaunchKernelGGL((mlp_kernel<1, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((mlp_kernel<2, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL((mlp_kernel<3, NW, RT, BWD>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((mlp_kernel<4, NW, RT, BWD>), grid, block, 0, st, a); break;
        }
    } else {                  // widths up to 512 in tiles of 64
        switch (CT) {
        case 1: hipLaunchKernelGGL((mlp_kernel<1, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((mlp_kernel<2, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL((mlp_kernel<3, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((mlp_kernel<4, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 5: hipLaunchKernelGGL((mlp_kernel<5, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 6: hipLaunchKernelGGL((mlp_kernel<6, NW, RT, BWD>), grid, block, 0, st, a); break;
        case 7: hipLaunchKernelGGL((mlp_kernel<7, NW, RT, BWD>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((mlp_kernel<8, NW, RT, BWD>), grid, block, 0, st, a); break;
        }
    }
}

// Forward pass only: four waves, 32 samples per workgroup.
void launch_forward(const MlpArgs &a, int NT, int members, hipStream_t st) {
    launch_mlp<4, 2, false>(a, NT, members, st);
}

// Loss, gradient and (with cfg) the Adam step of every member on a batch of
// nb samples described by `in` (inputs and targets; no outputs).
void train_step(eor_surrogate &s, MlpArgs in, int nb, const eor_train_cfg *cfg, int64_t step_add, bool write_grad,
                hipStream_t st) {
    const int64_t nbp = pad16(nb);
    in.nb = nb;
    in.H1T = s.H1T;
    in.dZ2T = s.dZ2T;
    in.nbp = nbp;
    in.part = s.part;
    in.PS = share_count(s.H, s.n_in);
    launch_mlp<8, 1, true>(in, s.CTB, s.M, st);
    UpdArgs u;
    std::memset(&u, 0, sizeof(u));
    u.H1T = s.H1T;
    u.dZ2T = s.dZ2T;
    u.nbp = nbp;
    u.HP = 128 * s.CTB;
    u.part = s.part;
    u.PS = in.PS;
    u.nblk = (int)(nbp / ST);
    u.H = s.H;
    u.n_in = s.n_in;
    u.nb = nb;
    u.PP = s.PP;
    u.offb1 = s.offb1;
    u.offW2 = s.offW2;
    u.offb2 = s.offb2;
    u.offW3 = s.offW3;
    u.offb3 = s.offb3;
    u.grad = write_grad ? s.grad : nullptr;
    u.loss = write_grad ? s.loss : nullptr;
    if (cfg) {
        u.params = s.params;
        u.mom = s.mom;
        u.vel = s.vel;
        u.lr = cfg->lr;
        u.b1 = cfg->beta1;
        u.b2 = cfg->beta2;
        u.eps = cfg->eps;
        u.step = s.d_step;
        u.step_add = step_add;
    }
    const int tt = u.HP / 32;
    const dim3 grid((unsigned)(tt * tt + (in.PS + 255) / 256), (unsigned)s.M);
    hipLaunchKernelGGL(mlp_update_kernel, grid, dim3(256), 0, st, u);
}

// All minibatch steps of one epoch, for capture into a graph: the indices of
// the epoch are refreshed in place before every replay; step k of the epoch
// uses Adam step count *d_step + k + 1, and the count advances once at the end.
void epoch_steps(eor_surrogate &s, const eor_train_cfg &cfg, int64_t steps, int nb, int64_t row, hipStream_t st) {
    MlpArgs in = net_args(s);
    in.X = s.X;
    in.Y = s.Y;
    in.idxz = row;
    for (int64_t k = 0; k < steps; ++k) {
        in.idx = s.idx + k * nb;
        train_step(s, in, nb, &cfg, k, false, st);
    }
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, st, s.d_step, steps);
}

void he_init(eor_surrogate &s, std::vector<float> &h) {
    h.assign((size_t)s.M * s.P, 0.0f);
    for (int z = 0; z < s.M; ++z) {
        std::mt19937_64 rng(s.seed + 7919ull * (uint64_t)z);
        std::normal_distribution<double> nd(0.0, 1.0);
        float *p = h.data() + (size_t)z * s.P;
        const double a1 = std::sqrt(2.0 / s.n_in), a2 = std::sqrt(2.0 / s.H);
        for (int64_t k = 0; k < (int64_t)s.H * s.n_in; ++k) p[s.offW1 + k] = (float)(a1 * nd(rng));
        for (int64_t k = 0; k < (int64_t)s.H * s.H; ++k) p[s.offW2 + k] = (float)(a2 * nd(rng));
        for (int64_t k = 0; k < s.H; ++k) p[s.offW3 + k] = (float)(a2 * nd(rng));
    }
}

// packed [M][P] <-> device [M][PP]
hipError_t copy_params(float *dst, int64_t dst_stride, const float *src, int64_t src_stride, const eor_surrogate &s,
                       hipMemcpyKind kind, hipStream_t st) {
    return hipMemcpy2DAsync(dst, (size_t)dst_stride * sizeof(float), src, (size_t)src_stride * sizeof(float),
                            (size_t)s.P * sizeof(float), (size_t)s.M, kind, st);
}

// Scratch of eor_surrogate_gate_noalloc: the members' outputs of one call,
// B * n_members floats at most. Every GPU the library runs on holds its own
// copy until the process ends. In host code `scratch` names a host-side
// stand-in, not the device array: host code uses the per-device address
// that hipGetSymbolAddress returns (scratch_address), never the name.
constexpr int64_t kGateScratchFloats = (int64_t)1 << 22;  // 16 MiB
static_assert(sizeof(scratch) == kGateScratchFloats * sizeof(float), "scratch size");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

eor_status need(const eor_surrogate *s) {
    if (!s) return eor::fail_status(EOR_ERR_ARG, "surrogate is NULL");
    return EOR_OK;
}

}  // namespace

extern "C" {

eor_status eor_surrogate_create(int device, int32_t n_in, int32_t n_members, int32_t hidden, uint64_t seed,
                                const double *lo, const double *hi, eor_surrogate **out) {
    if (!out) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_create: out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > NI_MAX || n_members < 1 || n_members > 64 || hidden < 4 || hidden > H_MAX ||
        hidden % 4 != 0 || !lo || !hi)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_create: need 1 <= n_in <= 64, 1 <= n_members <= 64, "
                                             "hidden a multiple of 4 in [4, 512] and a prior box");
    for (int k = 0; k < n_in; ++k)
        if (!(hi[k] > lo[k])) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_create: need hi > lo");
    eor_surrogate *s = new (std::nothrow) eor_surrogate;
    if (!s) return eor::fail_status(EOR_ERR_OOM, "eor_surrogate_create: host allocation failed");
    s->device = device;
    s->n_in = n_in;
    s->M = n_members;
    s->H = hidden;
    s->NT = (hidden + 63) / 64;
    s->CTB = (hidden + 127) / 128;
    s->seed = seed;
    s->offW1 = 0;
    s->offb1 = s->offW1 + (int64_t)hidden * n_in;
    s->offW2 = s->offb1 + hidden;
    s->offb2 = s->offW2 + (int64_t)hidden * hidden;
    s->offW3 = s->offb2 + hidden;
    s->offb3 = s->offW3 + hidden;
    s->P = s->offb3 + 1;
    s->PP = (s->P + 63) / 64 * 64;
    s->lo.assign(lo, lo + n_in);
    s->hi.assign(hi, hi + n_in);
    s->best_val.assign(n_members, 0.0);
    DevGuard dg(device);
    const size_t pb = (size_t)s->M * s->PP * sizeof(float);
    hipError_t e = hipMalloc(&s->params, pb);
    if (e == hipSuccess) e = hipMalloc(&s->best, pb);
    if (e == hipSuccess) e = hipMalloc(&s->grad, pb);
    if (e == hipSuccess) e = hipMalloc(&s->mom, pb);
    if (e == hipSuccess) e = hipMalloc(&s->vel, pb);
    if (e == hipSuccess) e = hipMalloc(&s->loss, (size_t)s->M * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&s->d_step, sizeof(int64_t));
    if (e == hipSuccess) e = hipMemset(s->d_step, 0, sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&s->d_lo, n_in * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&s->d_hi, n_in * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(s->d_lo, lo, n_in * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_hi, hi, n_in * sizeof(double), hipMemcpyHostToDevice);
    std::vector<float> h;
    he_init(*s, h);
    // the padding of every member stays zero (parameters, gradient and moments)
    if (e == hipSuccess) e = hipMemset(s->params, 0, pb);
    if (e == hipSuccess) e = hipMemset(s->grad, 0, pb);
    if (e == hipSuccess) e = hipMemset(s->mom, 0, pb);
    if (e == hipSuccess) e = hipMemset(s->vel, 0, pb);
    if (e == hipSuccess) e = copy_params(s->params, s->PP, h.data(), s->P, *s, hipMemcpyHostToDevice, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        eor_surrogate_destroy(s);
        return eor::hip_status(e, "eor_surrogate_create");
    }
    *out = s;
    return EOR_OK;
}

void eor_surrogate_destroy(eor_surrogate *s) {
    if (!s) return;
    DevGuard dg(s->device);
    (void)hipDeviceSynchronize();
    dfree(s->params); dfree(s->best); dfree(s->grad); dfree(s->mom); dfree(s->vel); dfree(s->loss);
    dfree(s->d_lo); dfree(s->d_hi);
    dfree(s->H1T); dfree(s->dZ2T); dfree(s->part); dfree(s->f);
    dfree(s->X); dfree(s->Y); dfree(s->idx); dfree(s->d_step);
    drop_epoch_graph(*s);
    s->order.destroy();
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
}

eor_status eor_surrogate_size(const eor_surrogate *s, int64_t *params_per_member, int32_t *n_members) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (params_per_member) *params_per_member = s->P;
    if (n_members) *n_members = s->M;
    return EOR_OK;
}

eor_status eor_surrogate_params(eor_surrogate *s, float *get, const float *set, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    DevGuard dg(s->device);
    const size_t pb = (size_t)s->M * s->PP * sizeof(float);
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = s->order.enter(hs);
    if (set && e == hipSuccess) {
        e = copy_params(s->params, s->PP, set, s->P, *s, hipMemcpyDeviceToDevice, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->mom, 0, pb, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->vel, 0, pb, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->d_step, 0, sizeof(int64_t), hs);
    }
    if (e == hipSuccess && get) e = copy_params(get, s->P, s->params, s->PP, *s, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = s->order.leave(hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_surrogate_params");
}

eor_status eor_surrogate_standardisation(eor_surrogate *s, double *get_mean_std, const double *set_mean_std) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (set_mean_std) {
        if (!(set_mean_std[1] > 0.0)) return eor::fail_status(EOR_ERR_ARG, "standard deviation must be > 0");
        s->ymean = set_mean_std[0];
        s->ystd = set_mean_std[1];
        s->trained = true;
    }
    if (get_mean_std) {
        get_mean_std[0] = s->ymean;
        get_mean_std[1] = s->ystd;
    }
    return EOR_OK;
}

eor_status eor_surrogate_loss_grad(eor_surrogate *s, int64_t nb, const float *x, const float *y, float *loss,
                                   float *grad, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (nb < 1 || nb > (1 << 24) || !x || !y) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_loss_grad: bad batch");
    DevGuard dg(s->device);
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = ensure_bwd(*s, nb);
    if (e == hipSuccess) e = s->order.enter(hs);
    if (e != hipSuccess) return eor::hip_status(e, "surrogate activations");
    MlpArgs in = net_args(*s);
    in.X = x;
    in.xz = nb * s->n_in;
    in.Y = y;
    in.yz = nb;
    train_step(*s, in, (int)nb, nullptr, 0, true, hs);
    if (loss) e = hipMemcpyAsync(loss, s->loss, s->M * sizeof(float), hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && grad) e = copy_params(grad, s->P, s->grad, s->PP, *s, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = s->order.leave(hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_surrogate_loss_grad");
}

eor_status eor_surrogate_adam_step(eor_surrogate *s, const eor_train_cfg *cfg, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (!cfg) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_adam_step: cfg is NULL");
    DevGuard dg(s->device);
    hipStream_t hs = (hipStream_t)stream;
    const int64_t n = (int64_t)s->M * s->PP;
    hipError_t e = s->order.enter(hs);
    if (e != hipSuccess) return eor::hip_status(e, "hipStreamWaitEvent");
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, hs, s->params, s->grad, s->mom,
                       s->vel, n, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, s->d_step);
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, hs, s->d_step, (int64_t)1);
    e = hipGetLastError();
    if (e == hipSuccess) e = s->order.leave(hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_surrogate_adam_step");
}

eor_status eor_surrogate_train(eor_surrogate *s, int64_t N, const double *theta, const double *logL,
                               const eor_train_cfg *cfg, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (!cfg || !theta || !logL || N < 8 || N > (int64_t)1 << 28)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_train: need 8 <= N <= 2^28 and non-NULL arrays");
    if (cfg->minibatch < 1 || cfg->epochs < 1 || !(cfg->val_frac >= 0.0f && cfg->val_frac < 0.9f) ||
        !(cfg->lr > 0.0f) || cfg->patience < 1)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_train: bad configuration");
    DevGuard dg(s->device);
    hipStream_t hs = (hipStream_t)stream;
    // queued work on another stream may still use the buffers rewritten here
    hipError_t e = s->order.drain();
    if (e != hipSuccess) return eor::hip_status(e, "hipEventSynchronize");
    // targets: standardise by the training values' mean and standard deviation
    std::vector<double> hy(N);
    e = hipMemcpyAsync(hy.data(), logL, N * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return eor::hip_status(e, "copy logL");
    for (double v : hy)
        if (!std::isfinite(v)) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_train: non-finite logL");
    double mu = 0.0;
    for (double v : hy) mu += v;
    mu /= (double)N;
    double var = 0.0;
    for (double v : hy) var += (v - mu) * (v - mu);
    const double sd = std::sqrt(var / (double)N);
    if (!(sd > 0.0)) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_train: logL values are all equal");
    s->ymean = mu;
    s->ystd = sd;
    if (s->data_cap < N) {
        drop_epoch_graph(*s);
        dfree(s->X);
        dfree(s->Y);
        s->data_cap = 0;
        e = hipMalloc(&s->X, (size_t)N * s->n_in * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&s->Y, (size_t)N * sizeof(float));
        if (e != hipSuccess) return eor::hip_status(e, "training data");
        s->data_cap = N;
    }
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((N * s->n_in + 255) / 256)), dim3(256), 0, hs, theta, logL, N,
                       s->n_in, s->d_lo, s->d_hi, mu, sd, s->X, s->Y);
    // split and bootstrap resamples (host RNG, seeded)
    std::mt19937_64 rng(cfg->seed);
    std::vector<int32_t> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    const int64_t n_val = std::max<int64_t>(cfg->val_frac > 0.0f ? 1 : 0, (int64_t)(cfg->val_frac * (double)N));
    const int64_t n_tr = N - n_val;
    const int nb = (int)std::min<int64_t>(cfg->minibatch, n_tr);
    const int64_t steps = std::max<int64_t>(1, n_tr / nb);
    std::vector<std::vector<int32_t>> boot(s->M, std::vector<int32_t>(n_tr));
    for (int z = 0; z < s->M; ++z) {
        std::uniform_int_distribution<int64_t> u(0, n_tr - 1);
        for (int64_t k = 0; k < n_tr; ++k) boot[z][k] = perm[n_val + u(rng)];
    }
    // one row of indices per member: an epoch's shuffled bootstrap sample, then the validation set
    const int64_t row = n_tr + n_val;
    if (s->idx_cap < s->M * row) {
        drop_epoch_graph(*s);
        dfree(s->idx);
        s->idx_cap = 0;
        e = hipMalloc(&s->idx, (size_t)s->M * row * sizeof(int32_t));
        if (e != hipSuccess) return eor::hip_status(e, "index buffer");
        s->idx_cap = s->M * row;
    }
    e = ensure_bwd(*s, nb);
    if (e == hipSuccess) e = ensure_f(*s, std::max<int64_t>(1, n_val));
    if (e != hipSuccess) return eor::hip_status(e, "surrogate activations");
    std::vector<int32_t> hidx((size_t)s->M * row);
    std::vector<float> hloss(s->M);
    std::vector<double> best(s->M, INFINITY);
    std::vector<int> since(s->M, 0);
    const size_t pb = (size_t)s->M * s->PP * sizeof(float);
    e = hipMemcpyAsync(s->best, s->params, pb, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return eor::hip_status(e, "best parameters");
    MlpArgs val = net_args(*s);
    val.X = s->X;
    val.Y = s->Y;
    val.idx = s->idx + n_tr;
    val.idxz = row;
    val.nb = (int)n_val;
    val.f = s->f;
    val.fz = n_val;
    // the graph bakes in the shapes and the optimiser's constants
    int64_t key[8] = {steps, nb, row, n_tr, 0, 0, 0, 0};
    std::memcpy(&key[4], &cfg->lr, sizeof(float));
    std::memcpy(&key[5], &cfg->beta1, sizeof(float));
    std::memcpy(&key[6], &cfg->beta2, sizeof(float));
    std::memcpy(&key[7], &cfg->eps, sizeof(float));
    int ep = 0;
    for (ep = 0; ep < cfg->epochs; ++ep) {
        for (int z = 0; z < s->M; ++z) {
            std::shuffle(boot[z].begin(), boot[z].end(), rng);
            std::copy(boot[z].begin(), boot[z].end(), hidx.begin() + (size_t)z * row);
            std::copy(perm.begin(), perm.begin() + n_val, hidx.begin() + (size_t)z * row + n_tr);
        }
        e = hipMemcpyAsync(s->idx, hidx.data(), hidx.size() * sizeof(int32_t), hipMemcpyHostToDevice, hs);
        if (e != hipSuccess) return eor::hip_status(e, "indices");
        if (!s->epoch_exec || std::memcmp(key, s->epoch_key, sizeof(key)) != 0) {
            drop_epoch_graph(*s);
            if (!s->cap_stream) {
                e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return eor::hip_status(e, "capture stream");
            }
            e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return eor::hip_status(e, "hipStreamBeginCapture");
            epoch_steps(*s, *cfg, steps, nb, row, s->cap_stream);
            e = hipStreamEndCapture(s->cap_stream, &s->epoch_graph);
            if (e == hipSuccess) e = hipGraphInstantiate(&s->epoch_exec, s->epoch_graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_epoch_graph(*s);
                return eor::hip_status(e, "epoch graph");
            }
            std::memcpy(s->epoch_key, key, sizeof(key));
        }
        e = hipGraphLaunch(s->epoch_exec, hs);
        if (e != hipSuccess) return eor::hip_status(e, "epoch replay");
        // hidx is overwritten for the next epoch only after this epoch ran
        if (n_val == 0) {
            e = hipStreamSynchronize(hs);
            if (e != hipSuccess) return eor::hip_status(e, "epoch");
            continue;
        }
        // validation loss of every member: residuals, then their mean square
        launch_forward(val, s->NT, s->M, hs);
        hipLaunchKernelGGL(loss_kernel, dim3((unsigned)s->M), dim3(256), 0, hs, s->f, (int)n_val, s->loss);
        e = hipMemcpyAsync(hloss.data(), s->loss, s->M * sizeof(float), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return eor::hip_status(e, "validation loss");
        bool any = false;
        for (int z = 0; z < s->M; ++z) {
            if (hloss[z] < best[z]) {
                best[z] = hloss[z];
                since[z] = 0;
                e = hipMemcpyAsync(s->best + (size_t)z * s->PP, s->params + (size_t)z * s->PP, s->PP * sizeof(float),
                                   hipMemcpyDeviceToDevice, hs);
                if (e != hipSuccess) return eor::hip_status(e, "best parameters");
            } else {
                ++since[z];
            }
            if (since[z] < cfg->patience) any = true;
        }
        if (!any) {
            ++ep;
            break;
        }
    }
    if (n_val > 0) {
        e = hipMemcpyAsync(s->params, s->best, pb, hipMemcpyDeviceToDevice, hs);
        if (e != hipSuccess) return eor::hip_status(e, "restore best");
    }
    e = hipStreamSynchronize(hs);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = s->order.leave(hs);
    if (e != hipSuccess) return eor::hip_status(e, "eor_surrogate_train");
    s->epochs_run = ep;
    for (int z = 0; z < s->M; ++z) s->best_val[z] = n_val > 0 ? best[z] : NAN;
    s->trained = true;
    return EOR_OK;
}

eor_status eor_surrogate_report(const eor_surrogate *s, int32_t *epochs_run, double *val_loss) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (epochs_run) *epochs_run = s->epochs_run;
    if (val_loss)
        for (int z = 0; z < s->M; ++z) val_loss[z] = s->best_val[z];
    return EOR_OK;
}

eor_status eor_surrogate_gate_noalloc(eor_surrogate *s, int64_t B, const double *theta, double L_min, double tau,
                                      double *mean, double *spread, float *members, int32_t *decision,
                                      void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (!s->trained) return eor::fail_status(EOR_ERR_STATE, "surrogate: train it (or set its standardisation) first");
    if (B < 0 || (B > 0 && !theta)) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_gate_noalloc: bad batch");
    if (B > kGateScratchFloats / s->M)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_gate_noalloc: B x n_members exceeds the fixed scratch of "
                                             "2^22 floats (B <= " + std::to_string(kGateScratchFloats / s->M) + ")");
    if (B == 0) return EOR_OK;
    if (s->device < 0 || s->device >= kMaxDevices)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_gate_noalloc: device index beyond 63");
    DevGuard dg(s->device);
    float *f = nullptr;
    {
        // Set-up, once per device with that device current: the device
        // address of this GPU's copy of the scratch array.
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_dev[s->device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return eor::hip_status(e, "hipGetSymbolAddress(scratch)");
            g_scratch_dev[s->device] = (float *)p;
        }
        f = g_scratch_dev[s->device];
    }
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = s->order.enter(hs);
    if (e != hipSuccess) return eor::hip_status(e, "hipStreamWaitEvent");
    MlpArgs in = net_args(*s);
    in.theta = theta;
    in.lo = s->d_lo;
    in.hi = s->d_hi;
    in.nb = (int)B;
    in.f = f;  // written for every (member, sample) of this call before it is read
    in.fz = B;
    launch_forward(in, s->NT, s->M, hs);
    if (members) {
        e = hipMemcpyAsync(members, f, (size_t)s->M * B * sizeof(float), hipMemcpyDeviceToDevice, hs);
        if (e != hipSuccess) return eor::hip_status(e, "member outputs");
    }
    hipLaunchKernelGGL(ensemble_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, hs, f, s->M, B, s->ymean,
                       s->ystd, mean, spread, decision ? 1 : 0, L_min, tau, decision);
    e = hipGetLastError();
    // The event that orders this handle's calls is created by an earlier
    // call (training); this call only records it, which allocates nothing.
    if (e == hipSuccess && s->order.ev) e = s->order.leave(hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_surrogate_gate_noalloc");
}

eor_status eor_surrogate_infer(eor_surrogate *s, int64_t B, const double *theta, double *mean, double *spread,
                               float *members, void *stream) {
    return eor_surrogate_gate(s, B, theta, 0.0, -1.0, mean, spread, members, nullptr, stream);
}

eor_status eor_surrogate_gate(eor_surrogate *s, int64_t B, const double *theta, double L_min, double tau,
                              double *mean, double *spread, float *members, int32_t *decision, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (!s->trained) return eor::fail_status(EOR_ERR_STATE, "surrogate: train it (or set its standardisation) first");
    if (B < 0 || B > (int64_t)1 << 30 || (B > 0 && !theta))
        return eor::fail_status(EOR_ERR_ARG, "surrogate: bad batch");
    if (B == 0) return EOR_OK;
    DevGuard dg(s->device);
    hipStream_t hs = (hipStream_t)stream;
    const int64_t chunk = (int64_t)1 << 20;
    hipError_t e = ensure_f(*s, std::min<int64_t>(B, chunk));
    if (e == hipSuccess) e = s->order.enter(hs);
    if (e != hipSuccess) return eor::hip_status(e, "surrogate outputs");
    for (int64_t c0 = 0; c0 < B; c0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - c0);
        // shared inputs for all members, scaled on the fly
        MlpArgs in = net_args(*s);
        in.theta = theta + c0 * s->n_in;
        in.lo = s->d_lo;
        in.hi = s->d_hi;
        in.nb = nb;
        in.f = s->f;
        in.fz = nb;
        launch_forward(in, s->NT, s->M, hs);
        if (members)
            for (int z = 0; z < s->M; ++z) {
                e = hipMemcpyAsync(members + (size_t)z * B + c0, s->f + (size_t)z * nb, nb * sizeof(float),
                                   hipMemcpyDeviceToDevice, hs);
                if (e != hipSuccess) return eor::hip_status(e, "member outputs");
            }
        hipLaunchKernelGGL(ensemble_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, hs, s->f, s->M,
                           (int64_t)nb, s->ymean, s->ystd, mean ? mean + c0 : nullptr, spread ? spread + c0 : nullptr,
                           decision ? 1 : 0, L_min, tau, decision ? decision + c0 : nullptr);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = s->order.leave(hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "surrogate inference");
}

eor_status eor_compact_rows(int64_t n, int32_t n_cols, const int32_t *keep, const double *rows, double *rows_out,
                            int32_t *index_out, int32_t *count_out, void *stream) {
    if (n < 0 || n > (int64_t)1 << 30 || n_cols < 0 || !keep || !count_out || (n_cols > 0 && rows_out && !rows))
        return eor::fail_status(EOR_ERR_ARG, "eor_compact_rows: bad arguments");
    hipStream_t hs = (hipStream_t)stream;
    const int64_t nblocks = std::max<int64_t>(1, (n + CB - 1) / CB);
    int32_t *counts = nullptr;
    hipError_t e = hipMallocAsync((void **)&counts, nblocks * sizeof(int32_t), hs);
    if (e != hipSuccess) return eor::hip_status(e, "eor_compact_rows scratch");
    if (n > 0) hipLaunchKernelGGL(count_kernel, dim3((unsigned)nblocks), dim3(CB), 0, hs, keep, n, counts);
    else (void)hipMemsetAsync(counts, 0, sizeof(int32_t), hs);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, hs, counts, nblocks, count_out);
    if (n > 0)
        hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nblocks), dim3(CB), 0, hs, keep, n, n_cols, rows, counts,
                           rows_out, index_out);
    e = hipGetLastError();
    (void)hipFreeAsync(counts, hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_compact_rows");
}

}  // extern "C"
