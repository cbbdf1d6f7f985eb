// Learned surrogate of logL(theta): an ensemble of small fully connected
// networks n_in -> H -> H -> 1 with GELU after each hidden layer, in FP32,
// trained on exact evaluations by these kernels (forward, hand-derived
// backward, Adam) and used to gate sampler proposals, with the exact FP64
// likelihood as the fallback and as the judge of every accepted point.
//
// Layout per member (flat FP32, row-major matrices):
//   W1 [H x n_in], b1 [H], W2 [H x H], b2 [H], W3 [H], b3 [1]
// Members are stored one after another (stride P = number of parameters).
// Inputs are theta mapped from the prior box to [-1, 1]; targets are logL
// standardised by the training mean and standard deviation.
//
// The dense layers and the weight gradients are one batched GEMM kernel on
// FP32 MFMA (16x16x4): a 64 x 64 output tile per workgroup, operand tiles of
// 16 k staged in LDS with coalesced loads whatever the operand strides.
// Every reduction (loss, biases, output layer) has a fixed order, so
// training is deterministic for a given seed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "common.h"

namespace {

using eor::f4;

__device__ inline f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C[z][i][j] = sum_k A[z][i][k] B[z][k][j]  (+ bias[z][j]) (GELU), with
// A[z][i][k] at A + z sAz + i sai + k sak and B[z][k][j] at B + z sBz + k sbk + j sbj.
struct GemmArgs {
    const float *A;
    int64_t sai, sak, sAz;
    const float *B;
    int64_t sbk, sbj, sBz;
    float *C;
    int64_t ldc, sCz;
    float *Z;              // pre-activation output (epilogue 2), same layout as C
    const float *bias;     // [z][j]
    int64_t sbiasz;
    int M, N, K;
    int epi;               // 0: AB; 1: AB + bias; 2: Z = AB + bias, C = GELU(Z)
};

constexpr int GT = 64;  // output tile
constexpr int GK = 16;  // k per LDS stage

__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    __shared__ float As[GK][GT];
    __shared__ float Bs[GK][GT];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    const int64_t z = blockIdx.z;
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    const float *A = g.A + z * g.sAz;
    const float *B = g.B + z * g.sBz;
    f4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = f4{0, 0, 0, 0};
    const bool a_kcontig = g.sak == 1;
    const bool b_jcontig = g.sbj == 1;
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        // stage the operand tiles; consecutive threads walk the unit-stride dimension
        for (int e = tid; e < GK * GT; e += 256) {
            int i, kk;
            if (a_kcontig) { i = e / GK; kk = e % GK; } else { i = e % GT; kk = e / GT; }
            const int gi = i0 + i, gk = k0 + kk;
            As[kk][i] = (gi < g.M && gk < g.K) ? A[gi * g.sai + gk * g.sak] : 0.0f;
            int j, kb;
            if (b_jcontig) { j = e % GT; kb = e / GT; } else { j = e / GK; kb = e % GK; }
            const int gj = j0 + j, gkb = k0 + kb;
            Bs[kb][j] = (gj < g.N && gkb < g.K) ? B[gkb * g.sbk + gj * g.sbj] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const float a = As[ks + q][16 * w + l16];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma32(a, Bs[ks + q][16 * cb + l16], acc[cb]);
        }
        __syncthreads();
    }
    // lane holds D[16w + 4q + r][16cb + l16]
    float *C = g.C + z * g.sCz;
    float *Zp = g.Z ? g.Z + z * g.sCz : nullptr;
    const float *bias = g.bias ? g.bias + z * g.sbiasz : nullptr;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int j = j0 + 16 * cb + l16;
        if (j >= g.N) continue;
        const float bj = (g.epi >= 1) ? bias[j] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * w + 4 * q + r;
            if (i >= g.M) continue;
            const float v = acc[cb][r] + bj;
            if (g.epi == 2) {
                Zp[(int64_t)i * g.ldc + j] = v;
                C[(int64_t)i * g.ldc + j] = gelu_f(v);
            } else {
                C[(int64_t)i * g.ldc + j] = v;
            }
        }
    }
}

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

// Xb[z][s][:] = X[idx[z][s]][:], Yb[z][s] = Y[idx[z][s]] for s < nb.
__global__ void gather_kernel(const float *__restrict__ X, const float *__restrict__ Y, int n_in,
                              const int32_t *__restrict__ idx, int64_t idx_stride, int nb,
                              float *__restrict__ Xb, float *__restrict__ Yb) {
    const int z = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * n_in) return;
    const int s = e / n_in, k = e % n_in;
    const int32_t src = idx[z * idx_stride + s];
    Xb[((int64_t)z * nb + s) * n_in + k] = X[(int64_t)src * n_in + k];
    if (k == 0) Yb[(int64_t)z * nb + s] = Y[src];
}

// f[z][s] = sum_k H2[z][s][k] W3[z][k] + b3[z]: one wave per (z, s), lanes
// over k, fixed shuffle tree.
__global__ void out_fwd_kernel(const float *__restrict__ H2, int64_t sHz, int H, const float *__restrict__ params,
                               int64_t P, int64_t offW3, int nb, float *__restrict__ f) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int z = blockIdx.y;
    if (wave >= nb) return;
    const float *h = H2 + z * sHz + (int64_t)wave * H;
    const float *W3 = params + z * P + offW3;
    float s = 0.0f;
    for (int k = lane; k < H; k += 64) s += h[k] * W3[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) f[(int64_t)z * nb + wave] = s + W3[H];  // b3 follows W3
}

// Per member: r = f - y, dF = 2 r / nb, loss = mean r^2 (one workgroup per member).
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ f, const float *__restrict__ y, int nb,
                                                   float *__restrict__ dF, float *__restrict__ loss) {
    __shared__ float red[256];
    const int z = blockIdx.x;
    float acc = 0.0f;
    for (int s = threadIdx.x; s < nb; s += 256) {
        const float r = f[(int64_t)z * nb + s] - y[(int64_t)z * nb + s];
        if (dF) dF[(int64_t)z * nb + s] = 2.0f * r / (float)nb;
        acc += r * r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[z] = red[0] / (float)nb;
}

// Output layer backward: gW3[k] = sum_s dF[s] H2[s][k], gb3 = sum_s dF[s];
// dZ2[s][k] = dF[s] W3[k] gelu'(Z2[s][k]).
__global__ void out_bwd_kernel(const float *__restrict__ dF, const float *__restrict__ H2,
                               const float *__restrict__ Z2, int64_t sHz, int H, const float *__restrict__ params,
                               float *__restrict__ grad, int64_t P, int64_t offW3, int nb, float *__restrict__ dZ2) {
    const int z = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const float *W3 = params + z * P + offW3;
    if (k < H) {
        float s = 0.0f;
        for (int t = 0; t < nb; ++t) s += dF[(int64_t)z * nb + t] * H2[z * sHz + (int64_t)t * H + k];
        grad[z * P + offW3 + k] = s;
        const float w3 = W3[k];
        for (int t = 0; t < nb; ++t) {
            const int64_t o = z * sHz + (int64_t)t * H + k;
            dZ2[o] = dF[(int64_t)z * nb + t] * w3 * gelu_grad_f(Z2[o]);
        }
    } else if (k == H) {
        float s = 0.0f;
        for (int t = 0; t < nb; ++t) s += dF[(int64_t)z * nb + t];
        grad[z * P + offW3 + H] = s;
    }
}

// dZ = dH * gelu'(Z), elementwise over [members][nb][H].
__global__ void gelu_bwd_kernel(const float *__restrict__ dH, const float *__restrict__ Z, int64_t n,
                                float *__restrict__ dZ) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dZ[e] = dH[e] * gelu_grad_f(Z[e]);
}

// grad[z][off + k] = sum_s dZ[z][s][k] (bias gradient).
__global__ void colsum_kernel(const float *__restrict__ dZ, int64_t sHz, int H, int nb, float *__restrict__ grad,
                              int64_t P, int64_t off) {
    const int z = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= H) return;
    float s = 0.0f;
    for (int t = 0; t < nb; ++t) s += dZ[z * sHz + (int64_t)t * H + k];
    grad[z * P + off + k] = s;
}

// Adam with bias-corrected moments: step t = *step + 1 (the counter lives
// in device memory so that a captured epoch can be replayed unchanged),
// c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            const int64_t *__restrict__ step) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double t = (double)(*step + 1);
    const float c1 = (float)(1.0 - pow((double)b1, t));
    const float c2 = (float)(1.0 - pow((double)b2, t));
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

__global__ void tick_kernel(int64_t *step) { *step += 1; }

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
    int64_t P = 0;                  // parameters per member
    int64_t offW1 = 0, offb1 = 0, offW2 = 0, offb2 = 0, offW3 = 0, offb3 = 0;
    double *d_lo = nullptr, *d_hi = nullptr;   // prior box
    std::vector<double> lo, hi;
    double ymean = 0.0, ystd = 1.0;
    bool trained = false;
    float *params = nullptr, *best = nullptr, *grad = nullptr, *mom = nullptr, *vel = nullptr;
    // activations for up to cap samples per member
    int64_t cap = 0;
    float *Xb = nullptr, *Yb = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr;
    float *dZ = nullptr, *dH = nullptr, *f = nullptr, *dF = nullptr, *loss = nullptr;
    // training data (scaled) and indices
    int64_t data_cap = 0;
    float *X = nullptr, *Y = nullptr;
    int32_t *idx = nullptr;
    int64_t idx_cap = 0;
    int32_t *d_counts = nullptr;
    int64_t counts_cap = 0;
    uint64_t seed = 0;
    int64_t *d_step = nullptr;      // Adam step count (device)
    hipGraphExec_t epoch_exec = nullptr;  // one captured training epoch
    hipGraph_t epoch_graph = nullptr;
    int64_t epoch_key[4] = {0, 0, 0, 0};  // (steps, nb, row, n_tr) it was captured for
    hipStream_t cap_stream = nullptr;
    int epochs_run = 0;
    std::vector<double> best_val;
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

// (Re)allocating any buffer a captured epoch refers to drops that graph.
hipError_t ensure_act(eor_surrogate &s, int64_t nb) {
    if (s.cap >= nb) return hipSuccess;
    drop_epoch_graph(s);
    dfree(s.Xb); dfree(s.Yb); dfree(s.Z1); dfree(s.H1); dfree(s.Z2); dfree(s.H2);
    dfree(s.dZ); dfree(s.dH); dfree(s.f); dfree(s.dF);
    s.cap = 0;
    const size_t hm = (size_t)s.M * nb * s.H * sizeof(float);
    hipError_t e = hipMalloc(&s.Xb, (size_t)s.M * nb * s.n_in * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&s.Yb, (size_t)s.M * nb * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&s.Z1, hm);
    if (e == hipSuccess) e = hipMalloc(&s.H1, hm);
    if (e == hipSuccess) e = hipMalloc(&s.Z2, hm);
    if (e == hipSuccess) e = hipMalloc(&s.H2, hm);
    if (e == hipSuccess) e = hipMalloc(&s.dZ, hm);
    if (e == hipSuccess) e = hipMalloc(&s.dH, hm);
    if (e == hipSuccess) e = hipMalloc(&s.f, (size_t)s.M * nb * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&s.dF, (size_t)s.M * nb * sizeof(float));
    if (e == hipSuccess) s.cap = nb;
    return e;
}

void launch_gemm(const GemmArgs &g, int members, hipStream_t st) {
    dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT), (unsigned)members);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, st, g);
}

// Forward pass of all members on Xb [M][nb][n_in] (per-member inputs when
// xz_stride != 0, shared inputs when 0): Z1, H1, Z2, H2, f.
void forward(eor_surrogate &s, const float *Xin, int64_t xz_stride, int nb, hipStream_t st) {
    const int64_t sHz = (int64_t)nb * s.H;
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    // layer 1: Z1[s][h] = sum_k X[s][k] W1[h][k] + b1[h]
    g.A = Xin; g.sai = s.n_in; g.sak = 1; g.sAz = xz_stride;
    g.B = s.params + s.offW1; g.sbk = 1; g.sbj = s.n_in; g.sBz = s.P;
    g.C = s.H1; g.Z = s.Z1; g.ldc = s.H; g.sCz = sHz;
    g.bias = s.params + s.offb1; g.sbiasz = s.P;
    g.M = nb; g.N = s.H; g.K = s.n_in; g.epi = 2;
    launch_gemm(g, s.M, st);
    // layer 2: Z2[s][h] = sum_k H1[s][k] W2[h][k] + b2[h]
    g.A = s.H1; g.sai = s.H; g.sak = 1; g.sAz = sHz;
    g.B = s.params + s.offW2; g.sbk = 1; g.sbj = s.H; g.sBz = s.P;
    g.C = s.H2; g.Z = s.Z2;
    g.bias = s.params + s.offb2;
    g.K = s.H;
    launch_gemm(g, s.M, st);
    // output layer
    const int waves_per_block = 4;
    hipLaunchKernelGGL(out_fwd_kernel, dim3((unsigned)((nb + waves_per_block - 1) / waves_per_block), (unsigned)s.M),
                       dim3(64 * waves_per_block), 0, st, s.H2, sHz, s.H, s.params, s.P, s.offW3, nb, s.f);
}

// Loss and gradient of every member on its own batch Xb, Yb (nb samples).
void backward(eor_surrogate &s, int nb, hipStream_t st) {
    const int64_t sHz = (int64_t)nb * s.H;
    hipLaunchKernelGGL(loss_kernel, dim3((unsigned)s.M), dim3(256), 0, st, s.f, s.Yb, nb, s.dF, s.loss);
    hipLaunchKernelGGL(out_bwd_kernel, dim3((unsigned)((s.H + 1 + 255) / 256), (unsigned)s.M), dim3(256), 0, st,
                       s.dF, s.H2, s.Z2, sHz, s.H, s.params, s.grad, s.P, s.offW3, nb, s.dZ);
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    // gW2[o][i] = sum_s dZ2[s][o] H1[s][i]
    g.A = s.dZ; g.sai = 1; g.sak = s.H; g.sAz = sHz;
    g.B = s.H1; g.sbk = s.H; g.sbj = 1; g.sBz = sHz;
    g.C = s.grad + s.offW2; g.ldc = s.H; g.sCz = s.P;
    g.M = s.H; g.N = s.H; g.K = nb; g.epi = 0;
    launch_gemm(g, s.M, st);
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((s.H + 255) / 256), (unsigned)s.M), dim3(256), 0, st, s.dZ,
                       sHz, s.H, nb, s.grad, s.P, s.offb2);
    // dH1[s][i] = sum_o dZ2[s][o] W2[o][i]
    g.A = s.dZ; g.sai = s.H; g.sak = 1; g.sAz = sHz;
    g.B = s.params + s.offW2; g.sbk = s.H; g.sbj = 1; g.sBz = s.P;
    g.C = s.dH; g.ldc = s.H; g.sCz = sHz;
    g.M = nb; g.N = s.H; g.K = s.H;
    launch_gemm(g, s.M, st);
    const int64_t nact = (int64_t)s.M * sHz;
    hipLaunchKernelGGL(gelu_bwd_kernel, dim3((unsigned)((nact + 255) / 256)), dim3(256), 0, st, s.dH, s.Z1, nact,
                       s.dZ);
    // gW1[h][k] = sum_s dZ1[s][h] X[s][k]
    g.A = s.dZ; g.sai = 1; g.sak = s.H; g.sAz = sHz;
    g.B = s.Xb; g.sbk = s.n_in; g.sbj = 1; g.sBz = (int64_t)nb * s.n_in;
    g.C = s.grad + s.offW1; g.ldc = s.n_in; g.sCz = s.P;
    g.M = s.H; g.N = s.n_in; g.K = nb;
    launch_gemm(g, s.M, st);
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((s.H + 255) / 256), (unsigned)s.M), dim3(256), 0, st, s.dZ,
                       sHz, s.H, nb, s.grad, s.P, s.offb1);
}

void adam(eor_surrogate &s, const eor_train_cfg &cfg, hipStream_t st) {
    const int64_t n = (int64_t)s.M * s.P;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.params, s.grad, s.mom,
                       s.vel, n, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, s.d_step);
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, st, s.d_step);
}

// All minibatch steps of one epoch (gather, forward, backward, Adam), for
// capture into a graph: the indices of the epoch are refreshed in place
// before every replay, and the Adam step count is read from device memory.
void epoch_steps(eor_surrogate &s, const eor_train_cfg &cfg, int64_t steps, int nb, int64_t row,
                 hipStream_t st) {
    for (int64_t k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nb * s.n_in + 255) / 256), (unsigned)s.M), dim3(256), 0,
                           st, s.X, s.Y, s.n_in, s.idx + k * nb, row, nb, s.Xb, s.Yb);
        forward(s, s.Xb, (int64_t)nb * s.n_in, nb, st);
        backward(s, nb, st);
        adam(s, cfg, st);
    }
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
    if (n_in < 1 || n_in > 1024 || n_members < 1 || n_members > 64 || hidden < 1 || hidden > 4096 || !lo || !hi)
        return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_create: bad sizes or NULL prior box");
    for (int k = 0; k < n_in; ++k)
        if (!(hi[k] > lo[k])) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_create: need hi > lo");
    eor_surrogate *s = new (std::nothrow) eor_surrogate;
    if (!s) return eor::fail_status(EOR_ERR_OOM, "eor_surrogate_create: host allocation failed");
    s->device = device;
    s->n_in = n_in;
    s->M = n_members;
    s->H = hidden;
    s->seed = seed;
    s->offW1 = 0;
    s->offb1 = s->offW1 + (int64_t)hidden * n_in;
    s->offW2 = s->offb1 + hidden;
    s->offb2 = s->offW2 + (int64_t)hidden * hidden;
    s->offW3 = s->offb2 + hidden;
    s->offb3 = s->offW3 + hidden;
    s->P = s->offb3 + 1;
    s->lo.assign(lo, lo + n_in);
    s->hi.assign(hi, hi + n_in);
    s->best_val.assign(n_members, 0.0);
    DevGuard dg(device);
    const size_t pb = (size_t)s->M * s->P * sizeof(float);
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
    if (e == hipSuccess) e = hipMemcpy(s->params, h.data(), pb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->mom, 0, pb);
    if (e == hipSuccess) e = hipMemset(s->vel, 0, pb);
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
    dfree(s->Xb); dfree(s->Yb); dfree(s->Z1); dfree(s->H1); dfree(s->Z2); dfree(s->H2);
    dfree(s->dZ); dfree(s->dH); dfree(s->f); dfree(s->dF);
    dfree(s->X); dfree(s->Y); dfree(s->idx); dfree(s->d_counts); dfree(s->d_step);
    drop_epoch_graph(*s);
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
    const size_t pb = (size_t)s->M * s->P * sizeof(float);
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (set) {
        e = hipMemcpyAsync(s->params, set, pb, hipMemcpyDeviceToDevice, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->mom, 0, pb, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->vel, 0, pb, hs);
        if (e == hipSuccess) e = hipMemsetAsync(s->d_step, 0, sizeof(int64_t), hs);
    }
    if (e == hipSuccess && get) e = hipMemcpyAsync(get, s->params, pb, hipMemcpyDeviceToDevice, hs);
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
    hipError_t e = ensure_act(*s, nb);
    if (e != hipSuccess) return eor::hip_status(e, "surrogate activations");
    const size_t xb = (size_t)s->M * nb * s->n_in * sizeof(float), yb = (size_t)s->M * nb * sizeof(float);
    e = hipMemcpyAsync(s->Xb, x, xb, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(s->Yb, y, yb, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return eor::hip_status(e, "surrogate inputs");
    forward(*s, s->Xb, (int64_t)nb * s->n_in, (int)nb, hs);
    backward(*s, (int)nb, hs);
    if (loss) e = hipMemcpyAsync(loss, s->loss, s->M * sizeof(float), hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && grad)
        e = hipMemcpyAsync(grad, s->grad, (size_t)s->M * s->P * sizeof(float), hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_surrogate_loss_grad");
}

eor_status eor_surrogate_adam_step(eor_surrogate *s, const eor_train_cfg *cfg, void *stream) {
    eor_status st = need(s);
    if (st != EOR_OK) return st;
    if (!cfg) return eor::fail_status(EOR_ERR_ARG, "eor_surrogate_adam_step: cfg is NULL");
    DevGuard dg(s->device);
    adam(*s, *cfg, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
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
    // targets: standardise by the training values' mean and standard deviation
    std::vector<double> hy(N);
    hipError_t e = hipMemcpyAsync(hy.data(), logL, N * sizeof(double), hipMemcpyDeviceToHost, hs);
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
    e = ensure_act(*s, std::max<int64_t>(nb, n_val));
    if (e != hipSuccess) return eor::hip_status(e, "surrogate activations");
    std::vector<int32_t> hidx((size_t)s->M * row);
    std::vector<float> hloss(s->M);
    std::vector<double> best(s->M, INFINITY);
    std::vector<int> since(s->M, 0);
    const size_t pb = (size_t)s->M * s->P * sizeof(float);
    e = hipMemcpyAsync(s->best, s->params, pb, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return eor::hip_status(e, "best parameters");
    int ep = 0;
    for (ep = 0; ep < cfg->epochs; ++ep) {
        for (int z = 0; z < s->M; ++z) {
            std::shuffle(boot[z].begin(), boot[z].end(), rng);
            std::copy(boot[z].begin(), boot[z].end(), hidx.begin() + (size_t)z * row);
            std::copy(perm.begin(), perm.begin() + n_val, hidx.begin() + (size_t)z * row + n_tr);
        }
        e = hipMemcpyAsync(s->idx, hidx.data(), hidx.size() * sizeof(int32_t), hipMemcpyHostToDevice, hs);
        if (e != hipSuccess) return eor::hip_status(e, "indices");
        const int64_t key[4] = {steps, nb, row, n_tr};
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
        }
        if (n_val == 0) continue;
        // validation loss of every member
        hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n_val * s->n_in + 255) / 256), (unsigned)s->M), dim3(256),
                           0, hs, s->X, s->Y, s->n_in, s->idx + n_tr, row, (int)n_val, s->Xb, s->Yb);
        forward(*s, s->Xb, n_val * s->n_in, (int)n_val, hs);
        hipLaunchKernelGGL(loss_kernel, dim3((unsigned)s->M), dim3(256), 0, hs, s->f, s->Yb, (int)n_val, nullptr,
                           s->loss);
        e = hipMemcpyAsync(hloss.data(), s->loss, s->M * sizeof(float), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return eor::hip_status(e, "validation loss");
        bool any = false;
        for (int z = 0; z < s->M; ++z) {
            if (hloss[z] < best[z]) {
                best[z] = hloss[z];
                since[z] = 0;
                e = hipMemcpyAsync(s->best + (size_t)z * s->P, s->params + (size_t)z * s->P, s->P * sizeof(float),
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
    const int64_t chunk = 65536;
    hipError_t e = ensure_act(*s, std::min<int64_t>(B, chunk));
    if (e != hipSuccess) return eor::hip_status(e, "surrogate activations");
    for (int64_t c0 = 0; c0 < B; c0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - c0);
        // shared inputs for all members
        hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((nb * s->n_in + 255) / 256)), dim3(256), 0, hs,
                           theta + c0 * s->n_in, nullptr, (int64_t)nb, s->n_in, s->d_lo, s->d_hi, 0.0, 1.0, s->Xb,
                           nullptr);
        forward(*s, s->Xb, 0, nb, hs);
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
