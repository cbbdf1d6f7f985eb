// Instrument forward model: the dense matrix T that takes the model's
// coefficients (a Fourier-domain sky cube) to visibilities, from the uv
// sampling, the primary beam and the model's basis (the instrument model of
// the paper's "Running BayesEoR" section; the paper gives no formula, the
// visibility equation used is stated with eor_forward_model).
//
// For channel f, G_f[b][k] = sum_p E_f[b][p] B_f[p][k] with
//   E_f[b][p] = exp(-2 pi i nu_f / c (x_b l_p + y_b m_p))   (made in LDS),
//   B_f[p][k] = A[f][p] S[p][k],  S[p][k] = exp(2 pi i (u_k l_p + v_k m_p))
// (S does not depend on the channel: a small kernel writes it once). The
// product runs on FP64 MFMA, three real 16x16x4 products per complex step
// (Gauss); each workgroup forms a 32 x 128 tile of G_f (32 baselines, so
// that each phase factor E_f[b][p] is made once for up to 128 uv cells) and
// its epilogue writes T[f n_bl + b][e n_uv + k] = norm Z[f][e] G_f[b][k] for
// every spectral mode e.
#include <cmath>

#include "common.h"

namespace eor {

namespace {

constexpr double C_LIGHT = 299792458.0;  // m / s
constexpr int FB = 32;                   // tile: 32 baselines ...
constexpr int FU = 128;                  // ... x 128 uv cells
constexpr int FK = 16;                   // pixels per LDS stage

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// S[p][k] = exp(2 pi i (u_k l_p + v_k m_p)), [n_pix][n_uv].
__global__ void sky_modes_kernel(const double *__restrict__ lm, const double *__restrict__ uv, int64_t n_pix,
                                 int n_uv, double2 *__restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_pix * n_uv) return;
    const int64_t p = e / n_uv;
    const int k = (int)(e - p * n_uv);
    double s, c;
    sincospi(2.0 * (uv[2 * k] * lm[2 * p] + uv[2 * k + 1] * lm[2 * p + 1]), &s, &c);
    S[e] = make_double2(c, s);
}

struct FmArgs {
    const double *freq, *bl, *lm, *beam;
    const double2 *Z;  // [F][n_eta]
    const double2 *S;  // [n_pix][n_uv]
    int64_t n_pix;
    int n_bl, n_uv, n_eta;
    double norm;
    double2 *T;
    int64_t ldT;
};

// Grid (uv tiles, baseline tiles, channels); wave w owns tile rows
// (baselines) 16 (w % 2) .. + 15 and uv columns 64 (w / 2) .. + 63, as four
// 16-column blocks.
__global__ __launch_bounds__(256) void fm_kernel(FmArgs a) {
    __shared__ double2 Es[FB][FK + 1];  // [baseline][pixel]
    __shared__ double2 Bs[FK][FU + 1];  // [pixel][uv cell]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    const int wr = 16 * (w & 1), wc = 64 * (w >> 1);
    const int k0 = blockIdx.x * FU, b0 = blockIdx.y * FB, f = blockIdx.z;
    const double fc = a.freq[f] / C_LIGHT;
    const double *beam = a.beam + (int64_t)f * a.n_pix;
    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) t1[c] = t2[c] = t3[c] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t p0 = 0; p0 < a.n_pix; p0 += FK) {
        for (int e = tid; e < FB * FK; e += 256) {
            const int bl = e / FK, pl = e % FK, b = b0 + bl;
            const int64_t p = p0 + pl;
            double2 v = make_double2(0.0, 0.0);
            if (b < a.n_bl && p < a.n_pix) {
                double s, c;
                sincospi(-2.0 * fc * (a.bl[2 * b] * a.lm[2 * p] + a.bl[2 * b + 1] * a.lm[2 * p + 1]), &s, &c);
                v = make_double2(c, s);
            }
            Es[bl][pl] = v;
        }
        for (int e = tid; e < FK * FU; e += 256) {
            const int pl = e / FU, kl = e % FU, k = k0 + kl;
            const int64_t p = p0 + pl;
            double2 v = make_double2(0.0, 0.0);
            if (p < a.n_pix && k < a.n_uv) {
                const double A = beam[p];
                const double2 s = a.S[p * a.n_uv + k];
                v = make_double2(A * s.x, A * s.y);
            }
            Bs[pl][kl] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < FK; ks += 4) {
            const double2 av = Es[wr + l16][ks + q];
            const double as = av.x + av.y;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 bv = Bs[ks + q][wc + 16 * c + l16];
                t1[c] = mfma64(av.x, bv.x, t1[c]);
                t2[c] = mfma64(av.y, bv.y, t2[c]);
                t3[c] = mfma64(as, bv.x + bv.y, t3[c]);
            }
        }
        __syncthreads();
    }
    // lane holds G_f[b0 + wr + q + 4 r][k0 + wc + 16 c + l16]:
    // re = T1 - T2, im = T3 - T1 - T2
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int b = b0 + wr + q + 4 * r;
        if (b >= a.n_bl) continue;
        double2 *Trow = a.T + ((int64_t)f * a.n_bl + b) * a.ldT;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = k0 + wc + 16 * c + l16;
            if (k >= a.n_uv) continue;
            const double gr = t1[c][r] - t2[c][r], gi = t3[c][r] - t1[c][r] - t2[c][r];
            for (int e = 0; e < a.n_eta; ++e) {
                const double2 z = a.Z[(int64_t)f * a.n_eta + e];
                const double zr = a.norm * z.x, zi = a.norm * z.y;
                Trow[(int64_t)e * a.n_uv + k] = make_double2(zr * gr - zi * gi, zr * gi + zi * gr);
            }
        }
    }
}

}  // namespace

}  // namespace eor

extern "C" eor_status eor_forward_model(int64_t n_freq, int64_t n_bl, int64_t n_pix, int64_t n_uv, int64_t n_eta,
                                        const double *freq, const double *bl, const double *lm, const double *beam,
                                        const double *uv, const double *Z, double norm, double *T, int64_t ldT,
                                        void *stream) {
    if (n_freq < 1 || n_bl < 1 || n_pix < 1 || n_uv < 1 || n_eta < 1 || n_freq > 65535 ||
        n_bl > (int64_t)65535 * 32 || n_uv > (int64_t)65535 * 64 || n_eta > (1 << 20) || n_pix > ((int64_t)1 << 31) ||
        n_pix * n_uv > ((int64_t)1 << 34))
        return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: sizes out of range");
    if (!freq || !bl || !lm || !beam || !uv || !Z || !T)
        return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: NULL array");
    if (ldT < n_eta * n_uv) return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: ldT < n_eta n_uv");
    if (!std::isfinite(norm)) return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: norm is not finite");
    hipStream_t hs = (hipStream_t)stream;
    double2 *S = nullptr;
    hipError_t e = hipMallocAsync((void **)&S, (size_t)n_pix * n_uv * sizeof(double2), hs);
    if (e != hipSuccess) return eor::hip_status(e, "eor_forward_model scratch");
    const int64_t ns = n_pix * n_uv;
    hipLaunchKernelGGL(eor::sky_modes_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, hs, lm, uv, n_pix,
                       (int)n_uv, S);
    eor::FmArgs a;
    a.freq = freq;
    a.bl = bl;
    a.lm = lm;
    a.beam = beam;
    a.Z = reinterpret_cast<const double2 *>(Z);
    a.S = S;
    a.n_pix = n_pix;
    a.n_bl = (int)n_bl;
    a.n_uv = (int)n_uv;
    a.n_eta = (int)n_eta;
    a.norm = norm;
    a.T = reinterpret_cast<double2 *>(T);
    a.ldT = ldT;
    const dim3 grid((unsigned)((n_uv + eor::FU - 1) / eor::FU), (unsigned)((n_bl + eor::FB - 1) / eor::FB),
                    (unsigned)n_freq);
    hipLaunchKernelGGL(eor::fm_kernel, grid, dim3(256), 0, hs, a);
    e = hipGetLastError();
    (void)hipFreeAsync(S, hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_forward_model");
}
