// Instrument forward model: the dense matrix T that takes the model's
// coefficients (a Fourier-domain sky cube) to visibilities, from the uv
// sampling, the primary beam and the model's basis (the instrument model of
// the paper's "Running BayesEoR" section; the paper gives no formula, the
// visibility equation used is stated with eor_forward_model).
//
// For channel f, G_f[b][k] = sum_p E_f[b][p] S[p][k] with
//   E_f[b][p] = A[f][p] exp(-2 pi i nu_f / c (x_b l_p + y_b m_p)),
//   S[p][k]   = exp(2 pi i (u_k l_p + v_k m_p))
// (S does not depend on the channel: a small kernel writes it once). Then
// T[f n_bl + b][e n_uv + k] = norm Z[f][e] G_f[b][k] for every spectral
// mode e. Two kernels:
//  - fm_partial_kernel: one workgroup per 32 x 128 tile of G_f (32
//    baselines, so that each phase factor is made once for up to 128 uv
//    cells) and chunk of the pixels, on FP64 MFMA with three real 16x16x4
//    products per complex step (Gauss). The pixel sum is cut into chunks so
//    that there are several workgroups per resident slot (the chip then
//    stays evenly loaded to the end); each chunk's sum goes to its own
//    partial of G. While the matrix cores work on one stage of 16 pixels,
//    the loads of the next stage's S rows, pixel directions and beam values
//    are in flight. Two workgroups share a CU (the register budget is bounded
//    for it), so one makes its phase factors and fills LDS while the other's
//    products run.
//  - fm_expand_kernel: adds the partials in chunk order and writes T, one
//    thread per (row, uv cell) and all the spectral modes, so that T is
//    written once, in full rows (non-temporal stores: it is not read here).
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"

namespace eor {

namespace {

constexpr double C_LIGHT = 299792458.0;  // m / s
constexpr int FB = 32;                   // tile: 32 baselines ...
constexpr int FU = 128;                  // ... x 128 uv cells
constexpr int FK = 16;                   // pixels per stage

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
    const double2 *S;  // [n_pix][n_uv]
    int64_t n_pix, chunk;  // pixels; pixels per chunk (a multiple of FK)
    int n_freq, n_bl, n_uv, nbt, n_chunk;
    double2 *G;  // partials [n_chunk][n_freq n_bl][n_uv]
};

// A thread's staging values: eight S entries of one pixel row (held as a
// register vector rather than an array), and the directions and beam values
// of two pixels, from which their phase factors are made.
typedef double d16 __attribute__((ext_vector_type(16)));
struct SRow {
    d16 v;  // entry i: (re, im) at 2 i, 2 i + 1
};
struct Pix {
    double2 lm[2];
    double beam[2];
};

// S row p0 + sp at columns k0 + sk + 16 i (both clamped to the last one).
__device__ __forceinline__ void load_s(const FmArgs &a, SRow &r, int64_t p0, int sp, int sk, int k0,
                                       int64_t klast) {
    const double2 *Srow = a.S + min(p0 + sp, a.n_pix - 1) * a.n_uv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 v = Srow[min<int64_t>(k0 + sk + 16 * i, klast)];
        r.v[2 * i] = v.x;
        r.v[2 * i + 1] = v.y;
    }
}

// Pixels p0 + ep and p0 + ep + 1: direction (clamped to the last pixel) and
// beam value (zero past the chunk's end).
__device__ __forceinline__ void load_pix(const FmArgs &a, Pix &x, int64_t p0, int64_t pend, int ep,
                                         const double2 *lm2, const double *beam) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t p = p0 + ep + j, pc = min(p, a.n_pix - 1);
        x.lm[j] = lm2[pc];
        const double bv = beam[pc];  // in bounds: pc is clamped
        x.beam[j] = p < pend ? bv : 0.0;
    }
}

// E for one baseline at the two pixels: A exp(-2 pi i nu / c (x l + y m)).
__device__ __forceinline__ void phases(const Pix &x, double fc, double bx, double by, double2 e[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        double s, c;
        sincospi(-2.0 * fc * (bx * x.lm[j].x + by * x.lm[j].y), &s, &c);
        e[j] = make_double2(x.beam[j] * c, x.beam[j] * s);
    }
}

// One workgroup per (uv tile, chunk, channel, baseline tile), baseline tile
// fastest. Wave w owns tile rows (baselines) 16 (w % 2) .. + 15 and uv
// columns 64 (w / 2) .. + 63, as four 16-column blocks. Staging: thread t
// makes the phases of baseline t / 8 at pixels 2 (t % 8) and 2 (t % 8) + 1,
// and copies S row t / 16 at columns t % 16 + 16 i, i = 0 .. 7. Indices past
// the last baseline, pixel row or uv cell are clamped to the last one (those
// rows and columns are never written); pixels past the chunk get a beam
// value of zero, so they add nothing.
// At most 256 registers per lane (two workgroups per CU): the accumulators
// then live in ordinary vector registers, with no copies to and from the
// accumulation registers at every stage.
__global__ __launch_bounds__(256, 2) void fm_partial_kernel(FmArgs a) {
    __shared__ double2 Es[FB][FK + 1];  // [baseline][pixel]
    __shared__ double2 Bs[FK][FU + 1];  // [pixel][uv cell]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    const int wr = 16 * (w & 1), wc = 64 * (w >> 1);
    int64_t u = blockIdx.x;
    const int bt = (int)(u % a.nbt);
    u /= a.nbt;
    const int f = (int)(u % a.n_freq);
    u /= a.n_freq;
    const int ch = (int)(u % a.n_chunk);
    const int ut = (int)(u / a.n_chunk);
    const int b0 = bt * FB, k0 = ut * FU;
    const int64_t pbeg = ch * a.chunk, pend = min(a.n_pix, pbeg + a.chunk);
    const double fc = a.freq[f] / C_LIGHT;
    const double *beam = a.beam + (int64_t)f * a.n_pix;
    const double2 *lm2 = reinterpret_cast<const double2 *>(a.lm);
    // this thread's staging roles
    const int eb = tid >> 3, ep = 2 * (tid & 7);
    const int be = min(b0 + eb, a.n_bl - 1);
    const double bx = a.bl[2 * be], by = a.bl[2 * be + 1];
    const int sp = tid >> 4, sk = tid & 15;
    const int64_t klast = a.n_uv - 1;

    // Pipeline: while the products of stage s run, stage s + 1's S row is in
    // flight, its phase factors are made from the pixel values loaded during
    // stage s - 1, and the pixel values of stage s + 2 are loaded. The loads
    // past the chunk's end are clamped and their results never stored.
    SRow sn;
    Pix xc, xn;
    double2 en[2];
    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) t1[c] = t2[c] = t3[c] = d4{0.0, 0.0, 0.0, 0.0};
    load_s(a, sn, pbeg, sp, sk, k0, klast);
    load_pix(a, xc, pbeg, pend, ep, lm2, beam);
    phases(xc, fc, bx, by, en);
    load_pix(a, xc, pbeg + FK, pend, ep, lm2, beam);
    Es[eb][ep] = en[0];
    Es[eb][ep + 1] = en[1];
#pragma unroll
    for (int i = 0; i < 8; ++i) Bs[sp][sk + 16 * i] = make_double2(sn.v[2 * i], sn.v[2 * i + 1]);
    __syncthreads();
    const int ns = (int)((pend - pbeg + FK - 1) / FK);  // stages of this chunk
    for (int it = 0; it < ns; ++it) {
        const int64_t p0 = pbeg + (int64_t)it * FK;
        load_s(a, sn, p0 + FK, sp, sk, k0, klast);
        load_pix(a, xn, p0 + 2 * FK, pend, ep, lm2, beam);
        phases(xc, fc, bx, by, en);
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
        if (it + 1 < ns) {  // uniform
            Es[eb][ep] = en[0];
            Es[eb][ep + 1] = en[1];
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[sp][sk + 16 * i] = make_double2(sn.v[2 * i], sn.v[2 * i + 1]);
            xc = xn;
        }
        __syncthreads();
    }
    // lane holds G[b0 + wr + q + 4 r][k0 + wc + 16 c + l16]:
    // re = T1 - T2, im = T3 - T1 - T2
    double2 *G = a.G + ((int64_t)ch * a.n_freq + f) * a.n_bl * a.n_uv;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int b = b0 + wr + q + 4 * r;
        if (b >= a.n_bl) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = k0 + wc + 16 * c + l16;
            if (k >= a.n_uv) continue;
            G[(int64_t)b * a.n_uv + k] = make_double2(t1[c][r] - t2[c][r], t3[c][r] - t1[c][r] - t2[c][r]);
        }
    }
}

typedef double dv2 __attribute__((ext_vector_type(2)));

struct ExpArgs {
    const double2 *G;  // partials [n_chunk][rows][n_uv]
    const double2 *Z;  // [n_freq][n_eta]
    int64_t rows;      // n_freq n_bl
    int n_bl, n_uv, n_eta, n_chunk;
    double norm;
    double2 *T;
    int64_t ldT;
};

// T[row][e n_uv + k] = norm Z[f][e] sum_chunks G[chunk][row][k], row = f n_bl + b.
__global__ __launch_bounds__(256) void fm_expand_kernel(ExpArgs a) {
    const int64_t total = a.rows * a.n_uv;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / a.n_uv;
        const int k = (int)(e - row * a.n_uv);
        const int f = (int)(row / a.n_bl);
        double2 g = a.G[e];
        for (int c = 1; c < a.n_chunk; ++c) {
            const double2 h = a.G[(int64_t)c * total + e];
            g.x += h.x;
            g.y += h.y;
        }
        // T is written once and not read here: non-temporal stores
        dv2 *Trow = reinterpret_cast<dv2 *>(a.T + row * a.ldT + k);
        const double2 *Zf = a.Z + (int64_t)f * a.n_eta;
        for (int m = 0; m < a.n_eta; ++m) {
            const double2 z = Zf[m];
            const double zr = a.norm * z.x, zi = a.norm * z.y;
            const dv2 t = {zr * g.x - zi * g.y, zr * g.y + zi * g.x};
            __builtin_nontemporal_store(t, Trow + (int64_t)m * a.n_uv);
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
    // Pixel chunks: enough workgroups for several per resident slot (about
    // 2048 in all), at most 16 chunks and at least one stage per chunk.
    const int64_t nbt = (n_bl + eor::FB - 1) / eor::FB, nut = (n_uv + eor::FU - 1) / eor::FU;
    const int64_t base = n_freq * nbt * nut, stages = (n_pix + eor::FK - 1) / eor::FK;
    int64_t want = (2048 + base - 1) / base;
    want = std::max<int64_t>(1, std::min<int64_t>({want, 16, stages}));
    const int64_t chunk = ((stages + want - 1) / want) * eor::FK;
    const int64_t n_chunk = (n_pix + chunk - 1) / chunk;
    const int64_t units = base * n_chunk, rows = n_freq * n_bl;
    if (units > (int64_t)INT32_MAX)
        return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: more than 2^31 - 1 tiles");
    if (rows * n_uv > ((int64_t)1 << 40))  // keeps the partials' byte count far from overflow
        return eor::fail_status(EOR_ERR_ARG, "eor_forward_model: n_freq n_bl n_uv > 2^40");
    hipStream_t hs = (hipStream_t)stream;
    double2 *S = nullptr, *G = nullptr;
    hipError_t e = hipMallocAsync((void **)&S, (size_t)n_pix * n_uv * sizeof(double2), hs);
    if (e != hipSuccess) return eor::hip_status(e, "eor_forward_model scratch");
    e = hipMallocAsync((void **)&G, (size_t)n_chunk * rows * n_uv * sizeof(double2), hs);
    if (e != hipSuccess) {
        (void)hipFreeAsync(S, hs);
        return eor::hip_status(e, "eor_forward_model scratch");
    }
    const int64_t ns = n_pix * n_uv;
    hipLaunchKernelGGL(eor::sky_modes_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, hs, lm, uv, n_pix,
                       (int)n_uv, S);
    eor::FmArgs a;
    a.freq = freq;
    a.bl = bl;
    a.lm = lm;
    a.beam = beam;
    a.S = S;
    a.n_pix = n_pix;
    a.chunk = chunk;
    a.n_freq = (int)n_freq;
    a.n_bl = (int)n_bl;
    a.n_uv = (int)n_uv;
    a.nbt = (int)nbt;
    a.n_chunk = (int)n_chunk;
    a.G = G;
    hipLaunchKernelGGL(eor::fm_partial_kernel, dim3((unsigned)units), dim3(256), 0, hs, a);
    eor::ExpArgs x;
    x.G = G;
    x.Z = reinterpret_cast<const double2 *>(Z);
    x.rows = rows;
    x.n_bl = (int)n_bl;
    x.n_uv = (int)n_uv;
    x.n_eta = (int)n_eta;
    x.n_chunk = (int)n_chunk;
    x.norm = norm;
    x.T = reinterpret_cast<double2 *>(T);
    x.ldT = ldT;
    const int64_t eblocks = std::min<int64_t>((rows * n_uv + 255) / 256, 4096);
    hipLaunchKernelGGL(eor::fm_expand_kernel, dim3((unsigned)eblocks), dim3(256), 0, hs, x);
    e = hipGetLastError();
    (void)hipFreeAsync(G, hs);
    (void)hipFreeAsync(S, hs);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "eor_forward_model");
}
