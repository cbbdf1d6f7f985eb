// Once-per-dataset products: A = T^H N^{-1} T (packed lower tiles),
// dbar = T^H N^{-1} d, c = d^H N^{-1} d and -sum ln sigma_i^2.
//
// A is a Hermitian rank-m product (HERK). Each workgroup forms one 64 x 64
// tile A[64i.., 64j..] (i >= j), or its share over a slice of the rows, on
// FP64 MFMA, with three real 16x16x4 MFMAs per complex step (Gauss).
// Wave w owns tile rows 16w..16w+15; the accumulator is kept transposed
// (MFMA rows = tile columns) so that each 16-lane group of a wave stores 16
// consecutive elements of a tile column.
#include <algorithm>

#include "common.h"

namespace eor {

namespace {

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline void tile_of(int64_t t, int64_t &i, int64_t &j) {
    // inverse of tile_index: largest i with i(i+1)/2 <= t
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    i = r;
    j = t - r * (r + 1) / 2;
}

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// Raw buffer over nbytes at p (a wave-uniform address); loads past nbytes
// return zero. A lane offset of OOB reads zero as well (used for the padded
// columns n..n_pad).
constexpr int OOB = 0x7ffffff0;

__device__ inline rsrc_t make_rsrc(const void *p, int64_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)nbytes, 0x00020000);
}

__device__ inline double2 ld2(rsrc_t r, int voff, int soff) {
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    double2 x;
    __builtin_memcpy(&x, &v, sizeof(x));
    return x;
}

__device__ inline double ld1(rsrc_t r, int voff, int soff) {
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    double x;
    __builtin_memcpy(&x, &v, sizeof(x));
    return x;
}

// Operands of one k-step (rows s0..s0+3 of T, row s0 + q in lane group q):
// the tile-row block (T[s][64 i + 16 w + l16]), the four tile-column blocks
// (T[s][64 j + 16 cb + l16]) and 1 / sigma_s^2 (zero past the last row).
struct HerkStep {
    double2 p;
    double2 qv[4];
    double wgt;
};

__device__ inline void herk_load(HerkStep &st, rsrc_t Trow, rsrc_t W, int vp, const int vq[4], int vw,
                                 int soff_w) {
    st.p = ld2(Trow, vp, 0);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) st.qv[cb] = ld2(Trow, vq[cb], 0);
    st.wgt = ld1(W, vw, soff_w);
}

// conj(p) q with p weighted, three real products (Gauss):
//   T1 = qr pr, T2 = qi pi, T3 = (qr + qi)(pr - pi)
//   Re = T1 + T2, Im = qi pr - qr pi = T3 - T1 + T2
__device__ inline void herk_step(const HerkStep &st, d4 t1[4], d4 t2[4], d4 t3[4]) {
    const double pr = st.p.x * st.wgt, pi = st.p.y * st.wgt;
    const double pd = pr - pi;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        t1[cb] = mfma64(st.qv[cb].x, pr, t1[cb]);
        t2[cb] = mfma64(st.qv[cb].y, pi, t2[cb]);
        t3[cb] = mfma64(st.qv[cb].x + st.qv[cb].y, pd, t3[cb]);
    }
}

// One work unit: tile u % tiles of the lower triangle over rows
// [split * rows_per, (split + 1) * rows_per), split = u / tiles (units that
// run at the same time share rows of T in L2). With one split the tile goes
// straight to A with the Hermitian and padding fix-ups; otherwise to its
// slot of `part`, and herk_reduce_kernel sums the splits in a fixed order.
constexpr int HERK_STAGES = 4;

__global__ __launch_bounds__(256, 2) void herk_fp64_kernel(const double2 *__restrict__ T, int64_t ldT,
                                                           int64_t m, int64_t n,
                                                           const double *__restrict__ invvar,
                                                           int64_t tiles, int64_t rows_per, int splits,
                                                           double2 *__restrict__ out) {
    const int64_t unit = blockIdx.x;
    const int64_t tile = unit % tiles, split = unit / tiles;
    int64_t ti, tj;
    tile_of(tile, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t r0 = split * rows_per;
    const int64_t r1 = r0 + rows_per < m ? r0 + rows_per : m;

    // lane offsets inside a 4-row block of T (padded columns read as zero)
    const int64_t col_p = TS * ti + 16 * w + l16;
    const int vp = col_p < n ? (int)((q * ldT + col_p) * 16) : OOB;
    int vq[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int64_t col = TS * tj + 16 * cb + l16;
        vq[cb] = col < n ? (int)((q * ldT + col) * 16) : OOB;
    }
    const rsrc_t W = make_rsrc(invvar, m * 8);
    const int vw = q * 8;

    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) t1[cb] = t2[cb] = t3[cb] = d4{0, 0, 0, 0};

    // Block of rows s..s+3: descriptor based at row s, sized to the rows
    // that exist; the prefetch may run past r1 (into rows of the next split,
    // or past m where the descriptor reads zero) and is never used.
    auto rows_at = [&](int64_t s) {
        const int64_t left = m - s;
        const int64_t nb = left <= 0 ? 0 : (left < 4 ? left : 4) * ldT * 16;
        return make_rsrc(T + (left <= 0 ? 0 : s * ldT), nb);
    };
    HerkStep buf[HERK_STAGES];
#pragma unroll
    for (int s0 = 0; s0 < HERK_STAGES - 1; ++s0) {
        const int64_t s = r0 + 4 * s0;
        herk_load(buf[s0], rows_at(s), W, vp, vq, vw, (int)(s * 8));
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t s0 = r0; s0 < r1; s0 += 4 * HERK_STAGES) {
        if (((s0 - r0) & (TS - 1)) == 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < HERK_STAGES; ++u) {
            const int64_t sl = s0 + 4 * (u + HERK_STAGES - 1);
            herk_load(buf[(u + HERK_STAGES - 1) % HERK_STAGES], rows_at(sl), W, vp, vq, vw, (int)(sl * 8));
            if (s0 + 4 * u < r1) herk_step(buf[u], t1, t2, t3);
        }
    }

    // lane holds A[64 ti + 16 w + l16][64 tj + 16 cb + q + 4 r] (the MFMA
    // returns D[l/16 + 4r][l%16] in register r)
    const int row = 16 * w + l16;
    const int64_t grow = TS * ti + row;
    double2 *dst = out + (splits > 1 ? (split * tiles + tile) : tile_index(ti, tj)) * TS2;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = 16 * cb + q + 4 * r;
            const int64_t gcol = TS * tj + col;
            double2 v = make_double2(t1[cb][r] + t2[cb][r], t3[cb][r] - t1[cb][r] + t2[cb][r]);
            if (splits == 1) {
                if (grow == gcol) v.y = 0.0;  // Hermitian: real diagonal
                if (grow >= n || gcol >= n) v = make_double2(grow == gcol ? 1.0 : 0.0, 0.0);
            }
            dst[col * TS + row] = v;
        }
    }
}

// A = sum over splits of the partial tiles (fixed order), then the real
// diagonal and the identity padding.
__global__ void herk_reduce_kernel(const double2 *__restrict__ part, int64_t tiles, int splits, int64_t n,
                                   double2 *__restrict__ A) {
    const int64_t total = tiles * TS2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / TS2;
        const int el = (int)(e % TS2), col = el / TS, row = el % TS;
        double2 v = part[e];
        for (int sp = 1; sp < splits; ++sp) {
            const double2 x = part[sp * total + e];
            v.x += x.x;
            v.y += x.y;
        }
        int64_t ti, tj;
        tile_of(t, ti, tj);
        const int64_t grow = TS * ti + row, gcol = TS * tj + col;
        if (grow == gcol) v.y = 0.0;
        if (grow >= n || gcol >= n) v = make_double2(grow == gcol ? 1.0 : 0.0, 0.0);
        A[t * TS2 + el] = v;
    }
}

// invvar_s = 1 / sigma_s^2
__global__ void invvar_kernel(const double *__restrict__ noise_var, int64_t m, double *__restrict__ invvar) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < m) invvar[s] = 1.0 / noise_var[s];
}

// Partial sums of dbar_j = sum_s conj(T_sj) d_s / sigma_s^2 over one slice of rows.
__global__ __launch_bounds__(256) void dbar_partial_kernel(const double2 *__restrict__ T, int64_t ldT,
                                                           int64_t m, int64_t n,
                                                           const double2 *__restrict__ d,
                                                           const double *__restrict__ invvar,
                                                           int64_t rows_per_split,
                                                           double2 *__restrict__ partial) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t split = blockIdx.y;
    if (j >= n) return;
    const int64_t s_lo = split * rows_per_split;
    const int64_t s_hi = s_lo + rows_per_split < m ? s_lo + rows_per_split : m;
    double sr = 0.0, si = 0.0;
    for (int64_t s = s_lo; s < s_hi; ++s) {
        const double2 t = T[s * ldT + j];
        const double2 ds = d[s];
        const double wv = invvar[s];
        sr += (t.x * ds.x + t.y * ds.y) * wv;
        si += (t.x * ds.y - t.y * ds.x) * wv;
    }
    partial[split * n + j] = make_double2(sr, si);
}

__global__ void dbar_reduce_kernel(const double2 *__restrict__ partial, int splits, int64_t n,
                                   int64_t n_pad, double2 *__restrict__ dbar) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    double sr = 0.0, si = 0.0;
    if (j < n) {
        for (int s = 0; s < splits; ++s) {
            sr += partial[s * n + j].x;
            si += partial[s * n + j].y;
        }
    }
    dbar[j] = make_double2(sr, si);
}

// scal[0] = sum_s |d_s|^2 / sigma_s^2, scal[1] = -sum_s ln sigma_s^2 (one
// workgroup, fixed-order tree so the result does not depend on timing).
__global__ __launch_bounds__(256) void scalars_kernel(const double2 *__restrict__ d,
                                                      const double *__restrict__ noise_var, int64_t m,
                                                      double *__restrict__ scal) {
    __shared__ double sc[256], sl[256];
    double c = 0.0, l = 0.0;
    for (int64_t s = threadIdx.x; s < m; s += 256) {
        const double2 ds = d[s];
        c += (ds.x * ds.x + ds.y * ds.y) / noise_var[s];
        l += log(noise_var[s]);
    }
    sc[threadIdx.x] = c;
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sc[threadIdx.x] += sc[threadIdx.x + h];
            sl[threadIdx.x] += sl[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[0] = sc[0];
        scal[1] = -sl[0];
    }
}

// Dense row-major full Hermitian copy of the packed lower tiles.
__global__ void export_A_kernel(const double2 *__restrict__ Ap, int64_t n, int64_t ldA,
                                double2 *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int64_t r = blockIdx.y; r < n; r += gridDim.y) {
        const bool lower = c <= r;
        const int64_t gi = lower ? r : c, gj = lower ? c : r;
        const int64_t ti = gi / TS, tj = gj / TS;
        double2 v = Ap[tile_index(ti, tj) * TS2 + (gj % TS) * TS + (gi % TS)];
        if (!lower) v.y = -v.y;
        out[r * ldA + c] = v;
    }
}

}  // namespace

// Rows of T per work unit, and how many units split each tile's rows: the
// count that best fills whole rounds of the resident workgroups (two per CU),
// with a small charge per split for the partial tiles it writes and reads.
void herk_split(int64_t m, int64_t N, int num_cu, int &splits, int64_t &rows_per) {
    const int64_t tiles = n_tiles(N), slots = 2 * (int64_t)(num_cu > 0 ? num_cu : 1);
    splits = 1;
    double best = -1.0;
    for (int sp = 1; sp <= 8; ++sp) {
        const int64_t rp = ((m + sp - 1) / sp + TS - 1) / TS * TS;
        if (sp > 1 && rp < 4 * TS) break;
        const int64_t units = tiles * sp, rounds = (units + slots - 1) / slots;
        const double score = (double)units / (double)(rounds * slots) - 0.01 * sp;
        if (score > best + 1e-12) {
            best = score;
            splits = sp;
        }
    }
    rows_per = ((m + splits - 1) / splits + TS - 1) / TS * TS;
}

size_t herk_scratch_bytes(int64_t m, int64_t N, int num_cu) {
    int splits;
    int64_t rows_per;
    herk_split(m, N, num_cu, splits, rows_per);
    return splits > 1 ? (size_t)splits * n_tiles(N) * TS2 * sizeof(double2) : 0;
}

hipError_t launch_precompute_fp64(const Context &c, const double2 *T, int64_t ldT, const double *invvar,
                                  void *scratch, hipStream_t s) {
    const int64_t tiles = n_tiles(c.N);
    int splits;
    int64_t rows_per;
    herk_split(c.m, c.N, c.num_cu, splits, rows_per);
    double2 *out = splits > 1 ? (double2 *)scratch : c.A;
    hipLaunchKernelGGL(herk_fp64_kernel, dim3((unsigned)(tiles * splits)), dim3(256), 0, s, T, ldT, c.m, c.n,
                       invvar, tiles, rows_per, splits, out);
    if (splits > 1) return launch_herk_reduce(out, tiles, splits, c.n, c.A, s);
    return hipGetLastError();
}

hipError_t launch_herk_reduce(const double2 *part, int64_t tiles, int splits, int64_t n, double2 *A,
                              hipStream_t s) {
    const int64_t total = tiles * TS2;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(herk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, tiles, splits, n, A);
    return hipGetLastError();
}

hipError_t launch_precompute_vectors(const Context &c, const double2 *T, int64_t ldT,
                                     const double *noise_var, const double2 *d, double *invvar,
                                     double2 *partial, int splits, hipStream_t s) {
    hipLaunchKernelGGL(invvar_kernel, dim3((unsigned)((c.m + 255) / 256)), dim3(256), 0, s, noise_var,
                       c.m, invvar);
    const int64_t rows = (c.m + splits - 1) / splits;
    hipLaunchKernelGGL(dbar_partial_kernel, dim3((unsigned)((c.n + 255) / 256), (unsigned)splits),
                       dim3(256), 0, s, T, ldT, c.m, c.n, d, invvar, rows, partial);
    hipLaunchKernelGGL(dbar_reduce_kernel, dim3((unsigned)((c.n_pad + 255) / 256)), dim3(256), 0, s,
                       partial, splits, c.n, c.n_pad, c.dbar);
    hipLaunchKernelGGL(scalars_kernel, dim3(1), dim3(256), 0, s, d, noise_var, c.m, c.scal);
    return hipGetLastError();
}

hipError_t launch_export_A(const Context &c, double2 *out, int64_t ldA, hipStream_t s) {
    hipLaunchKernelGGL(export_A_kernel, dim3((unsigned)((c.n + 255) / 256), (unsigned)(c.n < 65535 ? c.n : 65535)), dim3(256),
                       0, s, c.A, c.n, ldA, out);
    return hipGetLastError();
}

}  // namespace eor
