// Likelihood with Sigma factored through a bounded device window: the
// out-of-core case (the paper's MAGMA footnote: matrices larger than the
// GPU's memory). A stays in host memory (a pinned packed copy), the factor L
// of a theta in a pinned host buffer of the library, and the device holds a
// pass of tile columns of 64 x 64 tiles plus a window of earlier columns of
// L. Up to four theta run at once, each on a lane of its own (a stream, an
// equal share of the device budget, a host factor), so that one lane's
// copies and launch gaps overlap another's kernels.
//
// Blocked Cholesky over passes of J tile columns [j0, j1) (as many as half
// the device window holds), left-looking across passes:
//   C_ij = A_ij + [i == j] Phi^-1                    (i >= j, the pass copied in)
//   C_ij -= sum_{k < j0} L_ik L_jk^H                  (windows of earlier columns,
//                                                     each read once per pass)
// then, right-looking inside the pass, for j = j0 .. j1-1:
//   L_jj = chol(C_jj), Linv = L_jj^-1, y_j = Linv w_j (one workgroup)
//   L_ij = C_ij Linv^H,  w_i -= L_ij y_j              (i > j)
//   C_il -= L_ij L_lj^H                                (the pass's later columns l)
// with w = dbar at the start, then logL = K0 - ln det Phi - 2 sum ln L_dd -
// (c - |y|^2), the same combination as the batched path. Tiles are row-major
// 64 x 64 complex. On the host, A (copied once per call from the caller's
// row-major matrix) and L are packed by tile columns in pinned memory: tile
// (i, k), i >= k, at k N - k (k - 1) / 2 + (i - k), so that the part of a
// tile column below any row is one contiguous block and every transfer of
// the schedule is a single DMA. The tile products run on FP64 MFMA with
// three real products per complex step.
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <thread>
#include <vector>

#include "common.h"

namespace eor {

namespace {

constexpr int OT = 64;
constexpr int OT2 = OT * OT;

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Orders one wave's LDS accesses across its lanes. The hardware performs a
// wave's LDS instructions in program order; the wave-scope release, wave
// barrier and acquire keep the compiler from moving a lane's load of a value
// that another lane stores (or a store that another lane's load must precede)
// across this point. No instruction is emitted for it.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct OocState {
    double logdet;    // 2 sum ln L_dd
    double quad;      // |y|^2
    double lndetphi;  // ln det Phi
    int32_t info;     // 0, -1 (invalid theta), or the 1-based failing column
};

__global__ void ooc_reset_kernel(OocState *st) {
    st->logdet = 0.0;
    st->quad = 0.0;
    st->lndetphi = 0.0;
    st->info = 0;
}

// Diagonal tile of column j: add 1/phi_d to the diagonal (d < n), set the
// padding's diagonal to 1, and add the column's ln phi_d to ln det Phi in
// a fixed order.
__global__ __launch_bounds__(64) void ooc_diag_kernel(double2 *__restrict__ C0, int64_t j, int64_t n,
                                                     const double *__restrict__ theta,
                                                     const int32_t *__restrict__ bin_of,
                                                     const double *__restrict__ fixed_var,
                                                     const double *__restrict__ bin_scale, OocState *st) {
    __shared__ double lp[OT];
    __shared__ int bad[OT];
    const int t = threadIdx.x;
    const int64_t d = OT * j + t;
    double l = 0.0;
    int b_ = 0;
    if (d < n) {
        const int b = bin_of[d];
        const double phi = b >= 0 ? bin_scale[b] * exp10(theta[b]) : fixed_var[d];
        if (!(phi > 0.0) || !isfinite(phi)) b_ = 1;
        else {
            C0[t * OT + t].x += 1.0 / phi;
            l = log(phi);
        }
    } else {
        C0[t * OT + t] = make_double2(1.0, 0.0);
    }
    lp[t] = l;
    bad[t] = b_;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        int anybad = 0;
        for (int e = 0; e < OT; ++e) {
            s += lp[e];
            anybad |= bad[e];
        }
        if (anybad && st->info == 0) st->info = -1;
        st->lndetphi += s;
    }
}

// out[r][c] (+|-)= sum_s X[r][s] conj(Y[c][s]) for one 64 x 64 tile pair:
// four waves, wave w rows 16w..16w+15, four 16-column blocks; returns the
// accumulators T1 = xr yr, T2 = xi yi, T3 = (xr + xi)(yr - yi), so that
// re = T1 + T2 and im = T3 - T1 + T2.
__device__ inline void tile_xyh(const double2 *__restrict__ X, const double2 *__restrict__ Y, int w, int l16,
                                int q, d4 t1[4], d4 t2[4], d4 t3[4]) {
#pragma unroll 4
    for (int s0 = 0; s0 < OT; s0 += 4) {
        const double2 xv = X[(16 * w + l16) * OT + s0 + q];
        const double xs = xv.x + xv.y;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double2 yv = Y[(16 * cb + l16) * OT + s0 + q];
            t1[cb] = mfma64(xv.x, yv.x, t1[cb]);
            t2[cb] = mfma64(xv.y, yv.y, t2[cb]);
            t3[cb] = mfma64(xs, yv.x - yv.y, t3[cb]);
        }
    }
}

__device__ inline void tile_sub(double2 *__restrict__ Ct, int w, int l16, int q, const d4 t1[4], const d4 t2[4],
                                const d4 t3[4]) {
    // lane holds [16 w + q + 4 r][16 cb + l16]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + q + 4 * r;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            double2 &e = Ct[row * OT + 16 * cb + l16];
            const double re = t1[cb][r] + t2[cb][r], im = t3[cb][r] - t1[cb][r] + t2[cb][r];
            e = make_double2(e.x - re, e.y - im);
        }
    }
}

// Super-column [j0, j1) on the device, packed by tile columns (column j's
// tiles, rows j .. N-1, from local tile col_off(j) - col_off(j0)). One
// workgroup per tile (i, j): C_ij -= sum_k L_ik L_jk^H over the window of
// earlier columns, window column k holding rows j0 .. N-1 (N - j0 tiles).
__global__ __launch_bounds__(256, 2) void ooc_window_kernel(double2 *__restrict__ C, const double2 *__restrict__ Lw,
                                                         int W, int64_t j0, int64_t j1, int64_t N,
                                                         const OocState *st) {
    if (st->info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    int64_t b = blockIdx.x, j = j0;
    while (j < j1 - 1 && b >= N - j) {
        b -= N - j;
        ++j;
    }
    const int64_t i = j + b, rows = N - j0;
    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) t1[cb] = t2[cb] = t3[cb] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < W; ++k)
        tile_xyh(Lw + ((int64_t)k * rows + (i - j0)) * OT2, Lw + ((int64_t)k * rows + (j - j0)) * OT2, w, l16, q,
                 t1, t2, t3);
    tile_sub(C + (int64_t)blockIdx.x * OT2, w, l16, q, t1, t2, t3);
}

// After column k of a pass is factored: C_ij -= L_ik L_jk^H for every later
// column j < j1 of the pass and i >= j, one workgroup per tile (the tiles of
// columns k+1 .. j1-1 are one contiguous run of the pass's packing).
__global__ __launch_bounds__(256, 2) void ooc_pass_kernel(double2 *__restrict__ C, int64_t k, int64_t j0, int64_t j1,
                                                       int64_t N, const OocState *st) {
    if (st->info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    auto loc = [&](int64_t c) { return (c - j0) * N - ((c * (c - 1)) / 2 - (j0 * (j0 - 1)) / 2); };
    int64_t b = blockIdx.x, j = k + 1;
    while (j < j1 - 1 && b >= N - j) {
        b -= N - j;
        ++j;
    }
    const int64_t i = j + b;
    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) t1[cb] = t2[cb] = t3[cb] = d4{0.0, 0.0, 0.0, 0.0};
    tile_xyh(C + (loc(k) + (i - k)) * OT2, C + (loc(k) + (j - k)) * OT2, w, l16, q, t1, t2, t3);
    tile_sub(C + (loc(j) + (i - j)) * OT2, w, l16, q, t1, t2, t3);
}

// Diagonal tile of column j: Cholesky in LDS, ln det, the inverse of L_jj
// and y_j = L_jj^-1 w_j. One workgroup of PT threads, blocked on 16 x 16
// sub-blocks so that few steps wait on a barrier:
//  - Cholesky, right-looking over the four block columns: one wave factors
//    the diagonal block (no workgroup barrier: a wave's LDS accesses run in
//    program order, and wave_sync keeps the compiler to it), one thread per
//    row solves the panel below it, and the
//    rank-16 update of the rest runs on FP64 MFMA, one wave per 16 x 16 block;
//  - inverse: the four diagonal blocks are inverted at once, one wave each,
//    then the blocks below them, nearest the diagonal first, one wave per
//    block on FP64 MFMA: V_ij = -V_ii sum_{k=j..i-1} L_ik V_kj.
constexpr int PT = 512;  // threads of the diagonal factorisation
constexpr int PB = 16;   // sub-block size
constexpr int NPB = OT / PB;

__global__ __launch_bounds__(PT) void ooc_potrf_kernel(double2 *__restrict__ C0, double2 *__restrict__ Linv,
                                                        double2 *__restrict__ w, double2 *__restrict__ y,
                                                        int64_t j, OocState *st) {
    __shared__ double2 S[OT][OT + 1];              // C_jj, then L_jj (lower)
    __shared__ double2 V[OT][OT + 1];              // L_jj^-1 (lower; zero above)
    __shared__ double dinv[OT], lsq[OT];
    __shared__ double2 yj[OT];
    __shared__ int fail_col;
    if (st->info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    {
        // all of the thread's loads in flight before the first LDS store
        double2 v[OT2 / PT];
#pragma unroll
        for (int u = 0; u < OT2 / PT; ++u) v[u] = C0[tid + PT * u];
#pragma unroll
        for (int u = 0; u < OT2 / PT; ++u) {
            const int e = tid + PT * u;
            S[e / OT][e % OT] = v[u];
            V[e / OT][e % OT] = make_double2(0.0, 0.0);
        }
    }
    if (tid == 0) fail_col = 0;
    if (tid < OT) yj[tid] = w[OT * j + tid];  // w_j, read by the solve below
    __syncthreads();

    for (int kb = 0; kb < NPB; ++kb) {
        const int b0 = PB * kb, r0 = b0 + PB;
        // diagonal block, by wave 0: lane (r = lane / 4, s = lane % 4 + 4 u)
        if (wv == 0) {
            const int br = lane >> 2, bs = lane & 3;
            for (int c = 0; c < PB; ++c) {
                const double d = S[b0 + c][b0 + c].x;
                if (!(d > 0.0) || !isfinite(d)) {
                    if (lane == 0) fail_col = b0 + c + 1;
                    break;  // uniform: every lane of the wave reads the same value
                }
                const double l = sqrt(d), il = 1.0 / l;
                if (bs == 0 && br > c) {
                    const double2 x = S[b0 + br][b0 + c];
                    S[b0 + br][b0 + c] = make_double2(x.x * il, x.y * il);
                }
                if (lane == 0) S[b0 + c][b0 + c] = make_double2(l, 0.0);
                wave_sync();  // the scaled column c, stored by lanes bs = 0, is read by every lane
                if (br > c) {
                    const double2 a = S[b0 + br][b0 + c];
#pragma unroll
                    for (int u = 0; u < PB / 4; ++u) {
                        const int sc = bs + 4 * u;
                        if (sc > c && sc <= br) {
                            const double2 b = S[b0 + sc][b0 + c];
                            const double2 x = S[b0 + br][b0 + sc];
                            // x - a conj(b)
                            S[b0 + br][b0 + sc] = make_double2(x.x - (a.x * b.x + a.y * b.y),
                                                               x.y - (a.y * b.x - a.x * b.y));
                        }
                    }
                }
                wave_sync();  // column c + 1 and its pivot, updated by other lanes, are read next
            }
        }
        __syncthreads();
        if (fail_col != 0) break;  // uniform: read after the barrier
        if (r0 < OT) {
            // panel below: row r solves x L_kk^H = s, one thread per row
            if (tid < OT - r0) {
                const int r = r0 + tid;
                double2 x[PB];
#pragma unroll
                for (int c = 0; c < PB; ++c) {
                    double2 a = S[r][b0 + c];
#pragma unroll
                    for (int t = 0; t < c; ++t) {
                        const double2 l = S[b0 + c][b0 + t];  // x_t conj(l)
                        a.x -= x[t].x * l.x + x[t].y * l.y;
                        a.y -= x[t].y * l.x - x[t].x * l.y;
                    }
                    const double il = 1.0 / S[b0 + c][b0 + c].x;
                    x[c] = make_double2(a.x * il, a.y * il);
                }
#pragma unroll
                for (int c = 0; c < PB; ++c) S[r][b0 + c] = x[c];
            }
            __syncthreads();
            // rank-16 update of the rest, S[r][s] -= sum_t L[r][t] conj(L[s][t]), by
            // 16 x 16 blocks (I, J), kb < J <= I, one wave each on FP64 MFMA (a
            // diagonal block is updated whole: its upper part is never read)
            {
                int bi = 0, bj = 0, idx = 0;
                for (int ii = kb + 1; ii < NPB; ++ii)
                    for (int jj = kb + 1; jj <= ii; ++jj, ++idx)
                        if (idx == wv) bi = ii, bj = jj;
                if (wv < idx) {
                    const int l16 = lane & 15, q = lane >> 4;
                    d4 t1 = d4{0, 0, 0, 0}, t2 = d4{0, 0, 0, 0}, t3 = d4{0, 0, 0, 0};
#pragma unroll
                    for (int s0 = 0; s0 < PB; s0 += 4) {
                        const double2 xv = S[PB * bi + l16][b0 + s0 + q];  // A[i][k]
                        const double2 yv = S[PB * bj + l16][b0 + s0 + q];  // B[k][j] = conj(L[s][t]) parts
                        t1 = mfma64(xv.x, yv.x, t1);
                        t2 = mfma64(xv.y, yv.y, t2);
                        t3 = mfma64(xv.x + xv.y, yv.x - yv.y, t3);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double2 &e = S[PB * bi + q + 4 * r][PB * bj + l16];
                        e = make_double2(e.x - (t1[r] + t2[r]), e.y - (t3[r] - t1[r] + t2[r]));
                    }
                }
            }
            __syncthreads();
        }
    }
    if (fail_col != 0) {
        if (tid == 0) st->info = (int32_t)(OT * j + fail_col);
        return;
    }
    if (tid < OT) {
        const double l = S[tid][tid].x;
        dinv[tid] = 1.0 / l;
        lsq[tid] = log(l);
    }
    __syncthreads();
    // inverse: diagonal blocks, wave kb on block kb, lane = column
    if (wv < NPB && lane < PB) {
        const int b0 = PB * wv, cc = lane;
        V[b0 + cc][b0 + cc] = make_double2(dinv[b0 + cc], 0.0);
        for (int r = 1; r < PB; ++r) {
            if (r > cc) {
                double sr = 0.0, si = 0.0;
#pragma unroll 4
                for (int t = cc; t < r; ++t) {
                    const double2 a = S[b0 + r][b0 + t], b = V[b0 + t][b0 + cc];
                    sr += a.x * b.x - a.y * b.y;
                    si += a.x * b.y + a.y * b.x;
                }
                const double f = -dinv[b0 + r];
                V[b0 + r][b0 + cc] = make_double2(sr * f, si * f);
            }
        }
    }
    __syncthreads();
    // blocks below the diagonal, distance dd = ib - jb, one wave each on FP64
    // MFMA: X = sum_k L_ib,k V_k,jb, then V_ib,jb = -V_ib,ib X, with X kept in
    // the wave's accumulators (lane holds X[q + 4r][l16], which is the second
    // operand of k-step r of the next product); complex products with three
    // real ones: re = T1 - T2, im = T3 - T1 - T2
    for (int dd = 1; dd < NPB; ++dd) {
        if (wv < NPB - dd) {
            const int jb = wv, ib = jb + dd, l16 = lane & 15, q = lane >> 4;
            d4 t1 = d4{0, 0, 0, 0}, t2 = d4{0, 0, 0, 0}, t3 = d4{0, 0, 0, 0};
            for (int k0 = PB * jb; k0 < PB * ib; k0 += 4) {
                const double2 l = S[PB * ib + l16][k0 + q];  // A[i][k]
                const double2 v = V[k0 + q][PB * jb + l16];  // B[k][j]
                t1 = mfma64(l.x, v.x, t1);
                t2 = mfma64(l.y, v.y, t2);
                t3 = mfma64(l.x + l.y, v.x + v.y, t3);
            }
            const d4 xr = t1 - t2, xi = t3 - t1 - t2;
            d4 u1 = d4{0, 0, 0, 0}, u2 = d4{0, 0, 0, 0}, u3 = d4{0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double2 a = V[PB * ib + l16][PB * ib + 4 * r + q];  // V_ii (zero above its diagonal)
                u1 = mfma64(a.x, xr[r], u1);
                u2 = mfma64(a.y, xi[r], u2);
                u3 = mfma64(a.x + a.y, xr[r] + xi[r], u3);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                V[PB * ib + q + 4 * r][PB * jb + l16] = make_double2(-(u1[r] - u2[r]), -(u3[r] - u1[r] - u2[r]));
        }
        __syncthreads();
    }
    // write L_jj (zero above the diagonal) and its inverse
    for (int e = tid; e < OT2; e += PT) {
        const int r = e / OT, c = e % OT;
        C0[e] = c < r ? S[r][c] : (c == r ? make_double2(S[r][r].x, 0.0) : make_double2(0.0, 0.0));
        Linv[e] = c <= r ? V[r][c] : make_double2(0.0, 0.0);
    }
    // y_j = Linv w_j (w_j in yj since the start; every thread reads it before
    // the rows' results replace it)
    double sr = 0.0, si = 0.0;
    if (tid < OT) {
#pragma unroll 4
        for (int t = 0; t <= tid; ++t) {
            const double2 a = V[tid][t], b = yj[t];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
    }
    __syncthreads();
    if (tid < OT) {
        yj[tid] = make_double2(sr, si);
        y[OT * j + tid] = yj[tid];
    }
    __syncthreads();
    if (tid == 0) {
        double ld = 0.0, qd = 0.0;
        for (int d = 0; d < OT; ++d) {
            ld += lsq[d];
            qd += yj[d].x * yj[d].x + yj[d].y * yj[d].y;
        }
        st->logdet += 2.0 * ld;
        st->quad += qd;
    }
}

// L_ij = C_i Linv^H for the tiles below the diagonal (t = blockIdx.x + 1),
// then w_i -= L_ij y_j.
__global__ __launch_bounds__(256, 2) void ooc_trsm_kernel(double2 *__restrict__ C, const double2 *__restrict__ Linv,
                                                       double2 *__restrict__ w, const double2 *__restrict__ y,
                                                       int64_t j, const OocState *st) {
    if (st->info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, q = lane >> 4;
    const int64_t t = (int64_t)blockIdx.x + 1;
    double2 *Ct = C + t * OT2;
    d4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) t1[cb] = t2[cb] = t3[cb] = d4{0.0, 0.0, 0.0, 0.0};
    tile_xyh(Ct, Linv, wv, l16, q, t1, t2, t3);
    // each wave reads and writes only its own 16 rows of C_t
    const double2 *yj = y + OT * j;
    double pr[4] = {0.0, 0.0, 0.0, 0.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * wv + q + 4 * r;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double re = t1[cb][r] + t2[cb][r], im = t3[cb][r] - t1[cb][r] + t2[cb][r];
            Ct[row * OT + 16 * cb + l16] = make_double2(re, im);
            const double2 b = yj[16 * cb + l16];
            pr[r] += re * b.x - im * b.y;
            pi[r] += re * b.y + im * b.x;
        }
    }
    // sum over the 16 columns of a lane group, fixed xor tree
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            pr[r] += __shfl_xor(pr[r], o);
            pi[r] += __shfl_xor(pi[r], o);
        }
    }
    if (l16 == 0) {
        const int64_t i = j + t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double2 &e = w[OT * i + 16 * wv + q + 4 * r];
            e = make_double2(e.x - pr[r], e.y - pi[r]);
        }
    }
}

__global__ void ooc_finish_kernel(const OocState *st, double K0, double c, double *logL, int32_t *info) {
    if (st->info != 0) {
        *logL = -INFINITY;
        *info = st->info;
    } else {
        *logL = K0 - st->lndetphi - st->logdet - (c - st->quad);
        *info = 0;
    }
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// The schedule of a call, fixed by its arguments (never by the number of
// theta, so that a theta's result does not depend on the batch it is in).
struct OocPlan {
    int lanes = 1;      // theta factored at once, each on its own stream
    int64_t N = 0;      // tile rows
    int64_t n_pad = 0;  // N * 64
    int64_t J = 0;      // tile columns per pass
    int64_t capC = 0;   // tiles of a lane's pass buffer (J N)
    int64_t cap = 0;    // tiles of a lane's window of earlier columns (>= N)
    size_t shared_b = 0, lane_fixed_b = 0;
    int64_t link_bytes = 0;  // host <-> device bytes per theta
};

constexpr size_t TILE_B = (size_t)OT2 * sizeof(double2);
constexpr int MAX_LANES = 4;

int64_t ntiles(int64_t N) { return N * (N + 1) / 2; }

// Device bytes: shared dbar, bin map, fixed variances and scales; per lane
// Linv, w and y, the state and theta and result slots, then the lane's
// share of what is left in tiles, in whole full-height tile columns. The
// bytes over the host link depend only on the pass width (the rows of every
// earlier column below a pass cross once per pass); the window of earlier
// columns only sets how many of them one window kernel sums. So the window
// keeps min(4, half) of the columns and the pass takes the rest.
eor_status ooc_plan(int64_t n, int32_t n_k, size_t device_bytes, int32_t lanes, OocPlan &p) {
    p.N = (n + OT - 1) / OT;
    p.n_pad = p.N * OT;
    p.shared_b = (size_t)p.n_pad * sizeof(double2) + (size_t)n * (sizeof(int32_t) + sizeof(double)) +
                 (size_t)n_k * sizeof(double) + 4096;
    p.lane_fixed_b = TILE_B + 2 * (size_t)p.n_pad * sizeof(double2) + (size_t)n_k * sizeof(double) + 1024;
    auto avail_of = [&](int L) -> int64_t {
        if (device_bytes <= p.shared_b) return -1;
        const size_t per = (device_bytes - p.shared_b) / (size_t)L;
        return per < p.lane_fixed_b ? -1 : (int64_t)((per - p.lane_fixed_b) / TILE_B);
    };
    int L = lanes;
    if (lanes == 0) {
        // as many lanes (up to four) as leave each room for 2 min(N, 8)
        // full-height tile columns, and their pinned factors (plus the packed
        // A) within half of the host's physical memory
        L = 1;
        const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGE_SIZE);
        const double host = pages > 0 && page > 0 ? (double)pages * (double)page : 0.0;
        for (int cand = MAX_LANES; cand > 1; --cand) {
            const int64_t av = avail_of(cand);
            const bool fits_host = (double)(cand + 1) * (double)ntiles(p.N) * (double)TILE_B <= 0.5 * host;
            if (av >= 2 * std::min<int64_t>(p.N, 8) * p.N && fits_host) {
                L = cand;
                break;
            }
        }
    } else if (lanes < 1 || lanes > MAX_LANES) {
        return fail_status(EOR_ERR_ARG, "eor_loglike_host: lanes outside 0..4");
    }
    const int64_t avail = avail_of(L);
    if (avail < 2 * p.N) return fail_status(EOR_ERR_OOM, "eor_loglike_host: device_bytes below two columns of tiles per lane");
    p.lanes = L;
    const int64_t cols = avail / p.N;  // >= 2
    p.J = std::min<int64_t>(p.N, cols - std::min<int64_t>(4, cols / 2));
    p.capC = p.J * p.N;
    p.cap = avail - p.capC;  // >= N
    // A once; every earlier column's rows below each pass; and, written back,
    // the rows of a pass's columns that a later pass reads (rows j1 .. N-1)
    int64_t t = ntiles(p.N);
    for (int64_t j0 = 0; j0 < p.N; j0 += p.J) {
        const int64_t j1 = std::min<int64_t>(p.N, j0 + p.J);
        t += j0 * (p.N - j0) + (j1 - j0) * (p.N - j1);
    }
    p.link_bytes = t * (int64_t)TILE_B;
    return EOR_OK;
}

// One lane: a stream, its device buffers and its pinned host factor. The
// destructor waits for the lane's work before anything is freed.
struct OocLane {
    hipStream_t s = nullptr;
    DevBuf<double2> C, Lw, Linv, w, y;
    DevBuf<double> theta, out;
    DevBuf<int32_t> info;
    DevBuf<OocState> st;
    double2 *Lh = nullptr;  // pinned host factor, tile columns packed
    ~OocLane() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        if (Lh) (void)hipHostFree(Lh);
    }
};

template <typename T>
struct PinnedBuf {
    T *p = nullptr;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
};

}  // namespace

}  // namespace eor

extern "C" eor_status eor_loglike_host_plan(int64_t n, int32_t n_k, size_t device_bytes, int32_t lanes,
                                            int32_t *lanes_out, int64_t *cols_per_pass, int64_t *window_tiles,
                                            int64_t *link_bytes) {
    using namespace eor;
    if (n < 1 || n_k < 1 || n > ((int64_t)1 << 22))
        return fail_status(EOR_ERR_ARG, "eor_loglike_host_plan: bad sizes");
    OocPlan p;
    const eor_status r = ooc_plan(n, n_k, device_bytes, lanes, p);
    if (r != EOR_OK) return r;
    if (lanes_out) *lanes_out = p.lanes;
    if (cols_per_pass) *cols_per_pass = p.J;
    if (window_tiles) *window_tiles = p.cap;
    if (link_bytes) *link_bytes = p.link_bytes;
    return EOR_OK;
}

extern "C" eor_status eor_loglike_host(int device, int64_t n, const double *A, int64_t ldA,
                                       const double *dbar, double c, double K0, int32_t n_k,
                                       const int32_t *bin_of, const double *fixed_var, const double *bin_scale,
                                       int64_t B, const double *theta, size_t device_bytes, int32_t lanes,
                                       double *logL, int32_t *info) {
    using namespace eor;
    if (n < 1 || n_k < 1 || B < 0 || ldA < n || !A || !dbar || !bin_of || !fixed_var || (B > 0 && (!theta || !logL)))
        return fail_status(EOR_ERR_ARG, "eor_loglike_host: bad sizes or NULL array");
    if (n > ((int64_t)1 << 22)) return fail_status(EOR_ERR_ARG, "eor_loglike_host: n > 2^22");
    for (int64_t d = 0; d < n; ++d) {
        if (bin_of[d] >= n_k || bin_of[d] < -1) return fail_status(EOR_ERR_ARG, "eor_loglike_host: bin_of out of range");
        if (bin_of[d] < 0 && !(fixed_var[d] > 0.0 && std::isfinite(fixed_var[d])))
            return fail_status(EOR_ERR_ARG, "eor_loglike_host: fixed variance must be positive and finite");
    }
    OocPlan P;
    eor_status r = ooc_plan(n, n_k, device_bytes, lanes, P);
    if (r != EOR_OK) return r;
    if (B == 0) return EOR_OK;
    const int64_t N = P.N, n_pad = P.n_pad, J = P.J, capC = P.capC, cap = P.cap;
    const int S = (int)std::min<int64_t>(P.lanes, B);  // lanes in use
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_status(e, "eor_loglike_host: device");
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev};
    // declared before the lanes, so destroyed after them (the lanes wait for their streams)
    DevBuf<double2> dbar_d;
    DevBuf<int32_t> bin_d;
    DevBuf<double> fix_d, scale_d;
    PinnedBuf<double2> Ah;  // pinned host copy of A, tile columns packed
    PinnedBuf<double> theta_h, out_h;
    PinnedBuf<int32_t> info_h;
    std::unique_ptr<OocLane[]> lane(new OocLane[S]);
    const int64_t ntile = ntiles(N);
    auto col_off = [&](int64_t k) { return k * N - k * (k - 1) / 2; };  // first tile of tile column k
    e = hipMalloc(&dbar_d.p, n_pad * sizeof(double2));
    if (e == hipSuccess) e = hipMalloc(&bin_d.p, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&fix_d.p, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&scale_d.p, n_k * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void **)&Ah.p, (size_t)ntile * TILE_B, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&theta_h.p, (size_t)B * n_k * sizeof(double), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&out_h.p, (size_t)B * sizeof(double), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&info_h.p, (size_t)B * sizeof(int32_t), 0);
    for (int l = 0; l < S && e == hipSuccess; ++l) {
        OocLane &L = lane[l];
        e = hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(&L.C.p, (size_t)capC * TILE_B);
        if (e == hipSuccess) e = hipMalloc(&L.Lw.p, (size_t)cap * TILE_B);
        if (e == hipSuccess) e = hipMalloc(&L.Linv.p, TILE_B);
        if (e == hipSuccess) e = hipMalloc(&L.w.p, n_pad * sizeof(double2));
        if (e == hipSuccess) e = hipMalloc(&L.y.p, n_pad * sizeof(double2));
        if (e == hipSuccess) e = hipMalloc(&L.theta.p, n_k * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&L.out.p, sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&L.info.p, sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&L.st.p, sizeof(OocState));
        if (e == hipSuccess) e = hipHostMalloc((void **)&L.Lh, (size_t)ntile * TILE_B, 0);
    }
    if (e != hipSuccess) return hip_status(e, "eor_loglike_host: allocation");
    // A's lower tiles, zero-padded past n, into the packed host copy: tile
    // columns k = t, t + T, ... on host thread t of T (disjoint tiles)
    const double2 *Asrc = reinterpret_cast<const double2 *>(A);
    auto pack = [&](int64_t first, int64_t step) {
        for (int64_t k = first; k < N; k += step)
            for (int64_t i = k; i < N; ++i) {
                double2 *tile = Ah.p + (col_off(k) + (i - k)) * OT2;
                for (int rr = 0; rr < OT; ++rr) {
                    const int64_t gr = OT * i + rr;
                    double2 *dst = tile + rr * OT;
                    const int64_t cols = std::min<int64_t>(OT, n - OT * k);
                    if (gr < n) {
                        std::copy(Asrc + gr * ldA + OT * k, Asrc + gr * ldA + OT * k + cols, dst);
                        std::fill(dst + cols, dst + OT, make_double2(0.0, 0.0));
                    } else {
                        std::fill(dst, dst + OT, make_double2(0.0, 0.0));
                    }
                }
            }
    };
    {
        const int64_t hc = (int64_t)std::thread::hardware_concurrency();
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(8, N), hc));
        std::vector<std::thread> pool;
        int started = 0;
        try {
            for (int t = 1; t < T; ++t) {
                pool.emplace_back(pack, (int64_t)t, (int64_t)T);
                ++started;
            }
        } catch (...) {
            // a thread that could not start: its share is packed below
        }
        pack(0, T);
        for (int t = started + 1; t < T; ++t) pack(t, T);
        for (auto &th : pool) th.join();
    }
    std::copy(theta, theta + B * n_k, theta_h.p);
    std::vector<double> scale_h(n_k, 1.0);
    if (bin_scale) std::copy(bin_scale, bin_scale + n_k, scale_h.begin());
    hipStream_t s0 = lane[0].s;
    e = hipMemsetAsync(dbar_d.p, 0, n_pad * sizeof(double2), s0);
    if (e == hipSuccess) e = hipMemcpyAsync(dbar_d.p, dbar, n * sizeof(double2), hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipMemcpyAsync(bin_d.p, bin_of, n * sizeof(int32_t), hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipMemcpyAsync(fix_d.p, fixed_var, n * sizeof(double), hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipMemcpyAsync(scale_d.p, scale_h.data(), n_k * sizeof(double), hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipStreamSynchronize(s0);
    if (e != hipSuccess) return hip_status(e, "eor_loglike_host: inputs");

    // theta b on lane b mod S; each lane's theta run in order on its stream,
    // the lanes concurrently
    for (int64_t b = 0; b < B && e == hipSuccess; ++b) {
        OocLane &L = lane[b % S];
        hipStream_t s = L.s;
        e = hipMemcpyAsync(L.theta.p, theta_h.p + b * n_k, n_k * sizeof(double), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(ooc_reset_kernel, dim3(1), dim3(1), 0, s, L.st.p);
        e = hipMemcpyAsync(L.w.p, dbar_d.p, n_pad * sizeof(double2), hipMemcpyDeviceToDevice, s);
        for (int64_t j0 = 0; e == hipSuccess && j0 < N; j0 += J) {
            const int64_t j1 = std::min<int64_t>(N, j0 + J), nt = col_off(j1) - col_off(j0), rows0 = N - j0;
            // tile columns j0 .. j1-1 of A: one contiguous block
            e = hipMemcpyAsync(L.C.p, Ah.p + col_off(j0) * OT2, (size_t)nt * TILE_B, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) break;
            for (int64_t j = j0; j < j1; ++j)
                hipLaunchKernelGGL(ooc_diag_kernel, dim3(1), dim3(OT), 0, s, L.C.p + (col_off(j) - col_off(j0)) * OT2,
                                   j, n, L.theta.p, bin_d.p, fix_d.p, scale_d.p, L.st.p);
            // earlier tile columns, rows j0 .. N-1, in windows of W columns, each read once per pass
            const int64_t W = std::max<int64_t>(1, std::min<int64_t>(j0, cap / rows0));
            for (int64_t k0 = 0; k0 < j0; k0 += W) {
                const int64_t wk = std::min<int64_t>(W, j0 - k0);
                for (int64_t k = 0; k < wk && e == hipSuccess; ++k) {
                    const int64_t kk = k0 + k;
                    e = hipMemcpyAsync(L.Lw.p + k * rows0 * OT2, L.Lh + (col_off(kk) + (j0 - kk)) * OT2,
                                       (size_t)rows0 * TILE_B, hipMemcpyHostToDevice, s);
                }
                if (e != hipSuccess) break;
                hipLaunchKernelGGL(ooc_window_kernel, dim3((unsigned)nt), dim3(256), 0, s, L.C.p, L.Lw.p, (int)wk, j0,
                                   j1, N, L.st.p);
            }
            if (e != hipSuccess) break;
            // the pass's own columns, left to right; each finished column updates
            // the later columns of the pass at once
            for (int64_t j = j0; j < j1; ++j) {
                const int64_t rows = N - j;
                double2 *Cj = L.C.p + (col_off(j) - col_off(j0)) * OT2;
                hipLaunchKernelGGL(ooc_potrf_kernel, dim3(1), dim3(PT), 0, s, Cj, L.Linv.p, L.w.p, L.y.p, j, L.st.p);
                if (rows > 1)
                    hipLaunchKernelGGL(ooc_trsm_kernel, dim3((unsigned)(rows - 1)), dim3(256), 0, s, Cj, L.Linv.p,
                                       L.w.p, L.y.p, j, L.st.p);
                if (j + 1 < j1)
                    hipLaunchKernelGGL(ooc_pass_kernel, dim3((unsigned)(col_off(j1) - col_off(j + 1))), dim3(256), 0,
                                       s, L.C.p, j, j0, j1, N, L.st.p);
            }
            // to the host factor, what later passes read of tile columns j0 .. j1-1:
            // rows j1 .. N-1 of each (none after the last pass; the rows above j1
            // were only ever needed inside this pass)
            for (int64_t j = j0; j < j1 && j1 < N && e == hipSuccess; ++j)
                e = hipMemcpyAsync(L.Lh + (col_off(j) + (j1 - j)) * OT2,
                                   L.C.p + (col_off(j) - col_off(j0) + (j1 - j)) * OT2, (size_t)(N - j1) * TILE_B,
                                   hipMemcpyDeviceToHost, s);
        }
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(ooc_finish_kernel, dim3(1), dim3(1), 0, s, L.st.p, K0, c, L.out.p, L.info.p);
        e = hipMemcpyAsync(out_h.p + b, L.out.p, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(info_h.p + b, L.info.p, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipGetLastError();
    for (int l = 0; l < S; ++l) {
        const hipError_t e2 = hipStreamSynchronize(lane[l].s);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_status(e, "eor_loglike_host");
    std::copy(out_h.p, out_h.p + B, logL);
    if (info) std::copy(info_h.p, info_h.p + B, info);
    return EOR_OK;
}
