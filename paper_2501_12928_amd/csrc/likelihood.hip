// Per-theta marginal likelihood: assemble Sigma = A + Phi^{-1}(theta), factor
// Sigma = L L^H (blocked complex Cholesky, 64 x 64 tiles), forward-solve
// y = L^{-1} dbar, reduce ln det Sigma = 2 sum ln L_jj and ||y||^2 = dbar^H
// Sigma^{-1} dbar, and combine into logL.
//
// One workgroup (4 waves) owns one theta at a time and walks the tiles of L
// left-looking, column by column:
//
//   for each tile column j:
//     diagonal:  S = sum_{k<j} L_jk L_jk^H (MFMA), z = sum_{k<j} L_jk y_k
//                D = A_jj + diag(Phi^{-1}) - S  -> LDS; Cholesky of D in LDS;
//                in-place triangular inverse Linv = L_jj^{-1} (kept in LDS);
//                y_j = Linv (dbar_j - z)
//     below:     for i > j: X = A_ij - sum_{k<j} L_ik L_jk^H (MFMA)
//                           L_ij = X Linv^H (MFMA, operand from LDS)
//
// The panel updates form each complex product from three real FP64 MFMAs
// (Gauss's trick) instead of four; the TRSM step keeps four.
//
// Every entry of L is written once and read back only as an MFMA operand,
// so Sigma is never materialised: A is read once per theta, tile by tile,
// where the factorisation first needs it. Tile-row i of the packed storage
// is a column-major 64 x 64j panel (leading dimension 64), so both operands
// of the update stream with unit stride.
//
// The FP64 16x16x4 MFMA takes its A operand as lane l -> A[l%16][l/16], its
// B operand as lane l -> B[l/16][l%16], and returns D[l/16 + 4r][l%16] in
// register r. Accumulator layout (wave w owns tile rows 16w..16w+15): for
// column block cb and register r, lane (q = lane/16, l16 = lane%16) holds
// element [16w + l16][16cb + q + 4r]. Register r of block cb is then
// directly the A operand of a 16x16x4 MFMA over columns 16cb + 4r .. +3,
// which is what the TRSM step consumes without any data movement.
#include "common.h"

namespace eor {

namespace {

constexpr int NT = 256;  // threads per workgroup (4 waves of 64)

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Every value that steers a loop or branch containing a barrier is passed
// through readfirstlane, so the compiler sees it as wave-uniform and emits
// scalar branches. Left as per-lane values (they come from LDS or global
// memory), the structurizer may place a barrier inside a per-lane loop and
// different waves then execute different numbers of barriers.
__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Hides a lane-dependent value from loop-invariant code motion, so that the
// compiler forms tile addresses as one lane offset plus constants where they
// are used instead of hoisting one register per address out of the loops.
__device__ inline int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Operands of one k-step (4 consecutive columns k0..k0+3 of the panels).
struct Step {
    double2 p;     // P[16w + l16][k0 + q]
    double2 qv[4]; // Q[16cb + l16][k0 + q]
};

// The register prefetch depth of the panel update (k-steps in flight) is a
// template parameter; four steps cover HBM latency at two waves per SIMD on
// the large problems, and the autotuner may choose two.

__device__ inline void load_step(Step &s, const double2 *__restrict__ pp, const double2 *__restrict__ qp,
                                 int64_t k0) {
    s.p = pp[k0 * TS];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) s.qv[cb] = qp[k0 * TS + 16 * cb];
}

// acc[i][c] += P[i][k] conj(Q[c][k]) with three real products per complex
// product (Gauss):  with p = P, q = Q,
//   T1 = qr pr,  T2 = qi pi,  T3 = (qr - qi)(pr + pi)
//   re = T1 + T2,  im = T3 - T1 + T2  (= qr pi - qi pr)
__device__ inline void mma_step(const Step &s, d4 t1[4], d4 t2[4], d4 t3[4]) {
    const double ps = s.p.x + s.p.y;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        t1[cb] = mfma64(s.qv[cb].x, s.p.x, t1[cb]);
        t2[cb] = mfma64(s.qv[cb].y, s.p.y, t2[cb]);
        t3[cb] = mfma64(s.qv[cb].x - s.qv[cb].y, ps, t3[cb]);
    }
}

// S = P Q^H over K columns (K a multiple of 64), returned as (accR, accI).
// With WITHZ, also the partial z[i] = sum_k P[i][k] y[k] of the forward
// substitution. The four waves re-align once per 64 columns so that the
// column panel Q, which all of them read, is fetched from HBM once.
template <bool WITHZ, int STAGES>
__device__ inline void panel_update(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                    const double2 *__restrict__ y, int64_t K, int w, int l16, int q,
                                    d4 accR[4], d4 accI[4], double &zr, double &zi) {
    d4 t3[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        accR[cb] = d4{0, 0, 0, 0};
        accI[cb] = d4{0, 0, 0, 0};
        t3[cb] = d4{0, 0, 0, 0};
    }
    if (K == 0) return;
    const double2 *pp = P + q * TS + 16 * w + l16;
    const double2 *qp = Q + q * TS + l16;
    Step buf[STAGES];
#pragma unroll
    for (int s0 = 0; s0 < STAGES - 1; ++s0) load_step(buf[s0], pp, qp, 4 * s0);
    for (int64_t k0 = 0; k0 < K; k0 += 4 * STAGES) {
        if ((k0 & (TS - 1)) == 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < STAGES; ++u) {
            const int64_t kl = k0 + 4 * (u + STAGES - 1);
            if (kl < K) load_step(buf[(u + STAGES - 1) % STAGES], pp, qp, kl);
            if (WITHZ) {
                const double2 yk = y[k0 + 4 * u + q];
                zr += buf[u].p.x * yk.x - buf[u].p.y * yk.y;
                zi += buf[u].p.x * yk.y + buf[u].p.y * yk.x;
            }
            mma_step(buf[u], accR, accI, t3);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const d4 a = accR[cb], b = accI[cb];
        accR[cb] = a + b;
        accI[cb] = t3[cb] - a + b;
    }
}

template <int STAGES>
__global__ __launch_bounds__(NT, 2) void likelihood_kernel(LikeParams a) {
    __shared__ double2 Dt[TS2];   // diagonal tile: D, then L_jj, then L_jj^{-1}
    __shared__ double2 wv[TS];    // dbar_j - z, then y_j
    __shared__ double dg[TS];     // pivots of the current diagonal tile
    __shared__ double red[TS];    // |y_j|^2 per row
    __shared__ int task_sh;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    double2 *L = a.Lw + (int64_t)blockIdx.x * a.slot_tiles * TS2;
    double2 *yv = a.yw + (int64_t)blockIdx.x * a.slot_y;

    // Persistent workgroup: take tasks in list order (the host sorts them
    // longest first) until the list is exhausted.
    for (;;) {
        if (tid == 0) task_sh = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int t = uniform(task_sh);
        __syncthreads();
        if (t >= a.ntask) break;
        int inst = 0;
        int64_t bt = t;
        if (a.task) {
            const int2 td = a.task[t];
            inst = uniform(td.x);
            bt = uniform(td.y);
        }
        const InstDesc I = a.inst[inst];
        const CallDesc C = a.call[inst];
        const int64_t N = I.N;
        const double *th = C.theta + bt * I.n_k;
        // ln det Phi over the binned coefficients, and the theta check.
        bool ok = true;
        double ldp = 0.0;
        for (int b = 0; b < I.n_k; ++b) {
            const double tb = th[b];
            if (!isfinite(tb)) ok = false;
            if (I.bin_count[b] > 0) {
                const double phi = I.bin_scale[b] * exp10(tb);
                if (!(phi > 0.0) || !isfinite(phi)) ok = false;
                ldp += (double)I.bin_count[b] * log(phi);
            }
        }
        // An invalid theta still falls through to the barrier that closes
        // the task: every lane must reconverge there before tid 0 fetches the
        // next task, or the lanes that skip tid 0's stores can be scheduled
        // around the loop on their own and spin on the old task index.
        const bool valid = uniform(ok ? 1 : 0) != 0;
        if (!valid && tid == 0) {
            C.logL[bt] = -INFINITY;
            if (C.info) C.info[bt] = -1;
            if (C.terms) {
                for (int e = 0; e < 4; ++e) C.terms[4 * bt + e] = NAN;
            }
        }

        double logdet = 0.0, quad = 0.0;  // meaningful in thread 0 only
        int failed = 0;

        for (int64_t j = 0; valid && j < N && !failed; ++j) {
            __syncthreads();  // previous column's readers of Dt are done
            const double2 *panel_j = L + tile_index(j, 0) * TS2;

            // ---- diagonal tile --------------------------------------------
            d4 accR[4], accI[4];
            double zr = 0.0, zi = 0.0;
            panel_update<true, STAGES>(panel_j, panel_j, yv, j * TS, w, l16, q, accR, accI, zr, zi);
            {
                const double2 *Ajj = I.A + tile_index(j, j) * TS2;
                const int lo = opaque(q * TS + 16 * w + l16);  // [16w + l16][q], column-major
                const int dq = opaque(l16 - q);                // row == col iff cb == w, 4r == dq
                const int row = 16 * w + l16;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int off = lo + (16 * cb + 4 * r) * TS;
                        double2 v = Ajj[off];
                        v.x -= accR[cb][r];
                        v.y -= accI[cb][r];
                        if (cb == w && dq == 4 * r) {
                            const int64_t g = j * TS + row;
                            const int32_t b = I.coef_bin[g];
                            const double ip = b >= 0 ? 1.0 / (I.bin_scale[b] * exp10(th[b])) : I.coef_inv[g];
                            v.x += ip;
                        }
                        Dt[off] = v;
                    }
                }
                // reduce z over the four lane groups sharing a row
                zr += __shfl_xor(zr, 16);
                zi += __shfl_xor(zi, 16);
                zr += __shfl_xor(zr, 32);
                zi += __shfl_xor(zi, 32);
                if (q == 0) {
                    const double2 db = I.dbar[j * TS + row];
                    wv[row] = make_double2(db.x - zr, db.y - zi);
                }
            }

            // ---- Cholesky of the diagonal tile in LDS (right-looking) -------
            // Column c is left unscaled during the sweep; the update uses
            // D[r][s] -= D[r][c] conj(D[s][c]) / D[c][c].
            {
                const int r = tid & 63, qq = tid >> 6;
                for (int c = 0; c < TS; ++c) {
                    __syncthreads();
                    const double dcc = Dt[c * TS + c].x;
                    if (uniform((!(dcc > 0.0) || !isfinite(dcc)) ? 1 : 0)) {
                        failed = (int)(j * TS + c + 1);
                        break;
                    }
                    if (tid == 0) dg[c] = dcc;
                    if (r > c) {
                        const double2 lrc = Dt[c * TS + r];
                        const double sr = lrc.x / dcc, si = lrc.y / dcc;
                        for (int s = c + 1 + qq; s <= r; s += 4) {
                            const double2 lsc = Dt[c * TS + s];
                            // (sr + i si) * conj(lsc)
                            double2 v = Dt[s * TS + r];
                            v.x -= sr * lsc.x + si * lsc.y;
                            v.y -= si * lsc.x - sr * lsc.y;
                            Dt[s * TS + r] = v;
                        }
                    }
                }
            }
            if (failed) break;
            __syncthreads();
            // scale: L[c][c] = sqrt(d_c), L[r][c] = D[r][c] / sqrt(d_c); zero the upper part
            for (int e = tid; e < TS2; e += NT) {
                const int c = e / TS, r = e % TS;
                double2 v = Dt[e];
                if (r == c) {
                    v = make_double2(sqrt(dg[c]), 0.0);
                } else if (r > c) {
                    const double is = 1.0 / sqrt(dg[c]);
                    v.x *= is;
                    v.y *= is;
                } else {
                    v = make_double2(0.0, 0.0);
                }
                Dt[e] = v;
            }
            if (tid == 0) {
                for (int c = 0; c < TS; ++c) logdet += log(dg[c]);
            }
            __syncthreads();

            // ---- in-place inverse of the lower-triangular L_jj ---------------
            // Columns from the last to the first:
            //   Linv[c][c] = 1 / L[c][c]
            //   Linv[r][c] = -(sum_{k=c+1..r} Linv[r][k] L[k][c]) / L[c][c],  r > c
            for (int c = TS - 1; c >= 0; --c) {
                double2 nv = make_double2(0.0, 0.0);
                const int r = tid;
                const double lcc = Dt[c * TS + c].x;
                if (r < TS && r > c) {
                    double sr = 0.0, si = 0.0;
                    for (int k = c + 1; k <= r; ++k) {
                        const double2 x = Dt[k * TS + r];  // Linv[r][k] (already inverted)
                        const double2 l = Dt[c * TS + k];  // L[k][c]
                        sr += x.x * l.x - x.y * l.y;
                        si += x.x * l.y + x.y * l.x;
                    }
                    nv = make_double2(-sr / lcc, -si / lcc);
                }
                __syncthreads();
                if (r < TS && r > c) Dt[c * TS + r] = nv;
                if (r == c) Dt[c * TS + c] = make_double2(1.0 / lcc, 0.0);
                __syncthreads();
            }

            // ---- y_j = Linv (dbar_j - z) ---------------------------------
            if (tid < TS) {
                const int r = tid;
                double sr = 0.0, si = 0.0;
                for (int c = 0; c <= r; ++c) {
                    const double2 x = Dt[c * TS + r];
                    const double2 u = wv[c];
                    sr += x.x * u.x - x.y * u.y;
                    si += x.x * u.y + x.y * u.x;
                }
                yv[j * TS + r] = make_double2(sr, si);
                red[r] = sr * sr + si * si;
            }
            __syncthreads();
            if (tid == 0) {
                for (int r = 0; r < TS; ++r) quad += red[r];
            }

            // ---- tiles below the diagonal ---------------------------------
            for (int64_t i = j + 1; i < N; ++i) {
                const double2 *panel_i = L + tile_index(i, 0) * TS2;
                panel_update<false, STAGES>(panel_i, panel_j, nullptr, j * TS, w, l16, q, accR, accI, zr, zi);
                const double2 *Aij = I.A + tile_index(i, j) * TS2;
                const int lo = opaque(q * TS + 16 * w + l16);
                // X = A_ij - S, in the accumulator layout
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double2 v = Aij[lo + (16 * cb + 4 * r) * TS];
                        accR[cb][r] = v.x - accR[cb][r];
                        accI[cb][r] = v.y - accI[cb][r];
                    }
                }
                // Y = X Linv^H: Y[i][c'] = sum_c X[i][c] conj(Linv[c'][c]); Linv is
                // lower triangular, so output block cb2 needs column blocks cb <= cb2.
                double2 *Lij = L + tile_index(i, j) * TS2;
                const int lt = opaque(q * TS + l16);            // Linv[l16][q] in LDS
                const int lw = opaque(l16 * TS + 16 * w + q);   // Y[16w + q][l16] in the tile
#pragma unroll
                for (int cb2 = 0; cb2 < 4; ++cb2) {
                    d4 yR = d4{0, 0, 0, 0}, yI = d4{0, 0, 0, 0};
#pragma unroll
                    for (int cb = 0; cb <= cb2; ++cb) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            // Linv[16cb2 + l16][16cb + 4r + q]
                            const double2 lv = Dt[lt + (16 * cb + 4 * r) * TS + 16 * cb2];
                            const double xr = accR[cb][r], xi = accI[cb][r];
                            yR = mfma64(xr, lv.x, yR);
                            yR = mfma64(xi, lv.y, yR);
                            yI = mfma64(xi, lv.x, yI);
                            yI = mfma64(-xr, lv.y, yI);
                        }
                    }
                    // lane holds Y[16w + q + 4r][16cb2 + l16]
#pragma unroll
                    for (int r = 0; r < 4; ++r) Lij[lw + 16 * cb2 * TS + 4 * r] = make_double2(yR[r], yI[r]);
                }
            }
        }

        if (valid && tid == 0) {
            const double c = I.scal[0];
            if (failed) {
                C.logL[bt] = -INFINITY;
                if (C.info) C.info[bt] = failed;
                if (C.terms) {
                    for (int e = 0; e < 4; ++e) C.terms[4 * bt + e] = NAN;
                }
            } else {
                const double ldphi = ldp + I.fixed_logv;
                C.logL[bt] = (I.khost + I.scal[1]) - ldphi - logdet - (c - quad);
                if (C.info) C.info[bt] = 0;
                if (C.terms) {
                    C.terms[4 * bt + 0] = logdet;
                    C.terms[4 * bt + 1] = quad;
                    C.terms[4 * bt + 2] = ldphi;
                    C.terms[4 * bt + 3] = c;
                }
            }
        }
        __syncthreads();  // slot workspace is reused by the next task
    }
}

__global__ void zero_counter_kernel(unsigned int *counter) { *counter = 0u; }

}  // namespace

int like_max_resident_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, likelihood_kernel<4>, NT, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_likelihood(const LikeParams &p, int stages, int64_t grid, hipStream_t s) {
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, p.counter);
    if (stages == 2)
        hipLaunchKernelGGL(likelihood_kernel<2>, dim3((unsigned)grid), dim3(NT), 0, s, p);
    else
        hipLaunchKernelGGL(likelihood_kernel<4>, dim3((unsigned)grid), dim3(NT), 0, s, p);
    return hipGetLastError();
}

}  // namespace eor
