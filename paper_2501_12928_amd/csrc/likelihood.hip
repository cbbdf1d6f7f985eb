// Per-theta marginal likelihood: assemble Sigma = A + Phi^{-1}(theta), factor
// Sigma = L L^H (blocked complex Cholesky, 64 x 64 tiles), forward-solve
// y = L^{-1} dbar, reduce ln det Sigma = 2 sum ln L_jj and ||y||^2 = dbar^H
// Sigma^{-1} dbar, and combine into logL.
//
// One workgroup owns one theta at a time and walks the tiles of L
// left-looking, column by column, with the forward substitution carried
// right-looking alongside (w starts as dbar):
//
//   for each tile column j:
//     diagonal:  D = A_jj + diag(Phi^{-1}) - sum_{k<j} L_jk L_jk^H (MFMA) -> LDS;
//                Cholesky of D in LDS; in-place triangular inverse
//                Linv = L_jj^{-1} (kept in LDS; blocked on 16 x 16 blocks, the
//                blocks below its diagonal on MFMA); y_j = Linv w_j
//     below:     for i > j: X = A_ij - sum_{k<j} L_ik L_jk^H (MFMA)
//                           L_ij = X Linv^H (MFMA, operand from LDS)
//                           w_i -= L_ij y_j
//
// The workgroup is G groups of four waves (G = 1 or 2, the tiles per pass).
// The units of column j are the diagonal tile (unit 0) and the tiles below
// it (unit u = tile j + u); they are dealt to the groups in rounds of G, so
// with G = 2 two tiles are updated at once against one stream of the column
// panel L_j,0..j-1, which the eight waves share through the CU's L1: a
// quarter less HBM traffic than two workgroups on separate thetas. In the
// first round group 1 updates tile j + 1 while group 0 forms the diagonal,
// and holds its accumulators until L_jj^{-1} is ready.
//
// The panel updates and the TRSM form each complex product from three real
// FP64 MFMAs (Gauss's trick) instead of four. A tile's
// accumulators start from A_ij (loaded while the panel prefetch is in
// flight), so the update ends with X itself.
//
// Every entry of L is written once and read back only as an MFMA operand,
// so Sigma is never materialised: A is read once per theta, tile by tile,
// where the factorisation first needs it. Tile-row i of the packed storage
// is a column-major 64 x 64j panel (leading dimension 64), so both operands
// of the update stream with unit stride. Panels and tiles are read through
// raw buffer descriptors built from wave-uniform bases: the k-step offset is
// a scalar register and each lane keeps one 32-bit offset, which leaves the
// vector registers to the accumulators and the prefetch.
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

constexpr int A_COL_BYTES = TS * 16;  // one column of a storage tile of A
constexpr int ALIGN_COLS = 64;        // panel columns between re-alignments of the workgroup's waves

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Every value that steers a loop or branch containing a barrier is passed
// through readfirstlane, so the compiler sees it as wave-uniform and emits
// scalar branches. Left as per-lane values (they come from LDS or global
// memory), the structurizer may place a barrier inside a per-lane loop and
// different waves then execute different numbers of barriers.
__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Hides a lane-dependent value from loop-invariant code motion: addresses
// derived from it are formed where they are used instead of being hoisted
// out of the column loop, where they would stay live (and spill) across
// every tile update.
__device__ inline int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <class T>
__device__ inline T *uniform_ptr(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// Raw buffer over nbytes at p (a wave-uniform address). A load whose vector
// offset (plus instruction offset) is not below nbytes returns zero and
// touches no memory; the scalar offset is not part of that range check, so
// every load keeps its scalar offset inside the buffer whenever nbytes > 0.
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

// Operands of one k-step (4 consecutive columns k0..k0+3 of the panels) for
// a factorisation tile of side S = 16 NCB.
template <int NCB>
struct Step {
    double2 p;       // P[16w + l16][k0 + q]
    double2 qv[NCB]; // Q[16cb + l16][k0 + q]
};

// P's descriptor starts at row 16w, Q's at row 0; voff = (S q + l16) * 16.
template <int NCB>
__device__ inline void load_step(Step<NCB> &s, rsrc_t P, rsrc_t Q, int voff, int soff) {
    s.p = ld2(P, voff, soff);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) s.qv[cb] = ld2(Q, voff + 16 * 16 * cb, soff);
}

// t += P Q^H for one k-step with three real products per complex product
// (Gauss): with p = P, q = Q,
//   T1 = qr pr,  T2 = qi pi,  T3 = (qr - qi)(pr + pi)
//   re = T1 + T2,  im = T3 - T1 + T2  (= qr pi - qi pr)
template <int NCB>
__device__ inline void mma_step(const Step<NCB> &s, d4 t1[NCB], d4 t2[NCB], d4 t3[NCB]) {
    const double ps = s.p.x + s.p.y;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        t1[cb] = mfma64(s.qv[cb].x, s.p.x, t1[cb]);
        t2[cb] = mfma64(s.qv[cb].y, s.p.y, t2[cb]);
        t3[cb] = mfma64(s.qv[cb].x - s.qv[cb].y, ps, t3[cb]);
    }
}

// X = A - P Q^H over K columns (K a multiple of S), returned as (xr, xi) in
// the accumulator layout. The A tile goes straight into the accumulators
// (T1 = 0, T2 = -Re A, T3 = Re A - Im A, so that the final combine gives
// -(S - A)), issued before the panel prefetch so that its latency overlaps
// it. A is read from its 64 x 64 storage tiles (column stride 64 whatever S),
// the panels from L's S x S tiles (column stride S). All waves of the
// workgroup re-align once per 64 columns so that the column panel Q, which
// all of them read, is fetched from HBM once.
template <int S, int STAGES>
__device__ inline void tile_update(rsrc_t A, rsrc_t P, rsrc_t Q, int K, int voff, int voffA, d4 xr[S / 16],
                                   d4 xi[S / 16]) {
    constexpr int NCB = S / 16;
    constexpr int COLB = S * 16;  // one column of an L tile (or panel), bytes
    d4 t1[NCB], t3[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // A[16w + l16][16cb + 4r + q]: column (16cb + 4r + q), row 16w + l16
            const int so = (16 * cb + 4 * r) * A_COL_BYTES;
            xr[cb][r] = ld1(A, voffA, so);
            t3[cb][r] = ld1(A, voffA + 8, so);
        }
    }
    // The last STAGES - 1 prefetch slots of the loop have no step left to
    // load: they reload step K - 4 (a clamp on the scalar offset) and are
    // never used. The loads stay unconditional, since a guarded load would
    // make the compiler's wait counts conservative at the merge and drain the
    // whole prefetch once per loop iteration; and they stay inside the panel,
    // since past it lies tile (i, j), which this unit stores afterwards (no
    // line of it may be cached on the CU before that store).
    // The prologue keeps its program order (sched_barrier): with step 0's
    // loads issued first, the loop's first wait is the same partial count
    // as in every later iteration instead of a full drain.
    Step<NCB> buf[STAGES];
#pragma unroll
    for (int s0 = 0; s0 < STAGES - 1; ++s0) {
        load_step(buf[s0], P, Q, voff, 4 * s0 * COLB);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        t1[cb] = d4{0, 0, 0, 0};
        t3[cb] = xr[cb] - t3[cb];
        xr[cb] = -xr[cb];  // T2
    }
    d4 *t2 = xr;
    for (int k0 = 0; k0 < K; k0 += 4 * STAGES) {
        if ((k0 & (ALIGN_COLS - 1)) == 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < STAGES; ++u) {
            const int kl = min(k0 + 4 * (u + STAGES - 1), K - 4);
            load_step(buf[(u + STAGES - 1) % STAGES], P, Q, voff, kl * COLB);
            mma_step(buf[u], t1, t2, t3);
        }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const d4 a = t1[cb], b = t2[cb];
        xr[cb] = -(a + b);
        xi[cb] = a - b - t3[cb];
    }
}

// Column boundary. Tiles of L and entries of w written in one column are read
// in later columns by other waves of the workgroup. The workgroup-scope
// release and acquire of __syncthreads make that safe only through the CU's
// vector L1, which all waves of the workgroup share: the compiler emits no
// wait for stores and no L1 invalidation for them. Both are made explicit
// here: every wave waits until its own stores have completed (vmcnt(0)), and
// after the barrier an agent-scope acquire drops the CU's L1 (buffer_inv), so
// every later load of L or w misses it and is served from L2, where the
// completed stores are. A line cached before a store to it, whether by this
// task or by the previous task in the same slot, can then never be read.
__device__ inline void column_barrier() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt left at their maximum
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// The barriers of tile_update over K columns, for a group without a tile in
// the current round: every wave of the workgroup must pass the same number.
__device__ inline void panel_barriers(int K) {
    for (int k0 = 0; k0 < K; k0 += ALIGN_COLS) __syncthreads();
}

// LDS of one workgroup, sized for the largest factorisation tile (64).
struct Shared {
    double2 Dt[TS2];                // diagonal tile: D, then L_jj, then L_jj^{-1} (S x S, leading dimension S)
    double2 wv[TS];                 // w_j = dbar_j - sum_{k<j} L_jk y_k
    double2 ys[TS];                 // y_j
    double dg[TS];                  // pivots of the current diagonal tile
    double red[TS];                 // |y_j|^2 per row
    int task_sh;
};

// One theta of one instance, factored in tiles of side S by a workgroup of NW
// waves: groups of S / 16 waves (each wave owning 16 rows of a tile), so
// NW / (S / 16) tiles of a column are updated per pass of its panel.
template <int S, int STAGES, int NW>
__device__ inline void run_task(Shared &sh, double2 *L, double2 *yv, const InstDesc &I, const CallDesc &C,
                                int64_t bt) {
    constexpr int NT = 64 * NW;          // threads of the workgroup
    constexpr int GW = S / 16;           // waves per group
    constexpr int G = NW / GW;           // tiles per pass
    constexpr int NCB = S / 16;          // 16-column blocks of a tile
    constexpr int S2 = S * S;
    constexpr int COLB = S * 16;
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    const int w = uniform((tid >> 6) % GW);    // row slab 16w..16w+15 of the group's tile
    const int grp = uniform((tid >> 6) / GW);  // group within the workgroup
    const int voff = (q * S + l16) * 16;       // lane offset of L panel loads (bytes)
    const int voffA = (q * TS + l16) * 16;     // lane offset of A tile loads (bytes)
    // tiles per side: the instance's N counts 64-wide tiles
    const int N = uniform(I.N) * (TS / S);
    const double2 *Ab = uniform_ptr(I.A);
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
    // w = dbar; read back only after the barrier that opens column 0
    if (valid) {
        for (int e = tid; e < N * S; e += NT) yv[e] = I.dbar[e];
    }

    double logdet = 0.0, quad = 0.0;  // meaningful in thread 0 only
    int failed = 0;

    for (int j = 0; valid && j < N && !failed; ++j) {
        column_barrier();  // previous column's readers of Dt and writers of L and w are done
        const int K = j * S;
        const rsrc_t Qr = make_rsrc(L + tile_index(j, 0) * S2, (int64_t)K * COLB);
        const int units = N - j;  // unit 0: diagonal tile; unit u > 0: tile (j + u, j)

        for (int u0 = 0; u0 < units; u0 += G) {
            const int u = u0 + grp;
            const int i = j + u;
            d4 xr[NCB], xi[NCB];
            if (u < units) {
                // ---- X = A_ij - sum_k L_ik L_jk^H, in the accumulator layout.
                // Tile (i, j) of side S is the block at rows S (i mod m), columns
                // S (j mod m) of A's storage tile (i / m, j / m), m = 64 / S.
                constexpr int M = TS / S;
                const int64_t aoff = tile_index(i / M, j / M) * TS2 + (int64_t)(S * (j % M)) * TS + S * (i % M) + 16 * w;
                const rsrc_t Ar = make_rsrc(Ab + aoff, (int64_t)(tile_index(i / M, j / M) + 1) * TS2 * 16 - aoff * 16);
                const rsrc_t Pr = make_rsrc(L + tile_index(i, 0) * S2 + 16 * w, (int64_t)K * COLB);
                tile_update<S, STAGES>(Ar, Pr, Qr, K, voff, voffA, xr, xi);
            } else {
                panel_barriers(K);  // no tile for this group in the last round
                // Defined on this path too: otherwise the compiler carries the
                // previous round's values across the loop (64 live registers).
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) xr[cb] = xi[cb] = d4{0, 0, 0, 0};
            }
            if (u == 0) {
                // X of the diagonal tile -> LDS (column-major, leading dimension S)
                const int lo = opaque(q * S + 16 * w + l16);  // [16w + l16][q]
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sh.Dt[lo + (16 * cb + 4 * r) * S] = make_double2(xr[cb][r], xi[cb][r]);
                }
                if (tid < S) sh.wv[tid] = yv[(int64_t)j * S + tid];
            }

            if (u0 == 0) {
                const int tid = opaque(threadIdx.x);
                // ---- D = X + diag(Phi^{-1}) ------------------------------------
                __syncthreads();
                if (tid < S) {
                    const int64_t g = (int64_t)j * S + tid;
                    const int32_t b = I.coef_bin[g];
                    const double ip = b >= 0 ? 1.0 / (I.bin_scale[b] * exp10(th[b])) : I.coef_inv[g];
                    sh.Dt[tid * S + tid].x += ip;
                }
                // ---- Cholesky of the diagonal tile in LDS (right-looking)
                // Column c is left unscaled during the sweep; the update uses
                // D[r][s] -= D[r][c] conj(D[s][c]) / D[c][c].
                {
                    const int r = tid % S, qq = tid / S;
                    for (int c = 0; c < S; ++c) {
                        __syncthreads();
                        const double dcc = sh.Dt[c * S + c].x;
                        if (uniform((!(dcc > 0.0) || !isfinite(dcc)) ? 1 : 0)) {
                            failed = j * S + c + 1;
                            break;
                        }
                        if (tid == 0) sh.dg[c] = dcc;
                        if (r > c) {
                            const double2 lrc = sh.Dt[c * S + r];
                            const double sr = lrc.x / dcc, si = lrc.y / dcc;
                            for (int s = c + 1 + qq; s <= r; s += NT / S) {
                                const double2 lsc = sh.Dt[c * S + s];
                                // (sr + i si) * conj(lsc)
                                double2 v = sh.Dt[s * S + r];
                                v.x -= sr * lsc.x + si * lsc.y;
                                v.y -= si * lsc.x - sr * lsc.y;
                                sh.Dt[s * S + r] = v;
                            }
                        }
                    }
                }
                if (failed) break;
                __syncthreads();
                // scale: L[c][c] = sqrt(d_c), L[r][c] = D[r][c] / sqrt(d_c); zero the upper part
                for (int e = tid; e < S2; e += NT) {
                    const int c = e / S, r = e % S;
                    double2 v = sh.Dt[e];
                    if (r == c) {
                        v = make_double2(sqrt(sh.dg[c]), 0.0);
                    } else if (r > c) {
                        const double is = 1.0 / sqrt(sh.dg[c]);
                        v.x *= is;
                        v.y *= is;
                    } else {
                        v = make_double2(0.0, 0.0);
                    }
                    sh.Dt[e] = v;
                }
                if (tid == 0) {
                    for (int c = 0; c < S; ++c) logdet += log(sh.dg[c]);
                }
                __syncthreads();

                // ---- in-place inverse of the lower-triangular L_jj -----
                // Blocked on 16 x 16 blocks (NB of them per side). First every
                // diagonal block is inverted in place, one wave each, row by
                // row: Linv[r][c] = -(sum_{t=c..r-1} L[r][t] Linv[t][c]) / L[r][r]
                // (a wave's LDS accesses run in program order, so each row reads
                // L before the same row's results replace it). Then the block
                // columns from the right: for jb = NB-2 .. 0, every block below
                // the diagonal, Linv_ib,jb = -(sum_{k=jb+1..ib} Linv_ib,k L_k,jb)
                // Linv_jb,jb, one wave each on FP64 MFMA; its first product is
                // formed transposed, so that the accumulators are the first
                // operand of the second. Results wait for a barrier before they
                // replace the L blocks that other waves still read.
                {
                    constexpr int NB = S / 16;
                    const int wv = uniform(tid >> 6), ln = tid & 63, l16 = ln & 15, q = ln >> 4;
                    if (wv < NB && ln < 16) {
                        const int b0 = 16 * wv, cc = ln;
                        sh.Dt[(b0 + cc) * S + b0 + cc] = make_double2(1.0 / sqrt(sh.dg[b0 + cc]), 0.0);
                        for (int r = 1; r < 16; ++r) {
                            double sr = 0.0, si = 0.0;
                            if (r > cc) {
                                for (int t = cc; t < r; ++t) {
                                    const double2 l = sh.Dt[(b0 + t) * S + b0 + r];   // L[r][t]
                                    const double2 v = sh.Dt[(b0 + cc) * S + b0 + t];  // Linv[t][c]
                                    sr += l.x * v.x - l.y * v.y;
                                    si += l.x * v.y + l.y * v.x;
                                }
                                const double f = -1.0 / sqrt(sh.dg[b0 + r]);
                                sh.Dt[(b0 + cc) * S + b0 + r] = make_double2(sr * f, si * f);
                            }
                        }
                    }
                    __syncthreads();
                    for (int jb = NB - 2; jb >= 0; --jb) {
                        const int ib = jb + 1 + wv;
                        const bool mine = uniform(ib < NB ? 1 : 0) != 0;
                        d4 vr = d4{0, 0, 0, 0}, vi = d4{0, 0, 0, 0};
                        if (mine) {
                            // Y^T = sum_k L_k,jb^T Linv_ib,k^T: lane holds Y^T[q + 4r][l16]
                            d4 t1 = d4{0, 0, 0, 0}, t2 = d4{0, 0, 0, 0}, t3 = d4{0, 0, 0, 0};
                            for (int k = jb + 1; k <= ib; ++k) {
#pragma unroll
                                for (int s0 = 0; s0 < 16; s0 += 4) {
                                    const double2 a = sh.Dt[(16 * jb + l16) * S + 16 * k + s0 + q];  // L[16k+s0+q][16jb+l16]
                                    const double2 b = sh.Dt[(16 * k + s0 + q) * S + 16 * ib + l16];  // Linv[16ib+l16][16k+s0+q]
                                    t1 = mfma64(a.x, b.x, t1);
                                    t2 = mfma64(a.y, b.y, t2);
                                    t3 = mfma64(a.x + a.y, b.x + b.y, t3);
                                }
                            }
                            const d4 yr = t1 - t2, yi = t3 - t1 - t2;
                            // Linv_ib,jb = -Y Linv_jb,jb: k-step r takes Y[l16][4r + q] = (yr[r], yi[r])
                            d4 u1 = d4{0, 0, 0, 0}, u2 = d4{0, 0, 0, 0}, u3 = d4{0, 0, 0, 0};
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const double2 b = sh.Dt[(16 * jb + l16) * S + 16 * jb + 4 * r + q];  // Linv_jb,jb[4r+q][l16]
                                u1 = mfma64(yr[r], b.x, u1);
                                u2 = mfma64(yi[r], b.y, u2);
                                u3 = mfma64(yr[r] + yi[r], b.x + b.y, u3);
                            }
                            vr = -(u1 - u2);
                            vi = -(u3 - u1 - u2);
                        }
                        __syncthreads();
                        if (mine) {
                            // lane holds Linv_ib,jb[q + 4r][l16]
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                sh.Dt[(16 * jb + l16) * S + 16 * ib + q + 4 * r] = make_double2(vr[r], vi[r]);
                        }
                        __syncthreads();
                    }
                }

                // ---- y_j = Linv w_j ---------------------------------------
                if (tid < S) {
                    const int r = tid;
                    double sr = 0.0, si = 0.0;
                    for (int c = 0; c <= r; ++c) {
                        const double2 x = sh.Dt[c * S + r];
                        const double2 uu = sh.wv[c];
                        sr += x.x * uu.x - x.y * uu.y;
                        si += x.x * uu.y + x.y * uu.x;
                    }
                    yv[(int64_t)j * S + r] = make_double2(sr, si);
                    sh.ys[r] = make_double2(sr, si);
                    sh.red[r] = sr * sr + si * si;
                }
                __syncthreads();
                if (tid == 0) {
                    for (int r = 0; r < S; ++r) quad += sh.red[r];
                }
            }

            if (u > 0 && u < units) {
                const int lane = opaque(threadIdx.x & 63), l16 = lane & 15, q = lane >> 4;
                // ---- L_ij = X Linv^H; w_i -= L_ij y_j -----------------------
                // Y[i][c'] = sum_c X[i][c] conj(Linv[c'][c]); Linv is lower
                // triangular, so output block cb2 needs column blocks cb <= cb2.
                // The tile is read in later columns only, after column_barrier.
                double2 *Lij = L + tile_index(i, j) * S2 + l16 * S + 16 * w + q;  // Y[16w + q][l16]
                const int lt = q * S + l16;  // Linv[l16][q] in LDS
                double wr[4] = {0, 0, 0, 0}, wi[4] = {0, 0, 0, 0};
#pragma unroll
                for (int cb2 = 0; cb2 < NCB; ++cb2) {
                    // x conj(l) with three real products (Gauss):
                    //   T1 = xr lr, T2 = xi li, T3 = (xr + xi)(lr - li)
                    //   re = T1 + T2, im = xi lr - xr li = T3 - T1 + T2
                    d4 t1 = d4{0, 0, 0, 0}, t2 = d4{0, 0, 0, 0}, t3 = d4{0, 0, 0, 0};
#pragma unroll
                    for (int cb = 0; cb <= cb2; ++cb) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            // Linv[16cb2 + l16][16cb + 4r + q]
                            const double2 lv = sh.Dt[lt + (16 * cb + 4 * r) * S + 16 * cb2];
                            const double ar = xr[cb][r], ai = xi[cb][r];
                            t1 = mfma64(ar, lv.x, t1);
                            t2 = mfma64(ai, lv.y, t2);
                            t3 = mfma64(ar + ai, lv.x - lv.y, t3);
                        }
                    }
                    const d4 yR = t1 + t2, yI = t3 - t1 + t2;
                    // lane holds Y[16w + q + 4r][16cb2 + l16]
                    const double2 yc = sh.ys[16 * cb2 + l16];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Lij[16 * cb2 * S + 4 * r] = make_double2(yR[r], yI[r]);
                        wr[r] += yR[r] * yc.x - yI[r] * yc.y;
                        wi[r] += yR[r] * yc.y + yI[r] * yc.x;
                    }
                }
                // sum over the 16 lanes that share q (the columns), fixed tree
#pragma unroll
                for (int r = 0; r < 4; ++r) {
#pragma unroll
                    for (int m = 8; m >= 1; m >>= 1) {
                        wr[r] += __shfl_xor(wr[r], m);
                        wi[r] += __shfl_xor(wi[r], m);
                    }
                }
                if (l16 == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double2 *p = yv + (int64_t)i * S + 16 * w + q + 4 * r;
                        double2 v = *p;
                        v.x -= wr[r];
                        v.y -= wi[r];
                        *p = v;
                    }
                }
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
}

// Persistent workgroups of NW waves: take (instance, theta) tasks in list
// order (the host sorts them longest first) until the list is exhausted, and
// factor each in the tile side its instance was given (64, or 32).
template <int STAGES, int NW>
__global__ __launch_bounds__(64 * NW, 8 / NW) void likelihood_kernel(LikeParams a) {
    __shared__ Shared sh;
    const int tid = threadIdx.x;
    double2 *L = uniform_ptr(a.Lw + (int64_t)blockIdx.x * a.slot_elems);
    double2 *yv = uniform_ptr(a.yw + (int64_t)blockIdx.x * a.slot_y);
    for (;;) {
        if (tid == 0) sh.task_sh = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int t = uniform(sh.task_sh);
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
        if (uniform(I.ts) == 32)
            run_task<32, STAGES, NW>(sh, L, yv, I, C, bt);
        else
            run_task<64, STAGES, NW>(sh, L, yv, I, C, bt);
        __syncthreads();  // slot workspace is reused by the next task
    }
}

__global__ void zero_counter_kernel(unsigned int *counter) { *counter = 0u; }

}  // namespace

int like_max_resident_per_cu(int tiles) {
    int nb = 0;
    const hipError_t e =
        tiles == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, likelihood_kernel<4, 8>, 512, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, likelihood_kernel<4, 4>, 256, 0);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_likelihood(const LikeParams &p, const Tuning &t, int64_t grid, hipStream_t s) {
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, p.counter);
    const dim3 g((unsigned)grid);
    if (t.tiles == 2) {
        if (t.stages == 2)
            hipLaunchKernelGGL((likelihood_kernel<2, 8>), g, dim3(512), 0, s, p);
        else
            hipLaunchKernelGGL((likelihood_kernel<4, 8>), g, dim3(512), 0, s, p);
    } else {
        if (t.stages == 2)
            hipLaunchKernelGGL((likelihood_kernel<2, 4>), g, dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL((likelihood_kernel<4, 4>), g, dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace eor
