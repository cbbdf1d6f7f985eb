// Reduced-precision forms of A = W^H W, W = N^{-1/2} T (rows scaled by
// 1/sigma_s), stored in FP64 in the same packed lower tiles as the FP64 path.
//
// FP32: W is formed in FP64 and rounded to complex64; each 64 x 64 tile is a
//   sum of FP32 MFMA (16x16x4) products accumulated in FP32 over chunks of
//   64 rows of W; the chunk partials are added into FP64 accumulators.
// BF16x3: W is formed in FP64, rounded to FP32, and every real and imaginary
//   part x is split into three bfloat16 terms x = h + m + l (+ a remainder
//   below 2^-24 |x|); a real product x y keeps the six leading cross products
//   hh' + hm' + mh' + hl' + mm' + lh' on BF16 MFMA (16x16x32) with FP32
//   accumulation, and again the 64-row chunk partials go to FP64.
// BF16x2: the cheaper split into two terms x = h + l (a remainder below
//   2^-16 |x|) and the three leading products hh' + hl' + lh'.
//
// Both MFMAs return D[4(l/16) + r][l%16] in register r (FP32 16x16x4 and
// BF16 16x16x32), with the A operand lane l = A[l%16][k-group l/16] and the B
// operand lane l = B[k-group l/16][l%16].
#include "common.h"

namespace eor {

namespace {

// Rows of W accumulated in FP32 before the partial goes to FP64. The FP32
// error of a chunk grows with its length (positive diagonal terms make it
// systematic); 64 rows keep logL about ten times closer to FP64 than 256 at
// a negligible cost, and a multiple of 64 is what the split transpose needs.
constexpr int CHUNK_ROWS = 64;

__device__ inline f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

__device__ inline f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline void tile_of(int64_t t, int64_t &i, int64_t &j) {
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    i = r;
    j = t - r * (r + 1) / 2;
}

// Store a tile held as FP64 accumulators: lane holds
// A[64 ti + 16 w + l16][64 tj + 16 cb + 4 q + r].
__device__ inline void store_tile(double2 *__restrict__ Ap, int64_t ti, int64_t tj, int64_t n,
                                  const double (&sR)[4][4], const double (&sI)[4][4], int w, int l16,
                                  int q) {
    double2 *tile = Ap + tile_index(ti, tj) * TS2;
    const int row = 16 * w + l16;
    const int64_t grow = TS * ti + row;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = 16 * cb + 4 * q + r;
            const int64_t gcol = TS * tj + col;
            double2 v = make_double2(sR[cb][r], sI[cb][r]);
            if (grow == gcol) v.y = 0.0;
            if (grow >= n || gcol >= n) v = make_double2(grow == gcol ? 1.0 : 0.0, 0.0);
            tile[col * TS + row] = v;
        }
    }
}

// ---------------------------------------------------------------- FP32 ----

// W32[s][j] = complex64(T[s][j] / sigma_s), zero in the padding.
__global__ void w32_kernel(const double2 *__restrict__ T, int64_t ldT, int64_t m, int64_t n,
                           const double *__restrict__ invvar, int64_t m_pad, int64_t n_pad,
                           float2 *__restrict__ W) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = blockIdx.y;
    if (j >= n_pad) return;
    for (int64_t ss = s; ss < m_pad; ss += gridDim.y) {
        float2 v = make_float2(0.f, 0.f);
        if (ss < m && j < n) {
            const double2 t = T[ss * ldT + j];
            const double sc = sqrt(invvar[ss]);
            v = make_float2((float)(t.x * sc), (float)(t.y * sc));
        }
        W[ss * n_pad + j] = v;
    }
}

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

__device__ inline rsrc_t make_rsrc(const void *p, int64_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)nbytes, 0x00020000);
}

__device__ inline float2 ldf2(rsrc_t r, int voff) {
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
    float2 x;
    __builtin_memcpy(&x, &v, sizeof(x));
    return x;
}

// Operands of one 4-row step of W (row s0 + q in lane group q): the tile-row
// block W[s][64 ti + 16 w + l16] and the four tile-column blocks
// W[s][64 tj + 16 cb + l16].
struct F32Step {
    float2 a;
    float2 b[4];
};

constexpr int F32_STAGES = 4;  // steps in flight; divides the 16 steps of a chunk

// One work unit: tile u % tiles over rows [split * rows_per, ...), split =
// u / tiles, rows_per a multiple of CHUNK_ROWS; W is zero-padded to m_pad
// rows and n_pad columns, so every operand load is unguarded (the prefetch
// past the end of W reads zero through the descriptor). With one split the
// tile goes to A directly; otherwise to its slot of `out` (FP64), and the
// splits are added in a fixed order afterwards.
__global__ __launch_bounds__(256, 2) void herk_fp32_kernel(const float2 *__restrict__ W, int64_t m_pad,
                                                           int64_t n_pad, int64_t n, int64_t tiles,
                                                           int64_t rows_per, int splits,
                                                           double2 *__restrict__ out) {
    const int64_t unit = blockIdx.x;
    const int64_t tile = unit % tiles, split = unit / tiles;
    int64_t ti, tj;
    tile_of(tile, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t r0 = split * rows_per;
    const int64_t r1 = r0 + rows_per < m_pad ? r0 + rows_per : m_pad;
    // D[c][r] = sum_s b[s][c] conj(a[s][r]):  b = W[s][64 tj + c], a = W[s][64 ti + r]
    const int va = (int)((q * n_pad + TS * ti + 16 * w + l16) * 8);
    int vb[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) vb[cb] = (int)((q * n_pad + TS * tj + 16 * cb + l16) * 8);
    auto rows_at = [&](int64_t s) {
        const int64_t left = m_pad - s;
        return make_rsrc(W + (left <= 0 ? 0 : s * n_pad), left <= 0 ? 0 : (left < 4 ? left : 4) * n_pad * 8);
    };
    auto load = [&](F32Step &st, int64_t s) {
        const rsrc_t R = rows_at(s);
        st.a = ldf2(R, va);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) st.b[cb] = ldf2(R, vb[cb]);
    };

    double sR[4][4], sI[4][4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) sR[cb][r] = sI[cb][r] = 0.0;

    F32Step buf[F32_STAGES];
#pragma unroll
    for (int s0 = 0; s0 < F32_STAGES - 1; ++s0) {
        load(buf[s0], r0 + 4 * s0);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t c0 = r0; c0 < r1; c0 += CHUNK_ROWS) {
        __syncthreads();  // keep the four waves together on the shared column block
        f4 aR[4], aI[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) aR[cb] = aI[cb] = f4{0, 0, 0, 0};
        for (int64_t s0 = c0; s0 < c0 + CHUNK_ROWS; s0 += 4 * F32_STAGES) {
#pragma unroll
            for (int u = 0; u < F32_STAGES; ++u) {
                load(buf[(u + F32_STAGES - 1) % F32_STAGES], s0 + 4 * (u + F32_STAGES - 1));
                const F32Step &st = buf[u];
                const float nai = -st.a.y;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    aR[cb] = mfma32(st.b[cb].x, st.a.x, aR[cb]);
                    aR[cb] = mfma32(st.b[cb].y, st.a.y, aR[cb]);
                    aI[cb] = mfma32(st.b[cb].y, st.a.x, aI[cb]);
                    aI[cb] = mfma32(st.b[cb].x, nai, aI[cb]);
                }
            }
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sR[cb][r] += (double)aR[cb][r];
                sI[cb][r] += (double)aI[cb][r];
            }
    }
    if (splits == 1) {
        store_tile(out, ti, tj, n, sR, sI, w, l16, q);
        return;
    }
    // partial tile, column-major: lane holds [16 w + l16][16 cb + 4 q + r]
    double2 *dst = out + (split * tiles + tile) * TS2;
    const int row = 16 * w + l16;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(16 * cb + 4 * q + r) * TS + row] = make_double2(sR[cb][r], sI[cb][r]);
}

// -------------------------------------------------------------- BF16x3 ----

__device__ inline unsigned short bf16_bits(float x) {
    // round to nearest even
    unsigned int u = __float_as_uint(x);
    const unsigned int lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (unsigned short)(u >> 16);
}

__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// Split planes, transposed: plane p (0..5 = re h, m, l, im h, m, l) holds
// P[p][j][s] for s < m_pad (zero in the padding), so eight consecutive rows
// s of one column are 16 contiguous bytes. One block transposes a 64 x 64
// tile of W through LDS.
template <int NTERM>
__global__ __launch_bounds__(256) void split_kernel(const double2 *__restrict__ T, int64_t ldT,
                                                    int64_t m, int64_t n,
                                                    const double *__restrict__ invvar, int64_t m_pad,
                                                    int64_t n_pad, unsigned short *__restrict__ P) {
    __shared__ unsigned short sh[2 * NTERM][64][65];
    const int64_t s0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int rr = ty; rr < 64; rr += 4) {
        const int64_t s = s0 + rr, j = j0 + tx;
        float xr = 0.f, xi = 0.f;
        if (s < m && j < n) {
            const double2 t = T[s * ldT + j];
            const double sc = sqrt(invvar[s]);
            xr = (float)(t.x * sc);
            xi = (float)(t.y * sc);
        }
        const float xs[2] = {xr, xi};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // each term is the bfloat16 nearest what the earlier ones leave
            float x = xs[c];
#pragma unroll
            for (int k = 0; k < NTERM; ++k) {
                const unsigned short b = bf16_bits(x);
                sh[NTERM * c + k][tx][rr] = b;
                x = x - bf16_to_float(b);
            }
        }
    }
    __syncthreads();
    for (int cc = ty; cc < 64; cc += 4) {
        const int64_t j = j0 + cc, s = s0 + tx;
        if (j < n_pad && s < m_pad) {
#pragma unroll
            for (int p = 0; p < 2 * NTERM; ++p) P[((int64_t)p * n_pad + j) * m_pad + s] = sh[p][cc][tx];
        }
    }
}

__device__ inline bf8 ld_bf8(const unsigned short *p) {
    const s8v v = *reinterpret_cast<const s8v *>(p);
    return __builtin_bit_cast(bf8, v);
}

__device__ inline bf8 neg_bf8(bf8 x) {
    s8v v = __builtin_bit_cast(s8v, x);
    v ^= (short)0x8000;
    return __builtin_bit_cast(bf8, v);
}

// The leading products of x y with x and y split into NTERM bfloat16 terms,
// smallest first, term e being x[X[e]] y[Y[e]]: with three terms
// (h, m, l) the six of order at most 2^-16, with two (h, l) the three of
// order at most 2^-8.
template <int NTERM>
struct Prods;
template <>
struct Prods<3> {
    static constexpr int N = 6;
    static constexpr int X[6] = {2, 1, 0, 1, 0, 0};
    static constexpr int Y[6] = {0, 1, 2, 0, 1, 0};
};
template <>
struct Prods<2> {
    static constexpr int N = 3;
    static constexpr int X[3] = {1, 0, 0};
    static constexpr int Y[3] = {0, 1, 0};
};

// One workgroup per 64 x 64 tile; per step of 32 rows the workgroup copies
// both 64-column panels (2 NTERM planes each: 48 KiB for three terms) from
// HBM into LDS once,
// and every wave reads its operands there (each wave needs its own 16
// columns of the row panel and all 64 of the column panel, so reading them
// straight from memory fetched the column panel four times). Two LDS
// buffers: the next step's panels are read into registers while this
// step's are multiplied, and stored after it.
constexpr int BF_COL = 40;  // LDS stride of a column: 32 rows + 8 pad (bf16)

// Work unit u: tile u % tiles over the 32-row steps of rows [split rows_per,
// ...), split = u / tiles (rows_per a multiple of CHUNK_ROWS). With one split
// the tile goes to A; otherwise to its slot of `out` (FP64), and the splits
// are added in a fixed order afterwards.
template <int NTERM>
__global__ __launch_bounds__(256) void herk_bf16_kernel(const unsigned short *__restrict__ P,
                                                        int64_t m_pad, int64_t n_pad, int64_t n, int64_t tiles,
                                                        int64_t rows_per, int splits,
                                                        double2 *__restrict__ out) {
    constexpr int NP = 2 * NTERM;                     // planes: NTERM real, NTERM imaginary
    constexpr int BF_PANEL = NP * 64 * BF_COL;        // one panel, all planes
    constexpr int BF_LOADS = 2 * NP * 64 * 4 / 256;   // 16-byte reads per thread per step (12 or 8)
    using PR = Prods<NTERM>;
    __shared__ __align__(16) unsigned short lds[2][2 * BF_PANEL];
    const int64_t tile = blockIdx.x % tiles, split = blockIdx.x / tiles;
    const int64_t r0 = split * rows_per;
    const int64_t r1 = r0 + rows_per < m_pad ? r0 + rows_per : m_pad;
    int64_t ti, tj;
    tile_of(tile, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, q = lane >> 4;
    const int64_t plane = n_pad * m_pad;
    // the thread's share of a step: 16 bytes (8 rows) of one column of one
    // plane of one panel; e = ((panel * NP + p) * 64 + col) * 4 + 8-row group
    // = tid + 256 u, so read u is plane u % NP of panel u / NP, at the
    // thread's own column and row group. Two column bases per thread and
    // offsets that are uniform per read (the plane), rather than a pointer
    // and an LDS offset per read: fewer registers live through the loop.
    const int g8 = tid & 3, col = (tid >> 2) & 63;
    const unsigned short *base[2] = {P + (TS * ti + col) * m_pad + 8 * g8, P + (TS * tj + col) * m_pad + 8 * g8};
    const int dthr = col * BF_COL + 8 * g8;
    s8v pre[BF_LOADS];
    auto fetch = [&](int64_t s0) {
#pragma unroll
        for (int u = 0; u < BF_LOADS; ++u)
            pre[u] = *reinterpret_cast<const s8v *>(base[u / NP] + (int64_t)(u % NP) * plane + s0);
    };
    auto stash = [&](int b) {
#pragma unroll
        for (int u = 0; u < BF_LOADS; ++u)
            *reinterpret_cast<s8v *>(&lds[b][(u / NP) * BF_PANEL + (u % NP) * 64 * BF_COL + dthr]) = pre[u];
    };
    // B operand a = W[s][64 ti + 16 w + l16] (panel 0), A operands b = W[s][64 tj + 16 cb + l16] (panel 1)
    auto opnd = [&](int b, int panel, int p, int col) {
        return __builtin_bit_cast(bf8, *reinterpret_cast<const s8v *>(
                                           &lds[b][panel * BF_PANEL + (p * 64 + col) * BF_COL + 8 * q]));
    };
    double sR[4][4], sI[4][4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) sR[cb][r] = sI[cb][r] = 0.0;

    fetch(r0);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int64_t c0 = r0; c0 < r1; c0 += CHUNK_ROWS) {
        f4 aR[4], aI[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            aR[cb] = f4{0, 0, 0, 0};
            aI[cb] = f4{0, 0, 0, 0};
        }
        for (int64_t s0 = c0; s0 < c0 + CHUNK_ROWS; s0 += 32) {
            const bool more = s0 + 32 < r1;
            if (more) fetch(s0 + 32);
            bf8 ar[NTERM], ai[NTERM], nai[NTERM];
#pragma unroll
            for (int t = 0; t < NTERM; ++t) {
                ar[t] = opnd(buf, 0, t, 16 * w + l16);
                ai[t] = opnd(buf, 0, NTERM + t, 16 * w + l16);
                nai[t] = neg_bf8(ai[t]);
            }
            // re: br ar + bi ai;  im: bi ar - br ai. Two 16-column blocks at a
            // time, the products of their four accumulators issued in turn so
            // that no product waits on the one before it; each accumulator
            // still takes its twelve products in the same order
#pragma unroll
            for (int cp = 0; cp < 4; cp += 2) {
                bf8 br[2][NTERM], bi[2][NTERM];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int t = 0; t < NTERM; ++t) {
                        br[h][t] = opnd(buf, 1, t, 16 * (cp + h) + l16);
                        bi[h][t] = opnd(buf, 1, NTERM + t, 16 * (cp + h) + l16);
                    }
#pragma unroll
                for (int e = 0; e < PR::N; ++e)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        aR[cp + h] = mfma_bf16(br[h][PR::X[e]], ar[PR::Y[e]], aR[cp + h]);
                        aI[cp + h] = mfma_bf16(bi[h][PR::X[e]], ar[PR::Y[e]], aI[cp + h]);
                    }
#pragma unroll
                for (int e = 0; e < PR::N; ++e)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        aR[cp + h] = mfma_bf16(bi[h][PR::X[e]], ai[PR::Y[e]], aR[cp + h]);
                        aI[cp + h] = mfma_bf16(br[h][PR::X[e]], nai[PR::Y[e]], aI[cp + h]);
                    }
            }
            if (more) stash(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sR[cb][r] += (double)aR[cb][r];
                sI[cb][r] += (double)aI[cb][r];
            }
    }
    if (splits == 1) {
        store_tile(out, ti, tj, n, sR, sI, w, l16, q);
        return;
    }
    // partial tile, column-major: lane holds [16 w + l16][16 cb + 4 q + r]
    double2 *pt = out + (split * tiles + tile) * TS2;
    const int row = 16 * w + l16;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) pt[(16 * cb + 4 * q + r) * TS + row] = make_double2(sR[cb][r], sI[cb][r]);
}

}  // namespace

// Row slices of the FP32 product: herk_split's choice, in whole chunks.
void fp32_split(int64_t m_pad, int64_t N, int num_cu, int &splits, int64_t &rows_per) {
    herk_split(m_pad, N, num_cu, splits, rows_per);
    rows_per = (rows_per + CHUNK_ROWS - 1) / CHUNK_ROWS * CHUNK_ROWS;
}

// Row slices of the split-BF16 product. Its workgroups hold 120 KiB of LDS,
// one per CU, so a round is num_cu units; the slices (whole chunks) are
// chosen to minimise the chunk steps of the busiest CU, rounds x chunks per
// slice, each extra slice counted as half a chunk step per unit for its
// partial tile and its share of the reduction.
void bf16_split(int64_t m_pad, int64_t N, int num_cu, int &splits, int64_t &rows_per) {
    const int64_t tiles = n_tiles(N), slots = num_cu > 0 ? num_cu : 1, chunks = m_pad / CHUNK_ROWS;
    splits = 1;
    double best = 1e300;
    for (int sp = 1; sp <= 8 && sp <= chunks; ++sp) {
        const int64_t per = (chunks + sp - 1) / sp;
        if ((sp - 1) * per >= chunks) continue;  // no empty slice
        const int64_t rounds = (tiles * sp + slots - 1) / slots;
        const double cost = (double)rounds * (double)per + (sp > 1 ? 0.5 * (double)rounds : 0.0);
        if (cost < best - 1e-9) {
            best = cost;
            splits = sp;
        }
    }
    rows_per = (chunks + splits - 1) / splits * CHUNK_ROWS;
}

size_t lowp_scratch_bytes(eor_precision prec, int64_t m, int64_t n_pad, int num_cu) {
    const int64_t m_pad = (m + CHUNK_ROWS - 1) / CHUNK_ROWS * CHUNK_ROWS;
    if (prec == EOR_PREC_FP32) {
        int splits;
        int64_t rows_per;
        fp32_split(m_pad, n_pad / TS, num_cu, splits, rows_per);
        const size_t part = splits > 1 ? (size_t)splits * n_tiles(n_pad / TS) * TS2 * sizeof(double2) : 0;
        return (size_t)m_pad * n_pad * sizeof(float2) + part;
    }
    if (prec == EOR_PREC_BF16X3 || prec == EOR_PREC_BF16X2) {
        int splits;
        int64_t rows_per;
        bf16_split(m_pad, n_pad / TS, num_cu, splits, rows_per);
        const size_t part = splits > 1 ? (size_t)splits * n_tiles(n_pad / TS) * TS2 * sizeof(double2) : 0;
        return (size_t)(prec == EOR_PREC_BF16X3 ? 6 : 4) * m_pad * n_pad * sizeof(unsigned short) + part;
    }
    return 0;
}

hipError_t launch_precompute_fp32(const Context &c, const double2 *T, int64_t ldT, const double *invvar,
                                  void *scratch, hipStream_t s) {
    const int64_t m_pad = (c.m + CHUNK_ROWS - 1) / CHUNK_ROWS * CHUNK_ROWS;
    float2 *W = (float2 *)scratch;
    const unsigned gy = (unsigned)(m_pad < 65535 ? m_pad : 65535);
    hipLaunchKernelGGL(w32_kernel, dim3((unsigned)((c.n_pad + 255) / 256), gy), dim3(256), 0, s, T, ldT,
                       c.m, c.n, invvar, m_pad, c.n_pad, W);
    int splits;
    int64_t rows_per;
    fp32_split(m_pad, c.N, c.num_cu, splits, rows_per);
    const int64_t tiles = n_tiles(c.N);
    double2 *part = splits > 1 ? (double2 *)((char *)scratch + (size_t)m_pad * c.n_pad * sizeof(float2)) : c.A;
    hipLaunchKernelGGL(herk_fp32_kernel, dim3((unsigned)(tiles * splits)), dim3(256), 0, s, W, m_pad, c.n_pad,
                       c.n, tiles, rows_per, splits, part);
    if (splits > 1) return launch_herk_reduce(part, tiles, splits, c.n, c.A, s);
    return hipGetLastError();
}

hipError_t launch_precompute_bf16(const Context &c, const double2 *T, int64_t ldT, const double *invvar,
                                  void *scratch, int nterm, hipStream_t s) {
    const int64_t m_pad = (c.m + CHUNK_ROWS - 1) / CHUNK_ROWS * CHUNK_ROWS;
    unsigned short *P = (unsigned short *)scratch;
    const dim3 sgrid((unsigned)(c.n_pad / 64), (unsigned)(m_pad / 64));
    const int64_t tiles = n_tiles(c.N);
    int splits;
    int64_t rows_per;
    bf16_split(m_pad, c.N, c.num_cu, splits, rows_per);
    double2 *part = splits > 1 ? (double2 *)((char *)scratch + (size_t)(2 * nterm) * m_pad * c.n_pad *
                                                                 sizeof(unsigned short))
                               : c.A;
    const dim3 hgrid((unsigned)(tiles * splits));
    if (nterm == 3) {
        hipLaunchKernelGGL(split_kernel<3>, sgrid, dim3(256), 0, s, T, ldT, c.m, c.n, invvar, m_pad, c.n_pad, P);
        hipLaunchKernelGGL(herk_bf16_kernel<3>, hgrid, dim3(256), 0, s, P, m_pad, c.n_pad, c.n, tiles, rows_per,
                           splits, part);
    } else {
        hipLaunchKernelGGL(split_kernel<2>, sgrid, dim3(256), 0, s, T, ldT, c.m, c.n, invvar, m_pad, c.n_pad, P);
        hipLaunchKernelGGL(herk_bf16_kernel<2>, hgrid, dim3(256), 0, s, P, m_pad, c.n_pad, c.n, tiles, rows_per,
                           splits, part);
    }
    if (splits > 1) return launch_herk_reduce(part, tiles, splits, c.n, c.A, s);
    return hipGetLastError();
}

}  // namespace eor
