// Internal declarations shared by the HIP sources of libeor.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "eor.h"

namespace eor {

// Side of the square tiles in which A and the Cholesky factor are stored.
constexpr int TS = 64;
constexpr int TS2 = TS * TS;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Packed lower-triangular tile storage: tile (i, j), j <= i, starts at
// tile_index(i, j) * TS2 elements; inside a tile the layout is column-major
// (element (r, c) at c * TS + r). The tiles of tile-row i are therefore
// contiguous, and tile-row i restricted to tiles 0..j-1 is a column-major
// TS x (TS * j) panel with leading dimension TS.
__host__ __device__ inline int64_t tile_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }
__host__ __device__ inline int64_t n_tiles(int64_t N) { return N * (N + 1) / 2; }

void set_error(const std::string &msg);

// Everything the likelihood kernel needs about one dataset (one context).
struct InstDesc {
    const double2 *A;          // packed lower tiles
    const double2 *dbar;       // [n_pad]
    const int32_t *coef_bin;   // [n_pad]: bin, -1 fixed, -2 padding
    const double *coef_inv;    // [n_pad]: 1/v_j of fixed coefficients
    const double *bin_scale;   // [n_k]
    const int32_t *bin_count;  // [n_k]
    const double *scal;        // [2]: c, -sum ln sigma^2
    double khost;              // -m ln(pi)
    double fixed_logv;         // sum over fixed coefficients of ln v_j
    int32_t n_k;
    int32_t N;                 // 64-wide storage tiles per side
    int32_t ts;                // side of the factorisation tiles of L: 64 or 32
};

// Per-call arrays of one instance: theta [B x n_k], logL [B], info [B] or
// NULL, terms [B x 4] or NULL.
struct CallDesc {
    const double *theta;
    double *logL;
    int32_t *info;
    double *terms;
};

// Largest number of instances one launch serves (the per-call table travels
// in the kernel arguments).
constexpr int MAX_INST = 64;

struct LikeParams {
    const InstDesc *inst;         // device [n_inst]
    const int2 *task;             // device [ntask] (instance, theta index), or NULL: (0, t)
    int64_t ntask;                // < 2^31
    unsigned int *counter;        // next task; zeroed by the launch
    double2 *Lw;                  // per-slot packed tiles of L
    int64_t slot_elems;           // complex entries per slot (room for 64-wide tiles)
    double2 *yw;                  // per-slot y
    int64_t slot_y;
    CallDesc call[MAX_INST];
};

// Orders the calls on one handle across streams. A handle's device buffers
// (task counter, workspace slots, A and the tables, surrogate activations)
// are shared by all of its calls, so a call issued on a stream other than the
// previous call's first makes its stream wait for the previous call's work,
// and a call that rewrites what queued work may still read first waits on the
// host. Calls on one stream are ordered by the stream itself.
struct StreamOrder {
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;
    bool pending = false;
    // Before the call's first device work on s.
    hipError_t enter(hipStream_t s) const {
        return (pending && s != last) ? hipStreamWaitEvent(s, ev, 0) : hipSuccess;
    }
    // After the call's last device work on s.
    hipError_t leave(hipStream_t s) {
        if (!ev) {
            const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        const hipError_t e = hipEventRecord(ev, s);
        if (e == hipSuccess) {
            last = s;
            pending = true;
        }
        return e;
    }
    // Block the host until the previous call's device work has finished.
    hipError_t drain() const { return pending ? hipEventSynchronize(ev) : hipSuccess; }
    void destroy() {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
        pending = false;
    }
};

// Launch choices the autotuner picks between.
struct Tuning {
    int stages = 4;      // register prefetch depth of the panel update (2 or 4)
    int wg_per_cu = 1;   // resident workgroups (theta in flight) per CU (1 or 2)
    int tiles = 2;       // workgroups of 4 waves (1) or 8 waves (2, which fills a CU with one
                         // workgroup, so wg_per_cu is then 1); the tiles of a column updated per
                         // pass of its panel are 1 or 2 with 64-wide tiles, 2 or 4 with 32-wide ones
    int ts = 64;         // side of the factorisation tiles (64 or 32) of a lone context
};

// Size buckets of n, for the tile side chosen per bucket: n <= 512, <= 1024,
// <= 2048, <= 4096, larger.
constexpr int N_BUCKETS = 5;
inline int bucket_index(int64_t n) {
    return n <= 512 ? 0 : n <= 1024 ? 1 : n <= 2048 ? 2 : n <= 4096 ? 3 : 4;
}

// State behind an eor_ctx handle.
struct Context {
    int device = 0;
    int num_cu = 0;
    // problem
    bool ready = false;
    int64_t m = 0, n = 0, n_pad = 0, N = 0;
    int32_t n_k = 0;
    double khost = 0.0;          // -m ln(pi)
    double fixed_logv = 0.0;     // sum over fixed coefficients of ln v_j
    double2 *A = nullptr;        // packed lower tiles, n_tiles(N) * TS2
    double2 *dbar = nullptr;     // [n_pad], zero-padded
    double *scal = nullptr;      // device [2]: c, -sum ln sigma_i^2
    int32_t *coef_bin = nullptr; // [n_pad]: bin, -1 fixed, -2 padding
    double *coef_inv = nullptr;  // [n_pad]: 1/v_j for fixed coefficients, else 0
    double *bin_scale = nullptr; // [n_k]
    int32_t *bin_count = nullptr;// [n_k]
    InstDesc *d_inst = nullptr;  // device copy of this dataset's descriptor
    unsigned int *counter = nullptr;
    Tuning tune;
    // precompute temporaries, kept so a repeated precompute needs no allocation
    double *invvar = nullptr;    // [m]
    double2 *partial = nullptr;  // [splits * n]
    int splits = 0;
    // pinned staging of the host-side tables
    int32_t *h_bin = nullptr;
    double *h_inv = nullptr;
    double *h_scale = nullptr;
    int32_t *h_count = nullptr;
    InstDesc *h_inst = nullptr;
    void *lowp = nullptr;        // precompute scratch: FP64 partial tiles, or W in FP32 / split BF16
    size_t lowp_bytes = 0;
    int64_t alloc_m = 0, alloc_n = 0;
    int32_t alloc_k = -1;
    // per-theta workspace: one slot per resident workgroup
    double2 *Lw = nullptr;
    double2 *yw = nullptr;
    int64_t slots = 0;
    int64_t slot_tiles = 0;      // tiles per slot
    int64_t slot_y = 0;          // complex entries of y per slot
    size_t work_limit = 0;       // bytes; 0 = no limit
    int desc_ts = 64;            // tile side in the device copy of the descriptor
    StreamOrder order;           // the last call's work on its stream
};

// Shared helpers of the ABI layer (abi.hip).
eor_status fail_status(eor_status st, const std::string &msg);
eor_status hip_status(hipError_t e, const char *what);
int64_t resident_per_cu(const Tuning &t);
inline bool valid_tuning(int stages, int wg_per_cu, int tiles) {
    return (stages == 2 || stages == 4) &&
           ((tiles == 1 && (wg_per_cu == 1 || wg_per_cu == 2)) || (tiles == 2 && wg_per_cu == 1));
}

// Kernel launchers (precompute.hip, likelihood.hip).
void herk_split(int64_t m, int64_t N, int num_cu, int &splits, int64_t &rows_per);
size_t herk_scratch_bytes(int64_t m, int64_t N, int num_cu);
hipError_t launch_herk_reduce(const double2 *part, int64_t tiles, int splits, int64_t n, double2 *A,
                              hipStream_t s);
hipError_t launch_precompute_fp64(const Context &c, const double2 *T, int64_t ldT,
                                  const double *invvar, void *scratch, hipStream_t s);
size_t lowp_scratch_bytes(eor_precision prec, int64_t m, int64_t n_pad, int num_cu);
hipError_t launch_precompute_fp32(const Context &c, const double2 *T, int64_t ldT,
                                  const double *invvar, void *scratch, hipStream_t s);
hipError_t launch_precompute_bf16(const Context &c, const double2 *T, int64_t ldT,
                                  const double *invvar, void *scratch, int nterm, hipStream_t s);
hipError_t launch_precompute_vectors(const Context &c, const double2 *T, int64_t ldT,
                                     const double *noise_var, const double2 *d, double *invvar,
                                     double2 *partial, int splits, hipStream_t s);
hipError_t launch_export_A(const Context &c, double2 *out, int64_t ldA, hipStream_t s);

int like_max_resident_per_cu(int tiles);
hipError_t launch_likelihood(const LikeParams &p, const Tuning &t, int64_t grid, hipStream_t s);
InstDesc inst_desc(const Context &c);

}  // namespace eor

// The handle behind eor_ctx.
struct eor_ctx {
    eor::Context c;
};
