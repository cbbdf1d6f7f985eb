// C ABI of libeor: argument checking, device memory, and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace eor {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

eor_status fail_status(eor_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

eor_status hip_status(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? EOR_ERR_OOM : EOR_ERR_HIP;
}

int64_t resident_per_cu(const Tuning &t) {
    return std::min<int64_t>(t.tiles == 2 ? 1 : t.wg_per_cu, like_max_resident_per_cu(t.tiles));
}

InstDesc inst_desc(const Context &c) {
    InstDesc d;
    d.A = c.A;
    d.dbar = c.dbar;
    d.coef_bin = c.coef_bin;
    d.coef_inv = c.coef_inv;
    d.bin_scale = c.bin_scale;
    d.bin_count = c.bin_count;
    d.scal = c.scal;
    d.khost = c.khost;
    d.fixed_logv = c.fixed_logv;
    d.n_k = c.n_k;
    d.N = (int32_t)c.N;
    d.ts = c.tune.ts;
    return d;
}

}  // namespace eor

using eor::Context;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

eor_status fail(eor_status st, const std::string &msg) {
    eor::set_error(msg);
    return st;
}

eor_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? EOR_ERR_OOM : EOR_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
void free_dev(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_problem(Context &c) {
    free_dev(c.A);
    free_dev(c.dbar);
    free_dev(c.scal);
    free_dev(c.coef_bin);
    free_dev(c.coef_inv);
    free_dev(c.bin_scale);
    free_dev(c.bin_count);
    free_dev(c.invvar);
    free_dev(c.partial);
    free_dev(c.d_inst);
    free_dev(c.counter);
    if (c.h_inst) (void)hipHostFree(c.h_inst);
    c.h_inst = nullptr;
    if (c.lowp) (void)hipFree(c.lowp);
    c.lowp = nullptr;
    c.lowp_bytes = 0;
    if (c.h_bin) (void)hipHostFree(c.h_bin);
    if (c.h_inv) (void)hipHostFree(c.h_inv);
    if (c.h_scale) (void)hipHostFree(c.h_scale);
    if (c.h_count) (void)hipHostFree(c.h_count);
    c.h_bin = nullptr;
    c.h_inv = nullptr;
    c.h_scale = nullptr;
    c.h_count = nullptr;
    c.alloc_m = c.alloc_n = 0;
    c.alloc_k = -1;
    c.ready = false;
}

void free_work(Context &c) {
    free_dev(c.Lw);
    free_dev(c.yw);
    c.slots = 0;
}

// Scoped device switch so every call runs on the context's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Make sure there is workspace for `want` resident workgroups.
eor_status ensure_work(Context &c, int64_t want) {
    if (c.slots >= want) return EOR_OK;
    // queued work may still use the current slots
    const hipError_t ed = c.order.drain();
    if (ed != hipSuccess) return hip_fail(ed, "hipEventSynchronize");
    free_work(c);
    const int64_t slot_tiles = eor::n_tiles(c.N);
    const size_t per_slot = (size_t)slot_tiles * eor::TS2 * sizeof(double2) + (size_t)c.n_pad * sizeof(double2);
    int64_t slots = want;
    if (c.work_limit > 0) {
        const int64_t cap = (int64_t)(c.work_limit / per_slot);
        if (cap < 1) return fail(EOR_ERR_OOM, "workspace limit is below one theta slot");
        if (slots > cap) slots = cap;
    }
    // Back off if the device cannot hold every slot.
    while (slots >= 1) {
        double2 *Lw = nullptr, *yw = nullptr;
        hipError_t e1 = hipMalloc(&Lw, (size_t)slots * slot_tiles * eor::TS2 * sizeof(double2));
        hipError_t e2 = e1 == hipSuccess ? hipMalloc(&yw, (size_t)slots * c.n_pad * sizeof(double2)) : e1;
        if (e1 == hipSuccess && e2 == hipSuccess) {
            c.Lw = Lw;
            c.yw = yw;
            c.slots = slots;
            c.slot_tiles = slot_tiles;
            c.slot_y = c.n_pad;
            return EOR_OK;
        }
        if (Lw) (void)hipFree(Lw);
        if (yw) (void)hipFree(yw);
        (void)hipGetLastError();
        if (slots == 1) break;
        slots = slots / 2;
    }
    return fail(EOR_ERR_OOM, "cannot allocate the per-theta workspace");
}

}  // namespace

extern "C" {

const char *eor_last_error(void) { return eor::g_error.c_str(); }

const char *eor_version(void) { return "eor 0.1 gfx950"; }

eor_status eor_create(int device, eor_ctx **out) {
    if (!out) return fail(EOR_ERR_ARG, "eor_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(EOR_ERR_ARG, "eor_create: no such device");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(EOR_ERR_ARG, std::string("eor_create: built for gfx950, device is ") + prop.gcnArchName);
    eor_ctx *ctx = new (std::nothrow) eor_ctx;
    if (!ctx) return fail(EOR_ERR_OOM, "eor_create: host allocation failed");
    ctx->c.device = device;
    ctx->c.num_cu = prop.multiProcessorCount;
    *out = ctx;
    return EOR_OK;
}

void eor_destroy(eor_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->c.device);
    (void)hipDeviceSynchronize();
    free_problem(ctx->c);
    free_work(ctx->c);
    ctx->c.order.destroy();
    delete ctx;
}

eor_status eor_precompute(eor_ctx *ctx, int64_t m, int64_t n, const void *T, int64_t ldT,
                          const double *noise_var, const void *d, int32_t n_k, const int32_t *bin_of,
                          const double *fixed_var, const double *bin_scale, eor_precision prec,
                          void *stream) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_precompute: ctx is NULL");
    if (m < 1 || m > ((int64_t)1 << 28) || n < 1 || n > 65536)
        return fail(EOR_ERR_ARG, "eor_precompute: need 1 <= m <= 2^28 and 1 <= n <= 65536");
    if (ldT < n) return fail(EOR_ERR_ARG, "eor_precompute: ldT < n");
    if (ldT > ((int64_t)1 << 24)) return fail(EOR_ERR_ARG, "eor_precompute: ldT > 2^24");
    if (!T || !noise_var || !d || !bin_of) return fail(EOR_ERR_ARG, "eor_precompute: NULL array");
    if (n_k < 0 || n_k > 4096) return fail(EOR_ERR_ARG, "eor_precompute: need 0 <= n_k <= 4096");
    if (prec != EOR_PREC_FP64 && prec != EOR_PREC_FP32 && prec != EOR_PREC_BF16X3 && prec != EOR_PREC_BF16X2)
        return fail(EOR_ERR_ARG, "eor_precompute: unknown precision");
    // host-side bin map and constants
    std::vector<int32_t> cnt(n_k > 0 ? n_k : 1, 0);
    double fixed_logv = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const int32_t b = bin_of[j];
        if (b < -1 || b >= n_k) return fail(EOR_ERR_ARG, "eor_precompute: bin_of out of range");
        if (b < 0) {
            if (!fixed_var || !(fixed_var[j] > 0.0) || !std::isfinite(fixed_var[j]))
                return fail(EOR_ERR_ARG, "eor_precompute: fixed_var must be finite and > 0 where bin_of < 0");
            fixed_logv += std::log(fixed_var[j]);
        } else {
            cnt[b]++;
        }
    }
    std::vector<double> scale(n_k > 0 ? n_k : 1, 1.0);
    for (int32_t b = 0; b < n_k; ++b) {
        if (bin_scale) scale[b] = bin_scale[b];
        if (!(scale[b] > 0.0) || !std::isfinite(scale[b]))
            return fail(EOR_ERR_ARG, "eor_precompute: bin_scale must be finite and > 0");
    }

    Context &c = ctx->c;
    DeviceGuard g(c.device);
    hipStream_t s = (hipStream_t)stream;
    // Queued work, on this stream or on the stream of the context's (or a
    // group's) last call, may still read the previous problem's arrays and
    // the pinned staging buffers.
    hipError_t e = c.order.drain();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int64_t N = (n + eor::TS - 1) / eor::TS;
    if (c.alloc_m != m || c.alloc_n != n || c.alloc_k != n_k) {
        free_problem(c);
        if (c.N != N) free_work(c);
    }
    c.ready = false;
    c.m = m;
    c.n = n;
    c.N = N;
    c.n_pad = N * eor::TS;
    c.n_k = n_k;
    c.khost = -(double)m * std::log(kPi);
    c.fixed_logv = fixed_logv;

    const int nk1 = n_k > 0 ? n_k : 1;
#define EOR_TRY(call, what)                      \
    do {                                         \
        hipError_t _e = (call);                  \
        if (_e != hipSuccess) {                  \
            free_problem(c);                     \
            return hip_fail(_e, what);           \
        }                                        \
    } while (0)
    if (c.alloc_n == 0) {
        c.splits = (int)std::min<int64_t>(64, (m + 255) / 256);
        const size_t a_bytes = (size_t)eor::n_tiles(c.N) * eor::TS2 * sizeof(double2);
        EOR_TRY(hipMalloc(&c.A, a_bytes), "hipMalloc A");
        EOR_TRY(hipMalloc(&c.dbar, c.n_pad * sizeof(double2)), "hipMalloc dbar");
        EOR_TRY(hipMalloc(&c.scal, 2 * sizeof(double)), "hipMalloc scalars");
        EOR_TRY(hipMalloc(&c.coef_bin, c.n_pad * sizeof(int32_t)), "hipMalloc bins");
        EOR_TRY(hipMalloc(&c.coef_inv, c.n_pad * sizeof(double)), "hipMalloc fixed");
        EOR_TRY(hipMalloc(&c.bin_scale, nk1 * sizeof(double)), "hipMalloc scales");
        EOR_TRY(hipMalloc(&c.bin_count, nk1 * sizeof(int32_t)), "hipMalloc counts");
        EOR_TRY(hipMalloc(&c.invvar, m * sizeof(double)), "hipMalloc invvar");
        EOR_TRY(hipMalloc(&c.partial, (size_t)c.splits * n * sizeof(double2)), "hipMalloc partial");
        EOR_TRY(hipHostMalloc((void **)&c.h_bin, c.n_pad * sizeof(int32_t)), "hipHostMalloc");
        EOR_TRY(hipHostMalloc((void **)&c.h_inv, c.n_pad * sizeof(double)), "hipHostMalloc");
        EOR_TRY(hipHostMalloc((void **)&c.h_scale, nk1 * sizeof(double)), "hipHostMalloc");
        EOR_TRY(hipHostMalloc((void **)&c.h_count, nk1 * sizeof(int32_t)), "hipHostMalloc");
        EOR_TRY(hipHostMalloc((void **)&c.h_inst, sizeof(eor::InstDesc)), "hipHostMalloc");
        EOR_TRY(hipMalloc(&c.d_inst, sizeof(eor::InstDesc)), "hipMalloc descriptor");
        EOR_TRY(hipMalloc(&c.counter, sizeof(unsigned int)), "hipMalloc counter");
        c.alloc_m = m;
        c.alloc_n = n;
        c.alloc_k = n_k;
    }
    for (int64_t j = 0; j < c.n_pad; ++j) {
        c.h_bin[j] = j < n ? bin_of[j] : -2;
        c.h_inv[j] = (j < n && bin_of[j] < 0) ? 1.0 / fixed_var[j] : 0.0;
    }
    for (int b = 0; b < nk1; ++b) {
        c.h_scale[b] = scale[b];
        c.h_count[b] = cnt[b];
    }
    EOR_TRY(hipMemcpyAsync(c.coef_bin, c.h_bin, c.n_pad * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy bins");
    EOR_TRY(hipMemcpyAsync(c.coef_inv, c.h_inv, c.n_pad * sizeof(double), hipMemcpyHostToDevice, s), "copy fixed");
    EOR_TRY(hipMemcpyAsync(c.bin_scale, c.h_scale, nk1 * sizeof(double), hipMemcpyHostToDevice, s), "copy scales");
    EOR_TRY(hipMemcpyAsync(c.bin_count, c.h_count, nk1 * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy counts");
    *c.h_inst = eor::inst_desc(c);
    c.desc_ts = c.h_inst->ts;
    EOR_TRY(hipMemcpyAsync(c.d_inst, c.h_inst, sizeof(eor::InstDesc), hipMemcpyHostToDevice, s), "copy descriptor");

    const double2 *Td = (const double2 *)T;
    EOR_TRY(eor::launch_precompute_vectors(c, Td, ldT, noise_var, (const double2 *)d, c.invvar, c.partial,
                                           c.splits, s),
            "precompute vectors");
    {
        // precompute scratch: partial tiles of a row-split FP64 product, or W in reduced precision
        const size_t need = prec == EOR_PREC_FP64 ? eor::herk_scratch_bytes(m, N, c.num_cu)
                                                  : eor::lowp_scratch_bytes(prec, m, c.n_pad, c.num_cu);
        if (c.lowp_bytes < need) {
            if (c.lowp) (void)hipFree(c.lowp);
            c.lowp = nullptr;
            c.lowp_bytes = 0;
            EOR_TRY(hipMalloc(&c.lowp, need), "hipMalloc precompute scratch");
            c.lowp_bytes = need;
        }
    }
    if (prec == EOR_PREC_FP64)
        EOR_TRY(eor::launch_precompute_fp64(c, Td, ldT, c.invvar, c.lowp, s), "precompute A (fp64)");
    else if (prec == EOR_PREC_FP32)
        EOR_TRY(eor::launch_precompute_fp32(c, Td, ldT, c.invvar, c.lowp, s), "precompute A (fp32)");
    else if (prec == EOR_PREC_BF16X3)
        EOR_TRY(eor::launch_precompute_bf16(c, Td, ldT, c.invvar, c.lowp, 3, s), "precompute A (bf16x3)");
    else
        EOR_TRY(eor::launch_precompute_bf16(c, Td, ldT, c.invvar, c.lowp, 2, s), "precompute A (bf16x2)");
#undef EOR_TRY
    e = c.order.leave(s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    c.ready = true;
    return EOR_OK;
}

static eor_status loglike_impl(eor_ctx *ctx, int64_t B, const double *theta, double *logL, int32_t *info,
                               double *terms, void *stream) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_loglike_batch: ctx is NULL");
    Context &c = ctx->c;
    if (!c.ready) return fail(EOR_ERR_STATE, "eor_loglike_batch: call eor_precompute first");
    if (B < 0 || B > (int64_t)1 << 30) return fail(EOR_ERR_ARG, "eor_loglike_batch: need 0 <= B <= 2^30");
    if (B == 0) return EOR_OK;
    if ((!theta && c.n_k > 0) || !logL) return fail(EOR_ERR_ARG, "eor_loglike_batch: NULL array");
    DeviceGuard g(c.device);
    const int64_t resident = eor::resident_per_cu(c.tune) * c.num_cu;
    const int64_t want = B < resident ? B : resident;
    eor_status st = ensure_work(c, want);
    if (st != EOR_OK) return st;
    eor::LikeParams p;
    std::memset(&p, 0, sizeof(p));
    p.inst = c.d_inst;
    p.task = nullptr;
    p.ntask = B;
    p.counter = c.counter;
    p.Lw = c.Lw;
    p.slot_elems = c.slot_tiles * eor::TS2;
    p.yw = c.yw;
    p.slot_y = c.slot_y;
    p.call[0] = eor::CallDesc{theta, logL, info, terms};
    const int64_t grid = want < c.slots ? want : c.slots;
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (c.desc_ts != c.tune.ts) {
        // the tile side changed since the descriptor was copied: restage it
        // once the copy and the work that read it have finished
        e = c.order.drain();
        if (e == hipSuccess) {
            *c.h_inst = eor::inst_desc(c);
            e = hipMemcpyAsync(c.d_inst, c.h_inst, sizeof(eor::InstDesc), hipMemcpyHostToDevice, s);
        }
        if (e != hipSuccess) return hip_fail(e, "descriptor");
        c.desc_ts = c.tune.ts;
    }
    e = c.order.enter(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    e = eor::launch_likelihood(p, c.tune, grid, s);
    if (e != hipSuccess) return hip_fail(e, "likelihood launch");
    e = c.order.leave(s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return EOR_OK;
}

eor_status eor_loglike_batch(eor_ctx *ctx, int64_t B, const double *theta, double *logL, int32_t *info,
                             void *stream) {
    return loglike_impl(ctx, B, theta, logL, info, nullptr, stream);
}

eor_status eor_loglike_terms(eor_ctx *ctx, int64_t B, const double *theta, double *logL, int32_t *info,
                             double *terms, void *stream) {
    if (!terms) return fail(EOR_ERR_ARG, "eor_loglike_terms: terms is NULL");
    return loglike_impl(ctx, B, theta, logL, info, terms, stream);
}

eor_status eor_export_precompute(eor_ctx *ctx, void *A_out, int64_t ldA, void *dbar_out, double *scalars,
                                 void *stream) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_export_precompute: ctx is NULL");
    Context &c = ctx->c;
    if (!c.ready) return fail(EOR_ERR_STATE, "eor_export_precompute: call eor_precompute first");
    if (A_out && ldA < c.n) return fail(EOR_ERR_ARG, "eor_export_precompute: ldA < n");
    DeviceGuard g(c.device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = c.order.enter(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    if (A_out) {
        e = eor::launch_export_A(c, (double2 *)A_out, ldA, s);
        if (e != hipSuccess) return hip_fail(e, "export A");
    }
    if (dbar_out) {
        e = hipMemcpyAsync(dbar_out, c.dbar, c.n * sizeof(double2), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "export dbar");
    }
    if (scalars) {
        double sc[2];
        e = hipMemcpyAsync(sc, c.scal, sizeof(sc), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "export scalars");
        scalars[0] = sc[0];
        scalars[1] = c.khost + sc[1];
    }
    e = c.order.leave(s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return EOR_OK;
}

eor_status eor_set_workspace_limit(eor_ctx *ctx, size_t bytes) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_set_workspace_limit: ctx is NULL");
    Context &c = ctx->c;
    DeviceGuard g(c.device);
    if (c.slots > 0) {
        const size_t per_slot = (size_t)c.slot_tiles * eor::TS2 * sizeof(double2) + (size_t)c.slot_y * sizeof(double2);
        if (bytes > 0 && (size_t)c.slots * per_slot > bytes) {
            // the current workspace is over the new limit: free it once the
            // work that uses it has finished; the next call allocates anew
            const hipError_t e = c.order.drain();
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            free_work(c);
        }
    }
    c.work_limit = bytes;
    return EOR_OK;
}

eor_status eor_set_tuning(eor_ctx *ctx, int32_t stages, int32_t wg_per_cu, int32_t tiles_per_pass) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_set_tuning: ctx is NULL");
    if (!eor::valid_tuning(stages, wg_per_cu, tiles_per_pass))
        return fail(EOR_ERR_ARG, "eor_set_tuning: need stages 2|4, and wg_per_cu 1|2 with tiles_per_pass 1, "
                                 "or wg_per_cu 1 with tiles_per_pass 2");
    ctx->c.tune.stages = stages;
    ctx->c.tune.wg_per_cu = wg_per_cu;
    ctx->c.tune.tiles = tiles_per_pass;
    return EOR_OK;
}

eor_status eor_set_tile_size(eor_ctx *ctx, int32_t ts) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_set_tile_size: ctx is NULL");
    if (ts != 32 && ts != 64) return fail(EOR_ERR_ARG, "eor_set_tile_size: the tile side is 32 or 64");
    ctx->c.tune.ts = ts;
    return EOR_OK;
}

eor_status eor_get_tile_size(const eor_ctx *ctx, int32_t *ts) {
    if (!ctx || !ts) return fail(EOR_ERR_ARG, "eor_get_tile_size: NULL argument");
    *ts = ctx->c.tune.ts;
    return EOR_OK;
}

eor_status eor_get_tuning(const eor_ctx *ctx, int32_t *stages, int32_t *wg_per_cu, int32_t *tiles_per_pass) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_get_tuning: ctx is NULL");
    if (stages) *stages = ctx->c.tune.stages;
    if (wg_per_cu) *wg_per_cu = ctx->c.tune.wg_per_cu;
    if (tiles_per_pass) *tiles_per_pass = ctx->c.tune.tiles;
    return EOR_OK;
}

eor_status eor_shape(const eor_ctx *ctx, int64_t *m, int64_t *n, int32_t *n_k) {
    if (!ctx) return fail(EOR_ERR_ARG, "eor_shape: ctx is NULL");
    if (!ctx->c.ready) return fail(EOR_ERR_STATE, "eor_shape: call eor_precompute first");
    if (m) *m = ctx->c.m;
    if (n) *n = ctx->c.n;
    if (n_k) *n_k = ctx->c.n_k;
    return EOR_OK;
}

}  // extern "C"
