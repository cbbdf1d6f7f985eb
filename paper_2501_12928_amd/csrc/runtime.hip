// Multi-instance runtime: many theta of many datasets of uneven size in one
// persistent launch, optionally replayed from a captured HIP graph, with the
// launch choices picked by a timing autotuner whose results persist in a
// small JSON cache keyed by (GPU architecture, size bucket): the launch shape
// for the group, and the side of the factorisation tiles (64 or 32) for each
// bucket of instance sizes, which one launch mixes freely.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

using eor::Context;

struct eor_group {
    int device = 0;
    int num_cu = 0;
    std::vector<eor_ctx *> inst;
    eor::InstDesc *d_inst = nullptr;
    eor::InstDesc *h_inst = nullptr;     // pinned staging
    int2 *d_task = nullptr;
    int64_t ntask = 0;
    std::vector<int64_t> task_B;         // B per instance the task list was built for
    unsigned int *counter = nullptr;
    double2 *Lw = nullptr;
    double2 *yw = nullptr;
    int64_t slots = 0, slot_tiles = 0, slot_y = 0;
    int64_t N_max = 0;
    eor::Tuning tune;
    int ts_bucket[eor::N_BUCKETS] = {64, 64, 64, 64, 64};  // tile side per size bucket of n
    bool use_graph = true;
    // captured graph and what it was captured for
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    eor::LikeParams cap_params;
    int64_t cap_grid = 0;
    int cap_stages = 0;
    int cap_tiles = 0;
    int64_t replays = 0;
    int64_t captures = 0;
    eor::StreamOrder order;              // the last call's work on its stream
};

namespace {

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

void drop_graph(eor_group &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.cap_grid = 0;
}

void free_work(eor_group &g) {
    if (g.Lw) (void)hipFree(g.Lw);
    if (g.yw) (void)hipFree(g.yw);
    g.Lw = nullptr;
    g.yw = nullptr;
    g.slots = 0;
    drop_graph(g);
}

eor_status ensure_work(eor_group &g, int64_t want) {
    if (g.slots >= want && g.slot_tiles == eor::n_tiles(g.N_max)) return EOR_OK;
    // queued work may still use the current slots
    const hipError_t ed = g.order.drain();
    if (ed != hipSuccess) return eor::hip_status(ed, "hipEventSynchronize");
    free_work(g);
    const int64_t slot_tiles = eor::n_tiles(g.N_max);
    const int64_t n_pad = g.N_max * eor::TS;
    int64_t slots = want;
    while (slots >= 1) {
        double2 *Lw = nullptr, *yw = nullptr;
        hipError_t e1 = hipMalloc(&Lw, (size_t)slots * slot_tiles * eor::TS2 * sizeof(double2));
        hipError_t e2 = e1 == hipSuccess ? hipMalloc(&yw, (size_t)slots * n_pad * sizeof(double2)) : e1;
        if (e1 == hipSuccess && e2 == hipSuccess) {
            g.Lw = Lw;
            g.yw = yw;
            g.slots = slots;
            g.slot_tiles = slot_tiles;
            g.slot_y = n_pad;
            return EOR_OK;
        }
        if (Lw) (void)hipFree(Lw);
        if (yw) (void)hipFree(yw);
        (void)hipGetLastError();
        if (slots == 1) break;
        slots /= 2;
    }
    return eor::fail_status(EOR_ERR_OOM, "cannot allocate the group workspace");
}

// Task list: every theta of every instance, longest first (cost ~ N^3), so
// that the persistent workgroups, taking tasks in order, approximate a
// longest-processing-time schedule.
eor_status build_tasks(eor_group &g, const int64_t *B) {
    const int n = (int)g.inst.size();
    std::vector<int64_t> want(B, B + n);
    if (g.d_task && want == g.task_B) return EOR_OK;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return g.inst[a]->c.N > g.inst[b]->c.N; });
    int64_t total = 0;
    for (int64_t b : want) total += b;
    if (total > (int64_t)1 << 30) return eor::fail_status(EOR_ERR_ARG, "more than 2^30 theta in one group call");
    std::vector<int2> tasks;
    for (int i : order)
        for (int64_t b = 0; b < want[i]; ++b) tasks.push_back(make_int2(i, (int)b));
    // queued work may still read the current task list
    const hipError_t ed = g.order.drain();
    if (ed != hipSuccess) return eor::hip_status(ed, "hipEventSynchronize");
    if (g.d_task) (void)hipFree(g.d_task);
    g.d_task = nullptr;
    g.ntask = (int64_t)tasks.size();
    g.task_B = want;
    drop_graph(g);
    if (tasks.empty()) return EOR_OK;
    hipError_t e = hipMalloc(&g.d_task, tasks.size() * sizeof(int2));
    if (e == hipSuccess) e = hipMemcpy(g.d_task, tasks.data(), tasks.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        g.task_B.clear();
        return eor::hip_status(e, "task list");
    }
    return EOR_OK;
}

const char *const kBucketName[eor::N_BUCKETS] = {"n<=512", "n<=1024", "n<=2048", "n<=4096", "n>4096"};

std::string bucket_of(int64_t N) { return kBucketName[eor::bucket_index(N * eor::TS)]; }

std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Cache format: a JSON object of flat entries,
//   "<arch>|<bucket>|<kind>": {"stages": S, "wg_per_cu": W, "tiles": P, "ms": T}
//   "<arch>|<bucket>|tile": {"tile": 32 or 64, "ms64": T64, "ms32": T32}
// read as every "key": {...} pair in the file, whatever its line breaks.
std::map<std::string, std::string> read_cache(const char *path) {
    std::map<std::string, std::string> out;
    std::ifstream f(path);
    const std::string text((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    size_t pos = 0;
    for (;;) {
        const size_t a = text.find('"', pos);
        const size_t b = a == std::string::npos ? a : text.find('"', a + 1);
        const size_t c = b == std::string::npos ? b : text.find_first_not_of(" \t\r\n:", b + 1);
        if (c == std::string::npos) break;
        if (text[c] != '{') {  // not an entry (e.g. a key inside a value): go on after it
            pos = b + 1;
            continue;
        }
        const size_t d = text.find('}', c);
        if (d == std::string::npos) break;
        out[text.substr(a + 1, b - a - 1)] = text.substr(c, d - c + 1);
        pos = d + 1;
    }
    return out;
}

bool parse_entry(const std::string &v, eor::Tuning &t) {
    int s = 0, w = 0, p = 0;
    double ms = 0.0;
    if (std::sscanf(v.c_str(), "{\"stages\": %d, \"wg_per_cu\": %d, \"tiles\": %d, \"ms\": %lf}", &s, &w, &p,
                    &ms) < 3)
        return false;
    if (!eor::valid_tuning(s, w, p)) return false;
    t.stages = s;
    t.wg_per_cu = w;
    t.tiles = p;
    return true;
}

bool write_cache(const char *path, const std::map<std::string, std::string> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t k = 0;
        for (const auto &kv : m) {
            f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
        }
        f << "}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

eor::LikeParams make_params(const eor_group &g, const double *const *theta, double *const *logL,
                            int32_t *const *info) {
    eor::LikeParams p;
    std::memset(&p, 0, sizeof(p));
    p.inst = g.d_inst;
    p.task = g.d_task;
    p.ntask = g.ntask;
    p.counter = g.counter;
    p.Lw = g.Lw;
    p.slot_elems = g.slot_tiles * eor::TS2;
    p.yw = g.yw;
    p.slot_y = g.slot_y;
    for (size_t i = 0; i < g.inst.size(); ++i)
        p.call[i] = eor::CallDesc{theta[i], logL[i], info ? info[i] : nullptr, nullptr};
    return p;
}

// Marks the end of a group call on s, for the group and for each instance
// (whose A the launch reads until then).
eor_status record_call(eor_group &g, hipStream_t s) {
    hipError_t e = g.order.leave(s);
    for (size_t i = 0; i < g.inst.size() && e == hipSuccess; ++i) e = g.inst[i]->c.order.leave(s);
    return e == hipSuccess ? EOR_OK : eor::hip_status(e, "hipEventRecord");
}

// One launch of the whole group (eager or from the captured graph).
eor_status run_group(eor_group &g, const int64_t *B, const double *const *theta, double *const *logL,
                     int32_t *const *info, const eor::Tuning &t, bool allow_graph, hipStream_t s) {
    eor_status st = build_tasks(g, B);
    if (st != EOR_OK) return st;
    if (g.ntask == 0) return EOR_OK;
    int64_t N_max = 0;
    for (auto *c : g.inst) N_max = std::max<int64_t>(N_max, c->c.N);
    if (N_max != g.N_max) {
        free_work(g);
        g.N_max = N_max;
    }
    // The launch waits for the group's previous call and for each instance's
    // last call (a precompute that rewrote A) if they went to other streams.
    hipError_t e = g.order.enter(s);
    for (size_t i = 0; i < g.inst.size() && e == hipSuccess; ++i) e = g.inst[i]->c.order.enter(s);
    if (e != hipSuccess) return eor::hip_status(e, "hipStreamWaitEvent");
    // refresh the instance descriptors (a context may have been re-precomputed),
    // with the tile side of each instance's size bucket
    for (size_t i = 0; i < g.inst.size(); ++i) {
        g.h_inst[i] = eor::inst_desc(g.inst[i]->c);
        g.h_inst[i].ts = g.ts_bucket[eor::bucket_index(g.inst[i]->c.n)];
    }
    e = hipMemcpyAsync(g.d_inst, g.h_inst, g.inst.size() * sizeof(eor::InstDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return eor::hip_status(e, "instance descriptors");
    const int64_t resident = eor::resident_per_cu(t) * g.num_cu;
    const int64_t want = std::min<int64_t>(g.ntask, resident);
    st = ensure_work(g, want);
    if (st != EOR_OK) return st;
    const int64_t grid = std::min<int64_t>(want, g.slots);
    const eor::LikeParams p = make_params(g, theta, logL, info);
    if (!(allow_graph && g.use_graph)) {
        e = eor::launch_likelihood(p, t, grid, s);
        if (e != hipSuccess) return eor::hip_status(e, "group launch");
        return record_call(g, s);
    }
    const bool same = g.exec && g.cap_grid == grid && g.cap_stages == t.stages && g.cap_tiles == t.tiles &&
                      std::memcmp(&g.cap_params, &p, sizeof(p)) == 0;
    if (!same) {
        drop_graph(g);
        if (!g.cap_stream) {
            e = hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return eor::hip_status(e, "capture stream");
        }
        e = hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return eor::hip_status(e, "hipStreamBeginCapture");
        hipError_t el = eor::launch_likelihood(p, t, grid, g.cap_stream);
        e = hipStreamEndCapture(g.cap_stream, &g.graph);
        if (el != hipSuccess) e = el;
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(g);
            return eor::hip_status(e, "graph capture");
        }
        g.cap_params = p;
        g.cap_grid = grid;
        g.cap_stages = t.stages;
        g.cap_tiles = t.tiles;
        ++g.captures;
    }
    e = hipGraphLaunch(g.exec, s);
    if (e != hipSuccess) return eor::hip_status(e, "hipGraphLaunch");
    ++g.replays;
    return record_call(g, s);
}

eor_status check_call(const eor_group *g, const int64_t *B, const double *const *theta, double *const *logL) {
    if (!g) return eor::fail_status(EOR_ERR_ARG, "group is NULL");
    if (!B || !theta || !logL) return eor::fail_status(EOR_ERR_ARG, "NULL argument array");
    for (size_t i = 0; i < g->inst.size(); ++i) {
        if (!g->inst[i]->c.ready) return eor::fail_status(EOR_ERR_STATE, "an instance has no precompute");
        if (B[i] < 0 || B[i] > (int64_t)INT32_MAX) return eor::fail_status(EOR_ERR_ARG, "B out of range");
        if (B[i] > 0 && ((!theta[i] && g->inst[i]->c.n_k > 0) || !logL[i]))
            return eor::fail_status(EOR_ERR_ARG, "NULL theta or logL for a non-empty instance");
    }
    return EOR_OK;
}

}  // namespace

extern "C" {

eor_status eor_group_create(int32_t n_inst, eor_ctx *const *insts, eor_group **out) {
    if (!out) return eor::fail_status(EOR_ERR_ARG, "eor_group_create: out is NULL");
    *out = nullptr;
    if (n_inst < 1 || n_inst > eor::MAX_INST || !insts)
        return eor::fail_status(EOR_ERR_ARG, "eor_group_create: need 1 <= n_inst <= 64 contexts");
    for (int i = 0; i < n_inst; ++i) {
        if (!insts[i]) return eor::fail_status(EOR_ERR_ARG, "eor_group_create: NULL context");
        if (insts[i]->c.device != insts[0]->c.device)
            return eor::fail_status(EOR_ERR_ARG, "eor_group_create: contexts on different devices");
    }
    eor_group *g = new (std::nothrow) eor_group;
    if (!g) return eor::fail_status(EOR_ERR_OOM, "eor_group_create: host allocation failed");
    g->device = insts[0]->c.device;
    g->num_cu = insts[0]->c.num_cu;
    g->inst.assign(insts, insts + n_inst);
    DeviceGuard dg(g->device);
    hipError_t e = hipMalloc(&g->d_inst, n_inst * sizeof(eor::InstDesc));
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->h_inst, n_inst * sizeof(eor::InstDesc));
    if (e == hipSuccess) e = hipMalloc(&g->counter, sizeof(unsigned int));
    if (e != hipSuccess) {
        eor_group_destroy(g);
        return eor::hip_status(e, "eor_group_create");
    }
    *out = g;
    return EOR_OK;
}

void eor_group_destroy(eor_group *g) {
    if (!g) return;
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();
    free_work(*g);
    g->order.destroy();
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    if (g->d_inst) (void)hipFree(g->d_inst);
    if (g->h_inst) (void)hipHostFree(g->h_inst);
    if (g->d_task) (void)hipFree(g->d_task);
    if (g->counter) (void)hipFree(g->counter);
    delete g;
}

eor_status eor_group_loglike(eor_group *g, const int64_t *B, const double *const *theta, double *const *logL,
                             int32_t *const *info, void *stream) {
    eor_status st = check_call(g, B, theta, logL);
    if (st != EOR_OK) return st;
    DeviceGuard dg(g->device);
    // The instance descriptors are staged in pinned memory: wait until the
    // previous launch of this group (on this stream or another) has copied
    // them.
    hipError_t e = g->order.drain();
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return eor::hip_status(e, "hipStreamSynchronize");
    return run_group(*g, B, theta, logL, info, g->tune, true, (hipStream_t)stream);
}

eor_status eor_group_set_graph(eor_group *g, int32_t enable) {
    if (!g) return eor::fail_status(EOR_ERR_ARG, "eor_group_set_graph: group is NULL");
    g->use_graph = enable != 0;
    if (!g->use_graph) drop_graph(*g);
    return EOR_OK;
}

eor_status eor_group_set_tuning(eor_group *g, int32_t stages, int32_t wg_per_cu, int32_t tiles_per_pass) {
    if (!g) return eor::fail_status(EOR_ERR_ARG, "eor_group_set_tuning: group is NULL");
    if (!eor::valid_tuning(stages, wg_per_cu, tiles_per_pass))
        return eor::fail_status(EOR_ERR_ARG, "eor_group_set_tuning: need stages 2|4, and wg_per_cu 1|2 with "
                                             "tiles_per_pass 1, or wg_per_cu 1 with tiles_per_pass 2");
    g->tune.stages = stages;
    g->tune.wg_per_cu = wg_per_cu;
    g->tune.tiles = tiles_per_pass;
    return EOR_OK;
}

eor_status eor_group_set_tile_sizes(eor_group *g, const int32_t *ts_per_bucket) {
    if (!g || !ts_per_bucket) return eor::fail_status(EOR_ERR_ARG, "eor_group_set_tile_sizes: NULL argument");
    for (int b = 0; b < eor::N_BUCKETS; ++b)
        if (ts_per_bucket[b] != 32 && ts_per_bucket[b] != 64)
            return eor::fail_status(EOR_ERR_ARG, "eor_group_set_tile_sizes: each tile side is 32 or 64");
    for (int b = 0; b < eor::N_BUCKETS; ++b) g->ts_bucket[b] = ts_per_bucket[b];
    return EOR_OK;
}

eor_status eor_group_tile_sizes(const eor_group *g, int32_t *ts_per_bucket) {
    if (!g || !ts_per_bucket) return eor::fail_status(EOR_ERR_ARG, "eor_group_tile_sizes: NULL argument");
    for (int b = 0; b < eor::N_BUCKETS; ++b) ts_per_bucket[b] = g->ts_bucket[b];
    return EOR_OK;
}

eor_status eor_group_tuning(const eor_group *g, int32_t *stages, int32_t *wg_per_cu, int32_t *tiles_per_pass,
                            int64_t *graph_launches, int64_t *graph_captures) {
    if (!g) return eor::fail_status(EOR_ERR_ARG, "eor_group_tuning: group is NULL");
    if (stages) *stages = g->tune.stages;
    if (wg_per_cu) *wg_per_cu = g->tune.wg_per_cu;
    if (tiles_per_pass) *tiles_per_pass = g->tune.tiles;
    if (graph_launches) *graph_launches = g->replays;
    if (graph_captures) *graph_captures = g->captures;
    return EOR_OK;
}

eor_status eor_autotune(eor_group *g, const int64_t *B, const double *const *theta, const char *cache_path,
                        int32_t force, void *stream) {
    std::vector<double *> outs;
    {
        // validate with placeholder outputs
        std::vector<double *> fake(g ? g->inst.size() : 0, (double *)1);
        eor_status st = check_call(g, B, theta, fake.data());
        if (st != EOR_OK) return st;
    }
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    const int n_inst = (int)g->inst.size();
    int64_t N_max = 0;
    bool present[eor::N_BUCKETS] = {false, false, false, false, false};
    for (int i = 0; i < n_inst; ++i) {
        N_max = std::max<int64_t>(N_max, g->inst[i]->c.N);
        if (B[i] > 0) present[eor::bucket_index(g->inst[i]->c.n)] = true;
    }
    const std::string arch = arch_name(g->device);
    const std::string key = arch + "|" + bucket_of(N_max) + "|" + (n_inst == 1 ? "single" : "group");
    std::map<std::string, std::string> cache;
    if (cache_path) cache = read_cache(cache_path);
    // cached choices: the launch shape of this group's largest bucket, and
    // the tile side of each bucket it holds
    bool shape_known = false;
    if (!force && cache.count(key)) {
        eor::Tuning t;
        if (parse_entry(cache[key], t)) {
            g->tune = t;
            shape_known = true;
        }
    }
    bool tile_known[eor::N_BUCKETS] = {false, false, false, false, false};
    bool all_known = shape_known;
    for (int b = 0; b < eor::N_BUCKETS; ++b) {
        if (!present[b]) continue;
        const std::string tk = arch + "|" + kBucketName[b] + "|tile";
        int ts = 0;
        if (!force && cache.count(tk) && std::sscanf(cache[tk].c_str(), "{\"tile\": %d", &ts) == 1 &&
            (ts == 32 || ts == 64)) {
            g->ts_bucket[b] = ts;
            tile_known[b] = true;
        }
        all_known = all_known && tile_known[b];
    }
    if (all_known) return EOR_OK;
    // scratch outputs for the timing runs
    hipError_t e = g->order.drain();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return eor::hip_status(e, "hipStreamSynchronize");
    for (int i = 0; i < n_inst; ++i) {
        double *o = nullptr;
        e = hipMalloc(&o, std::max<int64_t>(B[i], 1) * sizeof(double));
        if (e != hipSuccess) {
            for (double *x : outs) (void)hipFree(x);
            return eor::hip_status(e, "autotune outputs");
        }
        outs.push_back(o);
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    eor_status st = EOR_OK;
    // one warm-up launch, then the mean of two timed ones
    auto time_launch = [&](const int64_t *Bv, const eor::Tuning &t) {
        st = run_group(*g, Bv, theta, outs.data(), nullptr, t, false, s);
        float ms_sum = 0.f;
        for (int r = 0; r < 2 && st == EOR_OK; ++r) {
            (void)hipEventRecord(e0, s);
            st = run_group(*g, Bv, theta, outs.data(), nullptr, t, false, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) st = eor::fail_status(EOR_ERR_HIP, "autotune timing");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_sum += ms;
        }
        return ms_sum / 2.0;
    };
    if (!shape_known) {
        eor::Tuning best;
        double best_ms = 1e300;
        const int cand_stages[2] = {4, 2};
        const int cand_shape[3][2] = {{1, 2}, {1, 1}, {2, 1}};  // (tiles per pass, workgroups per CU)
        for (int a = 0; a < 2 && st == EOR_OK; ++a) {
            for (int b = 0; b < 3 && st == EOR_OK; ++b) {
                eor::Tuning t;
                t.stages = cand_stages[a];
                t.tiles = cand_shape[b][0];
                t.wg_per_cu = cand_shape[b][1];
                const double ms = time_launch(B, t);
                if (st == EOR_OK && ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
        if (st == EOR_OK) {
            g->tune = best;
            std::ostringstream v;
            v << "{\"stages\": " << best.stages << ", \"wg_per_cu\": " << best.wg_per_cu << ", \"tiles\": "
              << best.tiles << ", \"ms\": " << best_ms << "}";
            cache[key] = v.str();
        }
    }
    // tile side per bucket, timed on that bucket's instances alone with the
    // chosen launch shape
    std::vector<int64_t> Bsub(n_inst);
    for (int b = 0; b < eor::N_BUCKETS && st == EOR_OK; ++b) {
        if (!present[b] || tile_known[b]) continue;
        for (int i = 0; i < n_inst; ++i) Bsub[i] = eor::bucket_index(g->inst[i]->c.n) == b ? B[i] : 0;
        double ms_ts[2] = {0.0, 0.0};
        const int cand_ts[2] = {64, 32};
        for (int c = 0; c < 2 && st == EOR_OK; ++c) {
            g->ts_bucket[b] = cand_ts[c];
            ms_ts[c] = time_launch(Bsub.data(), g->tune);
        }
        if (st != EOR_OK) break;
        g->ts_bucket[b] = ms_ts[1] < ms_ts[0] ? 32 : 64;
        std::ostringstream v;
        v << "{\"tile\": " << g->ts_bucket[b] << ", \"ms64\": " << ms_ts[0] << ", \"ms32\": " << ms_ts[1] << "}";
        cache[arch + "|" + kBucketName[b] + "|tile"] = v.str();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (double *x : outs) (void)hipFree(x);
    if (st != EOR_OK) return st;
    drop_graph(*g);
    if (cache_path && !write_cache(cache_path, cache))
        return eor::fail_status(EOR_ERR_ARG, std::string("eor_autotune: cannot write ") + cache_path);
    return EOR_OK;
}

}  // extern "C"
