"""Benchmark: batched FP64 logL evaluations per second at n = 4096.

One step is one pass of the path over one batch: eor_precompute of
A = T^H N^-1 T, dbar, c from inputs already resident in HBM (T complex128
20000 x 4096, sigma^2, d), then eor_loglike_batch over B = 512 theta (12
k-bins): assemble, batched blocked complex Cholesky, forward solve,
log-determinants and combine. `value` is whole-step throughput
(B * steps / wall time); the roofline object describes the dominant kernel
(the per-theta likelihood kernel), timed with HIP events on the stream it runs
on; the CPU baseline is the FP64 oracle on the host's cores over a bounded
sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 (matrix)
CONFIG_ID = 3               # 20000 x 4096, 12 bins, B = 512
KERNEL_SRCS = [os.path.join(ROOT, "paper_2501_12928_amd", "csrc", f) for f in ("likelihood.hip", "common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "likelihood_n4096_B512_traffic.json")


def flops_per_theta(n: int) -> float:
    """LAPACK complex convention: Cholesky (4/3) n^3 real flops plus the
    forward solve 4 n^2 (8 real flops per complex multiply-add)."""
    return (4.0 / 3.0) * n ** 3 + 4.0 * n ** 2


def kernel_digest() -> str:
    """Hash of the likelihood kernel's code (its source and the header it
    includes) with comments and blank space removed: counters taken on a
    build stay valid across comment edits, and only then."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        src = open(path).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(ln.strip() for ln in src.splitlines() if ln.strip()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def counters_per_launch():
    """(HBM bytes, FP64 MFMA instructions) per likelihood launch from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else (None, None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernel_sha") != kernel_digest():
        return None, None
    return t.get("bytes_per_launch"), t.get("mfma_instructions")


def cpu_baseline(inst, n_rows: int = 2000):
    """The oracle as it stands, on the host's cores, on a bounded sample:
    precompute over the first n_rows rows of T (scaled to all m rows) and
    one theta per core at the full n = 4096."""
    import oracle
    orc = oracle.get()
    cores = os.cpu_count() or 1
    env_threads = os.environ.get("OMP_NUM_THREADS")
    threads = int(env_threads) if env_threads and env_threads.isdigit() else cores
    threads = max(1, min(threads, cores))
    rows = min(n_rows, inst.m)
    t0 = time.perf_counter()
    A, dbar, c, K0 = orc.precompute(inst.T[:rows], inst.noise_var[:rows], inst.d[:rows], nthreads=threads)
    t_pre = (time.perf_counter() - t0) * inst.m / rows
    th = inst.theta[:threads]
    t0 = time.perf_counter()
    orc.loglike(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, th, nthreads=threads)
    t_like = time.perf_counter() - t0
    B = inst.theta.shape[0]
    step_s = t_pre + t_like * (B / th.shape[0])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": B / step_s, "unit": "evals/s", "cores": threads, "kind": "oracle", "cpu_model": model,
            "sample": (f"precompute over {rows} of {inst.m} rows (time scaled x{inst.m / rows:g}) + "
                       f"{th.shape[0]} theta at n={inst.n} in parallel (one per thread), scaled to "
                       f"B={B}; plain C FP64 oracle, OpenMP"),
            "seconds_measured": round(t_pre * rows / inst.m + t_like, 2)}


def cpu_lapack_reference(ctx, inst, per_n=((4096, 2), (2048, 4))):
    """A stronger CPU reference than the oracle (not the baseline): LAPACK's
    blocked Cholesky (scipy, multithreaded BLAS) plus the triangular solve and
    log-determinant, on Sigma = A + Phi^-1 built from the GPU path's exported
    A. Timing only; the n = 2048 case uses A's leading block."""
    import numpy as np
    import scipy.linalg as sl
    try:
        from threadpoolctl import threadpool_info
        blas = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        threads = blas[0]["num_threads"] if blas else None
        lib = f"{blas[0]['internal_api']} {blas[0]['version']}" if blas else "unknown"
    except Exception:
        threads, lib = None, "unknown"
    A, dbar, c, K0 = ctx.export_precompute()
    A = A.cpu().numpy()
    dbar = dbar.cpu().numpy()
    rep = {"kind": "lapack zpotrf + ztrsv via scipy", "blas": lib, "threads": threads, "unit": "evals/s"}
    for n, k in per_n:
        n = min(n, A.shape[0])
        best = []
        for t in range(k):
            th = inst.theta[t]
            b = inst.bin_of[:n]
            phi = np.where(b >= 0, inst.bin_scale[np.maximum(b, 0)] * 10.0 ** th[np.maximum(b, 0)],
                           inst.fixed_var[:n])
            t0 = time.perf_counter()
            S = A[:n, :n].copy()
            S[np.diag_indices(n)] += 1.0 / phi
            L = sl.cholesky(S, lower=True, check_finite=False)
            y = sl.solve_triangular(L, dbar[:n], lower=True, check_finite=False)
            _ = 2.0 * np.sum(np.log(np.real(np.diag(L)))) + np.vdot(y, y).real
            best.append(time.perf_counter() - t0)
        rep[f"n{n}"] = 1.0 / float(np.median(best))
    rep["value"] = rep.get(f"n{min(4096, A.shape[0])}")
    return rep


def precision_report(ctx, inst, T, nv, d, theta, logL64):
    """A in FP32 and in split BF16 against the FP64 A of the same GPU path
    (itself parity-checked against the oracle): relative Frobenius error of
    A, |dlogL| over the batch, and the precompute time of each precision."""
    import torch
    stream = torch.cuda.current_stream()

    def timed_pre(prec):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, prec=prec)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    rep = {"fp64_precompute_ms": timed_pre("fp64")}
    A64 = ctx.export_precompute()[0]
    nrm = torch.linalg.norm(A64).item()
    for prec in ("fp32", "bf16x3", "bf16x2"):
        ms = timed_pre(prec)
        A = ctx.export_precompute()[0]
        rel = (torch.linalg.norm(A - A64).item()) / nrm
        del A
        L, info = ctx.loglike_batch(theta)
        both = (info == 0) & torch.isfinite(logL64)
        dl = (L - logL64).abs()[both]
        rep[prec] = {"rel_frob_A": rel,
                     "max_abs_dlogL": dl.max().item() if dl.numel() else None,
                     "max_rel_dlogL": (dl / logL64.abs()[both]).max().item() if dl.numel() else None,
                     "precompute_ms": ms, "info_nonzero": int((info != 0).sum().item())}
    del A64
    ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, prec="fp64")
    return rep


def bench_group(args):
    """48 independent sub-band instances, n ~ U{256..4096}, T (4n x n),
    16-128 theta and 4-12 bins each: one persistent launch per step (graph
    replay), launch choices from the autotuner."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    ctxs, thetas, flops, ns = [], [], 0.0, []
    t_pre = 0.0
    for inst in synth.gen_group():
        T = torch.from_numpy(inst.T).cuda()
        ctx = eor.Context(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.precompute(T, torch.from_numpy(inst.noise_var).cuda(), torch.from_numpy(inst.d).cuda(),
                       inst.n_k, inst.bin_of, inst.fixed_var)
        torch.cuda.synchronize()
        t_pre += time.perf_counter() - t0
        del T
        ctxs.append(ctx)
        thetas.append(torch.from_numpy(inst.theta).cuda())
        flops += inst.theta.shape[0] * flops_per_theta(inst.n)
        ns.append(inst.n)
    g = eor.Group(ctxs)
    cache = os.environ.get("EOR_TUNE_CACHE", os.path.join("/tmp", "eor_tune.json"))
    stages, wg, tiles = g.autotune(thetas, cache_path=cache, force=True)
    outs, infos = g.loglike(thetas)
    for _ in range(args.warmup):
        outs, infos = g.loglike(thetas, outs=outs, infos=infos)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        outs, infos = g.loglike(thetas, outs=outs, infos=infos)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ok = all(bool((i == 0).all().item()) for i in infos)
    ntheta = sum(t.shape[0] for t in thetas)
    achieved = flops / (ms / 1e3) / 1e12
    print(json.dumps({
        "metric": "logL evals/s, 48 uneven sub-band instances in one persistent launch",
        "value": ntheta * args.steps / wall, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"48 instances, n in [{min(ns)}, {max(ns)}], T (4n x n), {ntheta} theta total",
                   "instances": len(ns), "theta": ntheta},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "kernel": "likelihood_kernel",
                     "launch_ms": ms, "flops_per_launch": flops},
        "tuning": {"stages": stages, "wg_per_cu": wg, "tiles_per_pass": tiles, "graph": list(g.tuning()[3:]),
                   "tile_side_per_bucket": dict(zip(("n<=512", "n<=1024", "n<=2048", "n<=4096", "n>4096"),
                                                    g.tile_sizes())),
                   "tile_timing_ms": {k.split("|")[1]: v for k, v in json.load(open(cache)).items()
                                      if k.endswith("|tile")}},
        "precompute_s_total": t_pre, "all_info_zero": ok}))
    g.close()
    for c in ctxs:
        c.close()


def bench_stress(args):
    """Precision under ill-conditioning (reported, not a metric): T with
    singular values over four decades at 8000 x 2048, with the usual
    foreground share and with a wide-field foreground model (n_fg = 1792 >>
    n_eor = 256). For each, the FP64 path's failures and time, and what FP32
    and split-BF16 A do to positive definiteness and to logL."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    out = {"metric": "precision under ill-conditioned instruments (report)", "n_gpus": 1,
           "dtype": "f64 (A also in f32 and split bf16)", "data": "synthetic", "variants": {}}
    for name in sorted(synth.STRESS):
        print(f"stress: {name}", file=sys.stderr, flush=True)
        inst = synth.gen_stress(name)
        T = torch.from_numpy(inst.T).cuda()
        nv = torch.from_numpy(inst.noise_var).cuda()
        d = torch.from_numpy(inst.d).cuda()
        theta = torch.from_numpy(inst.theta).cuda()
        ctx = eor.Context(0)
        ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale)
        L64, info64 = ctx.loglike_batch(theta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.loglike_batch(theta, out=L64, info=info64)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        rep = precision_report(ctx, inst, T, nv, d, theta, L64.clone())
        rep["fp64_info_nonzero"] = int((info64 != 0).sum().item())
        rep["fp64_loglike_ms"] = ms
        rep["shape"] = {k: v for k, v in synth.STRESS[name].items()}
        out["variants"][name] = rep
        ctx.close()
        del T, nv, d, theta
    print(json.dumps(out))


def gate_settings(args):
    """Surrogate and gate settings of the gated runs, from the command line."""
    import paper_2501_12928_amd as eor
    cfg = eor.train_cfg(epochs=args.train_epochs, minibatch=args.train_minibatch, patience=30, lr=1e-3, seed=5)
    # Warm retraining may run longer than the first training: late in the run
    # the ensemble keeps improving well past 300 epochs. A short one can be
    # worse than none: the members stay close to their common starting
    # point, agree with each other and are wrong together, which the audits
    # show as false rejections.
    rcfg = None if not args.retrain_epochs else eor.train_cfg(
        epochs=args.retrain_epochs, minibatch=args.train_minibatch, patience=30, lr=1e-3, seed=6)
    band = None if args.band_above <= 0 else (args.band_below, args.band_above)
    kw = dict(tau=args.tau, first_train=args.first_train, retrain_every=args.retrain_every, window=args.window,
              margin=args.margin, train_kwargs={"cfg": cfg}, retrain_kwargs=None if rcfg is None else {"cfg": rcfg},
              band=band, reach=args.reach, stale_gap=args.stale_gap, whiten=args.whiten, cold=args.cold, seed=11)
    text = (f"n_live={args.n_live}, gate tau={args.tau}, first training after {args.first_train} exact "
            f"evaluations ({args.train_epochs} epochs), retrain every {args.retrain_every} iterations on the last "
            f"{args.window} ({args.retrain_epochs or args.train_epochs} epochs{'' if args.cold else ', warm'}), "
            + (f"targets censored to [L_min - {args.band_below}, L_min + {args.band_above}] (band re-centred after "
               f"the threshold climbs {args.band_above / 2}, at most every {args.stale_gap} iterations; rejected "
               f"only within {args.reach} of the floor)" if band else f"within {args.margin} of the threshold")
            + (", inputs mapped to the training box" if args.whiten else "")
            + (", every training from fresh weights" if args.cold else "")
            + ", exact calls of 512 proposals the gate is unsure of")
    return kw, text


def gated_pair(ctx, n_k, lo, hi, args, seed=7, progress=2000):
    """The plain and the gated nested-sampling run on one context (same seed),
    and their comparison."""
    import paper_2501_12928_amd as eor
    from paper_2501_12928_amd.sampler import GatedLikelihood, NestedSampler, compare_runs, exact_gpu
    kw, text = gate_settings(args)
    loglike = exact_gpu(ctx)
    plain = NestedSampler(loglike, n_k, lo, hi, n_live=args.n_live, dlogz=0.01, batch=512, seed=seed,
                          progress=progress).run()
    sur = eor.Surrogate(n_k, -1.0 if args.whiten else lo, 1.0 if args.whiten else hi, n_members=5, hidden=256, seed=1)
    gated = NestedSampler(loglike, n_k, lo, hi, n_live=args.n_live, dlogz=0.01, batch=512, seed=seed,
                          gate=GatedLikelihood(sur, **kw), audit_frac=args.audit_frac, pool_factor=args.pool_factor,
                          progress=progress).run()
    sur.close()
    cmp = compare_runs(plain, gated, args.n_live)
    # accepted points carry exact logL: re-evaluate a sample of them
    idx = np.random.default_rng(0).choice(gated.samples.shape[0], 64, replace=False)
    cmp["accepted_max_abs_dlogL"] = float(np.max(np.abs(loglike(gated.samples[idx]) - gated.logl[idx])))
    cmp["accepted_checked"] = 64
    return plain, gated, cmp, text


def gated_leg(ctx, inst, args):
    """The gated half of the headline metric on the benchmark's own dataset:
    plain and surrogate-gated nested sampling with the same seed, both on
    the batched FP64 likelihood (n_live reduced to keep the default run
    short)."""
    import copy
    a = copy.copy(args)
    a.n_live = args.gated_n_live
    a.first_train = max(2000, args.first_train * args.gated_n_live // 500)
    print(f"bench: gated leg, plain and gated nested sampling with {a.n_live} live points", file=sys.stderr,
          flush=True)
    plain, gated, cmp, text = gated_pair(ctx, inst.n_k, inst.lo, inst.hi, a, progress=2000)
    keys = ("proposals_plain", "proposals_gated", "proposals_per_s_plain", "proposals_per_s_gated", "speedup",
            "exact_calls_plain", "exact_calls_gated", "exact_calls_avoided_frac", "logz_plain", "logz_gated",
            "logz_tolerance", "max_dmean_over_sigma", "max_dstd_rel", "gate_rejected", "audited",
            "false_rejections", "accepted_max_abs_dlogL", "accepted_checked", "confident_checked",
            "confident_max_err", "wall_plain_s", "wall_gated_s", "retrains", "train_s")
    out = {k: cmp[k] for k in keys}
    out["dlogz"] = cmp["logz_gated"] - cmp["logz_plain"]
    out["metric"] = "proposals judged per second, plain batched vs surrogate-gated nested sampling"
    out["config"] = text + f" (n_live {a.n_live}, first training after {a.first_train})"
    return out


def bench_gated(args):
    """Nested sampling on the 12-bin n = 4096 dataset, once with every
    proposal evaluated exactly and once gated by the surrogate ensemble
    (same seed): throughput in proposals judged per second, exact calls
    avoided, wall-clock speedup, and agreement of evidence and posterior.

    --phase both runs the two in this process. --phase plain / gated runs one
    of them, stopping after --time-limit seconds with its state in
    --checkpoint (continued by --resume) and writing the finished run to
    --result-out; --phase compare compares two such results."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    from paper_2501_12928_amd.sampler import (GatedLikelihood, NestedSampler, compare_runs, exact_gpu,
                                              load_result, save_result)
    kw, text = gate_settings(args)
    inst = synth.gen(args.gated_config, n_theta=1)
    head = {"unit": "proposals/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64 likelihood, f32 surrogate",
            "data": "synthetic", "config": {"workload": f"T complex128 {inst.m}x{inst.n}, {inst.n_k} k-bins, "
                                                        + text}}
    if args.phase == "compare":
        plain, gated = load_result(args.plain_result), load_result(args.gated_result)
        cmp = compare_runs(plain, gated, args.n_live)
        m, sd = gated.posterior_moments()
        print(json.dumps({"metric": "proposals judged per second by nested sampling at n=4096 complex FP64, "
                                    "surrogate-gated", "value": gated.n_proposed / gated.wall_s, **head,
                          "plain_proposals_per_s": plain.n_proposed / plain.wall_s, "comparison": cmp,
                          "gated_stats": {"retrains": gated.n_retrain, "train_s": gated.t_train_s,
                                          "gate_s": gated.t_gate_s, "exact_s": gated.t_exact_s},
                          "posterior_mean": m.tolist(), "posterior_std": sd.tolist(),
                          "theta_true": inst.theta_true.tolist(),
                          "power_recovery": gated.power_summary(inst.theta_true)}))
        return
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    if args.phase == "both":
        plain, gated, cmp, _ = gated_pair(ctx, inst.n_k, inst.lo, inst.hi, args)
        m, sd = gated.posterior_moments()
        print(json.dumps({"metric": "proposals judged per second by nested sampling at n=4096 complex FP64, "
                                    "surrogate-gated", "value": gated.n_proposed / gated.wall_s, **head,
                          "plain_proposals_per_s": plain.n_proposed / plain.wall_s, "comparison": cmp,
                          "posterior_mean": m.tolist(), "posterior_std": sd.tolist(),
                          "theta_true": inst.theta_true.tolist(),
                          "power_recovery": gated.power_summary(inst.theta_true)}))
        ctx.close()
        return
    sur = None
    gate = None
    if args.phase == "gated":
        sur = eor.Surrogate(inst.n_k, -1.0 if args.whiten else inst.lo, 1.0 if args.whiten else inst.hi,
                            n_members=5, hidden=256, seed=1)
        gate = GatedLikelihood(sur, **kw)
    ns = NestedSampler(exact_gpu(ctx), inst.n_k, inst.lo, inst.hi, n_live=args.n_live, dlogz=0.01, batch=512,
                       seed=7, gate=gate, audit_frac=args.audit_frac, pool_factor=args.pool_factor, progress=2000)
    r = ns.run(time_limit=args.time_limit, checkpoint=args.checkpoint, resume=args.resume)
    if r is None:
        print(json.dumps({"phase": args.phase, "stopped": True, "checkpoint": args.checkpoint,
                          "exact_calls": ns.stats["n_exact"], "proposals": ns.stats["n_proposed"]}))
    else:
        save_result(args.result_out, r)
        print(json.dumps({"phase": args.phase, "stopped": False, "result": args.result_out,
                          "iterations": r.iterations, "exact_calls": r.n_exact, "proposals": r.n_proposed,
                          "wall_s": r.wall_s, "logz": r.logz, "gate_rejected": r.n_gate_rejected,
                          "audited": r.n_audited, "false_rejections": r.n_false_reject,
                          "retrains": r.n_retrain, "train_s": r.t_train_s}))
    if sur is not None:
        sur.close()
    ctx.close()


def bench_instrument(args):
    """The path on data seen through a forward-modelled instrument: T built
    on the GPU (eor_forward_model) from the synthetic instrument (32 channels
    x 625 baselines = 20000 visibilities; 128 uv cells x (4 foreground + 28
    EoR) spectral modes = 4096 coefficients, 12 k-shells; 64 x 64 sky
    pixels, Gaussian beam), then the precompute and one likelihood batch of
    B = 512 theta. The data vector is drawn from the GPU-built T on the host."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    ins = synth.instrument(5)
    args_fm = (ins.freq, ins.bl, ins.lm, ins.beam, ins.uv, ins.Z, ins.norm)
    T = eor.forward_model(*args_fm)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    dev_in = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in args_fm[:6]]
    for a, b in ev:
        a.record(stream)
        eor.forward_model(*dev_in, ins.norm, out=T)
        b.record(stream)
    torch.cuda.synchronize()
    fm_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    F, n_bl, n_pix, n_uv = ins.freq.size, ins.bl.shape[0], ins.lm.shape[0], ins.uv.shape[0]
    fm_flop = 8.0 * F * n_bl * n_pix * n_uv
    inst = synth.instrument_instance(ins, T.cpu().numpy(), seed=7, n_theta=512)
    ctx = eor.Context(0)
    nv = torch.from_numpy(inst.noise_var).cuda()
    d = torch.from_numpy(inst.d).cuda()
    theta = torch.from_numpy(inst.theta).cuda()
    ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale)
    logL, info = ctx.loglike_batch(theta)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.loglike_batch(theta, out=logL, info=info)
    e1.record(stream)
    torch.cuda.synchronize()
    like_ms = e0.elapsed_time(e1)
    sampled = None
    if args.instrument_sample:
        # nested sampling of the 12 shells' power on this instrument: evidence,
        # per-shell posterior and Delta^2(k) against the power the data were drawn at
        from paper_2501_12928_amd.sampler import NestedSampler, exact_gpu
        r = NestedSampler(exact_gpu(ctx), inst.n_k, inst.lo, inst.hi, n_live=args.n_live, dlogz=0.01, batch=512,
                          seed=7, progress=2000).run()
        sampled = {"logz": r.logz, "logz_err": r.logz_err, "iterations": r.iterations, "exact_calls": r.n_exact,
                   "wall_s": r.wall_s, "n_live": args.n_live,
                   "power_recovery": r.power_summary(inst.theta_true, k=ins.k_shell)}
    print(json.dumps({
        "metric": "logL evals/s at n=4096 complex FP64 on a forward-modelled instrument (report)",
        "value": theta.shape[0] / (like_ms / 1e3), "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"T from the forward model: {F} channels x {n_bl} baselines, {n_uv} uv cells x "
                               f"{ins.Z.shape[1]} spectral modes, {n_pix} pixels, Gaussian beam; "
                               f"{ins.n_k} k-shells; B=512 theta"},
        "forward_model_ms": fm_ms, "forward_model_tflops": fm_flop / (fm_ms / 1e3) / 1e12,
        "forward_model_write_gbs": ins.m * ins.n * 16 / (fm_ms / 1e3) / 1e9,
        "loglike_ms": like_ms, "info_nonzero": int((info != 0).sum().item()),
        "logL_range": [float(logL.min().item()), float(logL.max().item())],
        "nested_sampling": sampled}))
    ctx.close()


def link_probe(mib: int = 512, reps: int = 5):
    """Pinned host <-> device copy rates on this machine (GB/s): one direction at
    a time, then both at once on two streams. The reference for how much of
    the host link the out-of-core schedule uses."""
    import torch
    n = mib << 20
    h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    h2 = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(n, dtype=torch.uint8, device="cuda")
    d2 = torch.empty(n, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return nbytes * reps / (time.perf_counter() - t0) / 1e9

    def both():
        with torch.cuda.stream(s1):
            d.copy_(h, non_blocking=True)
        with torch.cuda.stream(s2):
            h2.copy_(d2, non_blocking=True)

    out = {"h2d_gbs": rate(lambda: d.copy_(h, non_blocking=True), n),
           "d2h_gbs": rate(lambda: h.copy_(d, non_blocking=True), n),
           "both_directions_gbs": rate(both, 2 * n), "bytes_per_copy": n}
    del h, h2, d, d2
    return out


def bench_ooc(args):
    """Out-of-core likelihood at 20000 x 4096 (12 bins): A exported to host
    memory, then eor_loglike_host with the device limited to a window of
    `--ooc-mib` MiB, for the first `--ooc-theta` theta of the metric batch,
    `--ooc-lanes` at a time (0 = the library's choice). Reports evals/s over
    the whole call (packing A into pinned memory included), the time of a
    one-theta call, the library's schedule (lanes, pass width, host<->device
    bytes per theta) and the algorithmic FP64 rate, beside the in-core batch
    and the box's raw pinned copy rates."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    inst = synth.gen(CONFIG_ID)
    n = inst.n
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale)
    A, dbar, c, K0 = ctx.export_precompute()
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    dbar = dbar.cpu().numpy()
    th = inst.theta[:args.ooc_theta]
    # in-core reference timing on the same theta
    thd = torch.from_numpy(np.ascontiguousarray(th)).cuda()
    Lin, infin = ctx.loglike_batch(thd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.loglike_batch(thd, out=Lin, info=infin)
    torch.cuda.synchronize()
    t_in = time.perf_counter() - t0
    Lin = Lin.cpu().numpy()
    ctx.close()
    budget = args.ooc_mib << 20
    lanes = args.ooc_lanes
    plan = eor.loglike_host_plan(n, inst.n_k, budget, lanes)
    t0 = time.perf_counter()
    eor.loglike_host(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, th[:1], budget,
                     lanes=lanes)
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    L, info = eor.loglike_host(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale, th, budget,
                               lanes=lanes)
    t_ooc = time.perf_counter() - t0
    B = th.shape[0]
    moved = plan["link_bytes"]
    print(json.dumps({
        "metric": "out-of-core logL evals/s at n=4096 complex FP64 (report)",
        "value": B / t_ooc, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"T complex128 {inst.m}x{n}, {inst.n_k} k-bins; A in host memory, device window "
                               f"{args.ooc_mib} MiB; {B} theta, {plan['lanes']} at a time"},
        "seconds_per_theta": t_ooc / B, "seconds_one_theta_call": t_one,
        "lanes": plan["lanes"], "columns_per_pass": plan["cols_per_pass"],
        "host_device_bytes_per_theta": moved, "host_device_gbs": moved * B / t_ooc / 1e9,
        "tflops": B * flops_per_theta(n) / t_ooc / 1e12,
        "in_core_evals_per_s": B / t_in,
        "link_probe": link_probe(),
        "info_nonzero": int((info != 0).sum()),
        "max_rel_diff_vs_in_core": float(np.max(np.abs(L - Lin) / np.abs(Lin)))}))


def surrogate_flops(n_in: int, H: int):
    """(inference, training) FP32 flop per sample and member of an
    n_in -> H -> H -> 1 network: the forward pass is its three dense layers;
    a training step adds the weight gradients of both hidden layers and the
    input gradient of the second (two multiply-adds per weight each)."""
    fwd = 2.0 * (n_in * H + H * H + H)
    bwd = 2.0 * (n_in * H + H * H) + 2.0 * H * H + 2.0 * H
    return fwd, fwd + bwd


def bench_surrogate(args):
    """Throughput of the learned part alone: training the 5-member ensemble
    (12 -> 256 -> 256 -> 1, GELU, FP32) on 1e5 exact evaluations, then gating
    1e6 prior proposals. The training targets are exact FP64 logL values of a
    12-bin instance at n = 1024 (cheap to evaluate; the network only sees them
    standardised)."""
    import torch
    import synth
    import paper_2501_12928_amd as eor
    n_train, n_prop = args.surrogate_train, args.surrogate_proposals
    inst = synth.small(3001, m=4096, n=1024, n_k=12, n_theta=1)
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale)
    rng = np.random.default_rng(3002)
    theta = torch.from_numpy(synth.theta_batch(rng, n_train, inst.n_k, inst.lo, inst.hi)).cuda()
    logL = torch.empty(n_train, dtype=torch.float64, device="cuda")
    info = torch.empty(n_train, dtype=torch.int32, device="cuda")
    for c0 in range(0, n_train, 4096):
        c1 = min(n_train, c0 + 4096)
        ctx.loglike_batch(theta[c0:c1], out=logL[c0:c1], info=info[c0:c1])
    torch.cuda.synchronize()
    ctx.close()
    if not bool((info == 0).all().item()):
        print(json.dumps({"error": "failed exact evaluations in the training set"}))
        sys.exit(1)
    H, M = 256, 5
    sur = eor.Surrogate(inst.n_k, inst.lo, inst.hi, n_members=M, hidden=H, seed=1)
    # early stopping off: a fixed number of epochs is timed
    cfg = eor.train_cfg(epochs=args.surrogate_epochs, minibatch=args.train_minibatch,
                        patience=args.surrogate_epochs + 1, lr=1e-3, seed=5)
    warm = eor.train_cfg(epochs=2, minibatch=args.train_minibatch, patience=3, lr=1e-3, seed=4)
    sur.train(theta, logL, warm)          # builds the epoch graph and the buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    epochs, val = sur.train(theta, logL, cfg)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    n_val = max(1, int(0.1 * n_train))
    n_tr = n_train - n_val
    steps = max(1, n_tr // min(args.train_minibatch, n_tr))
    samples_per_epoch = steps * min(args.train_minibatch, n_tr)
    f_inf, f_train = surrogate_flops(inst.n_k, H)
    train_flop = epochs * M * (samples_per_epoch * f_train + n_val * f_inf)

    prop = torch.from_numpy(synth.theta_batch(rng, n_prop, inst.n_k, inst.lo, inst.hi)).cuda()
    L_min = float(torch.quantile(logL, 0.5).item())
    stream = torch.cuda.current_stream()
    sur.gate(prop, L_min, args.tau)
    torch.cuda.synchronize()
    reps = 5
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        mean, spread, dec = sur.gate(prop, L_min, args.tau)
        b.record(stream)
    torch.cuda.synchronize()
    gate_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    gate_flop = n_prop * M * f_inf
    achieved = gate_flop / (gate_ms / 1e3) / 1e12
    sur.close()
    print(json.dumps({
        "metric": "surrogate proposals gated per second (5 x MLP 12-256-256-1, FP32)",
        "value": n_prop / (gate_ms / 1e3), "unit": "proposals/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"train on {n_train} exact logL of a 12-bin n=1024 instance "
                               f"({args.surrogate_epochs} epochs, minibatch {args.train_minibatch}, "
                               f"10% validation); gate {n_prop} prior proposals at tau={args.tau}",
                   "members": M, "hidden": H, "n_in": inst.n_k},
        "gate_ms": gate_ms, "gate_tflops": achieved,
        "gate_rejected_frac": float((dec == 0).float().mean().item()),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None, "kernel": "surrogate gate (all kernels)",
                     "flops_per_launch": gate_flop},
        "train": {"seconds": train_s, "epochs": epochs, "samples_per_epoch": samples_per_epoch,
                  "sample_epochs_per_s": epochs * samples_per_epoch * M / train_s,
                  "tflops": train_flop / train_s / 1e12, "val_loss": val.tolist()},
    }))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true", help="skip the reduced-precision report")
    ap.add_argument("--no-gated", action="store_true", help="skip the gated nested-sampling leg")
    ap.add_argument("--gated-n-live", type=int, default=200,
                    help="live points of the default run's gated leg (plain and gated)")
    ap.add_argument("--workload", choices=["metric", "group", "gated", "stress", "surrogate", "instrument", "ooc"], default="metric",
                    help="metric: 20000x4096, B=512 (default); group: 48 uneven sub-band instances; "
                         "gated: nested sampling at 20000x4096 without and with the surrogate gate; "
                         "stress: reduced precision on ill-conditioned instruments at 8000x2048; "
                         "surrogate: ensemble training on 1e5 samples and gating of 1e6 proposals; "
                         "instrument: T from the forward model, then precompute and one batch; "
                         "ooc: the likelihood with A in host memory through a small device window")
    ap.add_argument("--gated-config", type=int, default=4, help="workload of the gated run (1 or 4)")
    ap.add_argument("--n-live", type=int, default=500)
    ap.add_argument("--first-train", type=int, default=30000)
    ap.add_argument("--retrain-every", type=int, default=1000)
    ap.add_argument("--window", type=int, default=8000)
    ap.add_argument("--tau", type=float, default=0.05)
    ap.add_argument("--margin", type=float, default=10.0)
    ap.add_argument("--train-epochs", type=int, default=300)
    ap.add_argument("--retrain-epochs", type=int, default=1000,
                    help="epochs of each warm retraining (0: as the first training)")
    ap.add_argument("--train-minibatch", type=int, default=512)
    ap.add_argument("--pool-factor", type=int, default=1)
    ap.add_argument("--band-below", type=float, default=0.5,
                    help="gated: censor training targets this far below the threshold")
    ap.add_argument("--band-above", type=float, default=1.0,
                    help="gated: ... and this far above it (0: no censoring; train near the threshold)")
    ap.add_argument("--reach", type=float, default=0.2,
                    help="gated runs: reject a confident prediction only within this of the band's floor")
    ap.add_argument("--audit-frac", type=float, default=0.01,
                    help="gated runs: fraction of the gate's rejections evaluated anyway")
    ap.add_argument("--no-whiten", dest="whiten", action="store_false",
                    help="gated: keep the prior box as the inputs' scale (default: the training data's box)")
    ap.add_argument("--no-cold", dest="cold", action="store_false",
                    help="gated: retrain from the previous weights (default: from fresh weights)")
    ap.add_argument("--stale-gap", type=int, default=250)
    ap.add_argument("--phase", choices=["both", "plain", "gated", "compare"], default="both")
    ap.add_argument("--time-limit", type=float, default=None, help="gated workload, one phase: stop after this many s")
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--result-out", default=None)
    ap.add_argument("--plain-result", default=None)
    ap.add_argument("--gated-result", default=None)
    ap.add_argument("--instrument-sample", action="store_true",
                    help="instrument workload: also run nested sampling and report the recovered spectrum")
    ap.add_argument("--ooc-mib", type=int, default=256, help="ooc workload: device window in MiB")
    ap.add_argument("--ooc-theta", type=int, default=8, help="ooc workload: theta evaluated")
    ap.add_argument("--ooc-lanes", type=int, default=0,
                    help="ooc workload: theta factored at once (0 = the library's choice)")
    ap.add_argument("--surrogate-train", type=int, default=100000)
    ap.add_argument("--surrogate-proposals", type=int, default=1000000)
    ap.add_argument("--surrogate-epochs", type=int, default=50)
    ap.add_argument("--tuning", default=None,
                    help="launch choices 'stages,wg_per_cu,tiles_per_pass' of the likelihood batch "
                         "(default: the library's)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this size (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build targets one GPU: the likelihood batch shards by theta "
                                   "across GPUs only in design; run with --gpus 1"}))
        sys.exit(2)

    import torch

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        x = torch.ones(nel, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nel * 8, "copy_bytes_written": nel * 8}))
        return

    import synth
    import paper_2501_12928_amd as eor

    if args.workload == "group":
        return bench_group(args)
    if args.workload == "gated":
        return bench_gated(args)
    if args.workload == "stress":
        return bench_stress(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "instrument":
        return bench_instrument(args)
    if args.workload == "ooc":
        return bench_ooc(args)

    inst = synth.gen(CONFIG_ID)
    B, n, m = inst.theta.shape[0], inst.n, inst.m
    T = torch.from_numpy(inst.T).cuda()
    nv = torch.from_numpy(inst.noise_var).cuda()
    d = torch.from_numpy(inst.d).cuda()
    theta = torch.from_numpy(inst.theta).cuda()
    logL = torch.empty(B, dtype=torch.float64, device="cuda")
    info = torch.empty(B, dtype=torch.int32, device="cuda")
    ctx = eor.Context(0)
    if args.tuning:
        ctx.set_tuning(*[int(v) for v in args.tuning.split(",")])
    stream = torch.cuda.current_stream()

    def step(ev=None):
        ctx.precompute(T, nv, d, inst.n_k, inst.bin_of, inst.fixed_var, inst.bin_scale)
        if ev is not None:
            ev[0].record(stream)
        ctx.loglike_batch(theta, out=logL, info=info)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    like_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    ok = bool((info == 0).all().item()) and bool(torch.isfinite(logL).all().item())
    if not ok:
        print(json.dumps({"error": "non-finite logL or nonzero info in the benchmark batch"}))
        sys.exit(1)

    fl = B * flops_per_theta(n)
    achieved = fl / (like_ms / 1e3) / 1e12
    like_ms_median = float(np.median([a.elapsed_time(b) for a, b in events]))
    traffic, mfma_insts = counters_per_launch()
    # flops the matrix cores execute (16x16x4 FP64 MFMA = 2048 flops each): with
    # three real products per complex step they are about 3/4 of the LAPACK count,
    # so `frac` (LAPACK count) can pass 1 while the executed fraction cannot
    executed = None if mfma_insts is None else mfma_insts * 2048.0 / (like_ms / 1e3) / 1e12
    # measured FP64 matrix peak over a run about as long as one likelihood
    # launch (a round is 8 MFMAs of 64 cycles for each of the two waves that
    # share a SIMD: 1024 cycles)
    probe_iters = int(like_ms * 1e-3 * 2.4e9 / 1024)
    peak_meas, probe_ms = eor.probe_fp64_mfma(probe_iters)
    out = {
        "metric": "logL evals/s at n=4096 complex FP64, batched",
        "value": B * args.steps / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"T complex128 {m}x{n} (entries CN(0,1)/sqrt(m)), sigma^2~U(0.5,2), "
                               f"{inst.n_k} k-bins, {int((inst.bin_of >= 0).sum())} EoR + "
                               f"{int((inst.bin_of < 0).sum())} foreground coefficients, "
                               f"B={B} theta~U[-1,3]^{inst.n_k} per call; step = precompute + batch",
                   "m": m, "n": n, "n_k": inst.n_k, "B": B},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "likelihood_kernel", "launch_ms": like_ms, "launch_ms_median": like_ms_median,
                     "flops_per_launch": fl, "flops_basis": "LAPACK complex count, 8 real flops per complex "
                                                            "multiply-add; the kernel runs 3 real MFMA "
                                                            "products per complex step",
                     "executed_tflops": executed,
                     "executed_frac": None if executed is None else executed / PEAK_FP64_TFLOPS,
                     "peak_measured": peak_meas,
                     "frac_measured": achieved / peak_meas, "peak_measured_run_ms": probe_ms},
        "loglike_evals_per_s": B / (like_ms / 1e3),
        "tuning": dict(zip(("stages", "wg_per_cu", "tiles_per_pass"), ctx.tuning())),
        "gated": None,
    }
    if not args.no_gated:
        out["gated"] = gated_leg(ctx, inst, args)
    if not args.no_precision:
        out["precision"] = precision_report(ctx, inst, T, nv, d, theta, logL.clone())
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst)
        out["cpu_lapack"] = cpu_lapack_reference(ctx, inst)
    else:
        out["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
