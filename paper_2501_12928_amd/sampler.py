"""Nested sampling over the power-spectrum parameters, with batched
proposals and an optional surrogate gate.

The sampler plays the role the paper gives MultiNest (Summary: posterior
samples and the Bayesian evidence for model selection): Skilling's nested
sampling with n_live live points, replacements drawn uniformly from the
prior box restricted to an enlarged bounding ellipsoid of the live points
(single-ellipsoid rejection sampling, Mukherjee, Parkinson & Liddle 2006),
and the evidence accumulated as Z = sum_i L_i (X_{i-1} - X_i) with
X_i = exp(-i / n_live).

Proposals are drawn and evaluated in batches (the GPU likelihood wants
hundreds of theta per call) and consumed in order. A proposal evaluated
against an older, lower threshold remains a valid replacement later: a
point uniform in {L > L_old}, conditioned on L > L_new >= L_old, is uniform
in {L > L_new}. The price is that the threshold rises while a batch is
consumed, so many exactly evaluated proposals end up below it.

With a gate (see GatedLikelihood), the surrogate's ensemble mean and
spread are computed for a whole pool of proposals, and each proposal is
judged when its turn comes, against the threshold of that moment: a
proposal the surrogate is confident lies below it (spread <= tau and
mean below the gate's rejection line, at most L_min) is rejected without an
exact evaluation; the uncertain ones
are evaluated exactly, a batch of them at a time. Only exact values ever
enter the live set, so every accepted point carries its exact FP64 logL. A
small random fraction of the surrogate's rejections is evaluated anyway to
measure false rejections.

The bookkeeping is host logic in numpy; the likelihood, the surrogate and
the compaction of proposals run in the library's kernels.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Result:
    logz: float
    logz_err: float
    information: float
    samples: np.ndarray        # dead points then the final live points
    logl: np.ndarray
    logw: np.ndarray           # log posterior weights (normalised)
    iterations: int
    n_exact: int               # exact likelihood evaluations
    n_proposed: int            # proposals drawn inside the prior box
    n_gate_rejected: int       # proposals rejected by the surrogate without an exact call
    n_audited: int             # surrogate rejections evaluated anyway
    n_false_reject: int        # ... of which the exact logL was above the threshold
    n_retrain: int
    wall_s: float
    t_exact_s: float
    t_gate_s: float
    t_train_s: float
    n_conf_checked: int = 0    # confident predictions (spread <= tau) that went to an exact call anyway
    max_conf_err: float = 0.0  # ... their largest |mean - exact logL| (on the gate's censored scale)
    # one row per audited rejection: exact logL, threshold in force, ensemble
    # mean and spread, the band (floor, cap) the network was trained on, and
    # the iteration (AUDIT_COLUMNS)
    audit_log: np.ndarray | None = None

    def posterior_moments(self):
        w = np.exp(self.logw - self.logw.max())
        w /= w.sum()
        mean = w @ self.samples
        var = w @ (self.samples - mean) ** 2
        return mean, np.sqrt(var)

    def power_summary(self, theta_true=None, k=None):
        """Per k-bin power P_b = 10^theta_b recovered from the weighted
        samples (theta is log10 power per bin): posterior mean and standard
        deviation of P_b, the median and 16-84% interval of theta_b, and, given
        the values the data were drawn at, the fractional error of the mean
        power and the offset of the median in posterior standard deviations.
        Given the bins' wavenumbers k_b, also the dimensionless spectrum
        Delta^2_b = k_b^3 P_b / (2 pi^2) (eq. 2), its posterior mean and
        standard deviation (and its true value)."""
        w = np.exp(self.logw - self.logw.max())
        w /= w.sum()
        P = 10.0 ** self.samples
        pm = w @ P
        ps = np.sqrt(w @ (P - pm) ** 2)
        out = {"power_mean": pm.tolist(), "power_std": ps.tolist(),
               "theta_median": [], "theta_lo": [], "theta_hi": []}
        for b in range(self.samples.shape[1]):
            order = np.argsort(self.samples[:, b])
            cw = np.cumsum(w[order])
            q = lambda f: float(self.samples[order[min(np.searchsorted(cw, f), len(cw) - 1)], b])
            out["theta_median"].append(q(0.5))
            out["theta_lo"].append(q(0.16))
            out["theta_hi"].append(q(0.84))
        if theta_true is not None:
            tt = np.asarray(theta_true, dtype=np.float64)
            pt = 10.0 ** tt
            out["power_true"] = pt.tolist()
            out["power_frac_err"] = ((pm - pt) / pt).tolist()
            half = 0.5 * (np.array(out["theta_hi"]) - np.array(out["theta_lo"]))
            out["theta_offset_sigma"] = ((np.array(out["theta_median"]) - tt) / half).tolist()
        if k is not None:
            c = np.asarray(k, dtype=np.float64) ** 3 / (2.0 * math.pi ** 2)
            out["k"] = np.asarray(k, dtype=np.float64).tolist()
            out["delta2_mean"] = (c * pm).tolist()
            out["delta2_std"] = (c * ps).tolist()
            if theta_true is not None:
                out["delta2_true"] = (c * pt).tolist()
        return out


AUDIT_COLUMNS = ("logl", "L_min", "mean", "spread", "floor", "cap", "iteration")


def save_result(path, r: Result):
    """A Result as one .npz (arrays, and the scalars as JSON; no pickles)."""
    import json
    arrays = ("samples", "logl", "logw", "audit_log")
    meta = {f.name: getattr(r, f.name) for f in dataclasses.fields(r) if f.name not in arrays}
    extra = {} if r.audit_log is None else {"audit_log": r.audit_log}
    np.savez(path, samples=r.samples, logl=r.logl, logw=r.logw, **extra,
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_result(path) -> Result:
    import json
    z = np.load(path, allow_pickle=False)
    meta = json.loads(z["meta"].tobytes().decode())
    log = z["audit_log"] if "audit_log" in z.files else None
    return Result(samples=z["samples"], logl=z["logl"], logw=z["logw"], audit_log=log, **meta)


def _logsubexp(a, b):
    """log(exp(a) - exp(b)) for a > b."""
    return a + math.log1p(-math.exp(b - a))


class Ellipsoid:
    """Bounding ellipsoid of a point set, enlarged by a volume factor."""

    def __init__(self, pts: np.ndarray, enlarge: float):
        d = pts.shape[1]
        self.mu = pts.mean(axis=0)
        C = np.cov(pts, rowvar=False).reshape(d, d) + 1e-12 * np.eye(d)
        Ci = np.linalg.inv(C)
        dx = pts - self.mu
        k = float(np.max(np.einsum("ij,jk,ik->i", dx, Ci, dx)))
        self.L = np.linalg.cholesky(C * k * enlarge ** (2.0 / d))

    def sample(self, rng: np.random.Generator, n: int) -> np.ndarray:
        d = self.mu.size
        g = rng.standard_normal((n, d))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        r = rng.uniform(size=(n, 1)) ** (1.0 / d)
        return self.mu + (g * r) @ self.L.T


class NestedSampler:
    """loglike(theta [B, d] float64) -> logL [B]; gate (optional) is a
    GatedLikelihood-like object with predict(theta) -> (mean, spread) or
    None, tau, trained, reject_below(L_min, band), band_now(), censor(logL, band), observe(theta,
    logL) and maybe_retrain(iteration, L_min).

    run() may stop at an iteration boundary once `time_limit` seconds have
    passed, saving its whole state (live and dead points, pool, random
    generators, counters, the gate's history and the surrogate's parameters)
    to `checkpoint`; run(resume=path) continues from such a file exactly
    where it stopped (the surrogate's Adam moments restart at zero there)."""

    def __init__(self, loglike, n_dim, lo, hi, n_live=500, enlarge=1.5, dlogz=0.01, batch=512,
                 seed=0, gate=None, audit_frac=0.01, max_iter=2_000_000, pool_factor=1, progress=0):
        self.loglike = loglike
        self.d = int(n_dim)
        self.lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (self.d,)).copy()
        self.hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (self.d,)).copy()
        self.n_live = int(n_live)
        self.enlarge = float(enlarge)
        self.dlogz = float(dlogz)
        self.batch = int(batch)
        self.rng = np.random.default_rng(seed)
        self.audit_rng = np.random.default_rng([seed, 1])
        self.gate = gate
        self.audit_frac = float(audit_frac)
        self.max_iter = int(max_iter)
        self.pool_factor = int(pool_factor)
        self.progress = int(progress)
        self.stats = dict(n_exact=0, n_proposed=0, n_gate_rejected=0, n_audited=0, n_false_reject=0,
                          t_exact=0.0, t_gate=0.0, n_conf_checked=0, max_conf_err=0.0, n_screened=0,
                          n_confident=0)

    def _exact(self, th):
        t0 = time.perf_counter()
        L = np.asarray(self.loglike(th), dtype=np.float64)
        self.stats["t_exact"] += time.perf_counter() - t0
        self.stats["n_exact"] += th.shape[0]
        if self.gate is not None:
            self.gate.observe(th, L)
        return L

    def _propose(self, live, count):
        """`count` proposals inside the prior box from the live points'
        enlarged bounding ellipsoid."""
        ell = Ellipsoid(live, self.enlarge)
        out = []
        need = count
        while need > 0:
            x = ell.sample(self.rng, max(need * 2, 64))
            x = x[np.all((x >= self.lo) & (x <= self.hi), axis=1)]
            out.append(x[:need])
            need -= out[-1].shape[0]
        return np.concatenate(out)

    def _new_pool(self, live, L_min):
        """A pool of proposals. Without a trained gate: one batch, evaluated
        exactly now. With one: proposals are drawn and screened by the
        surrogate until the pool holds `batch` that it is unsure of at the
        current threshold (at most pool_factor x 8 batches), and the pool ends
        at that one; so the exact call it leads to fills whole rounds of the
        GPU, while the proposals stay an i.i.d. sequence consumed in order
        (the cut is a stopping time). Exact logL are left for later (NaN)."""
        gated = self.gate is not None and self.gate.trained
        if not gated:
            th = self._propose(live, self.batch)
            self.stats["n_proposed"] += th.shape[0]
            pool = {"th": th, "L": np.full(th.shape[0], np.nan), "mean": None, "spread": None, "pos": 0}
            pool["L"][:] = self._exact(th)
            return pool
        ths, means, spreads = [], [], []
        unsure = 0
        cap = self.batch * self.pool_factor * 8
        drawn = 0
        while unsure < self.batch and drawn < cap:
            th = self._propose(live, self.batch * self.pool_factor)
            t0 = time.perf_counter()
            m, sp = self.gate.predict(th)
            self.stats["t_gate"] += time.perf_counter() - t0
            self.stats["n_screened"] += th.shape[0]
            self.stats["n_confident"] += int(np.count_nonzero(sp <= self.gate.tau))
            u = ~((sp <= self.gate.tau) & (m < self.gate.reject_below(L_min, self.gate.band_now())))
            c = np.cumsum(u)
            if unsure + int(c[-1]) >= self.batch:
                cut = int(np.searchsorted(c, self.batch - unsure)) + 1
                th, m, sp = th[:cut], m[:cut], sp[:cut]
                unsure = self.batch
            else:
                unsure += int(c[-1])
            ths.append(th)
            means.append(m)
            spreads.append(sp)
            drawn += th.shape[0]
        th = np.concatenate(ths)
        self.stats["n_proposed"] += th.shape[0]
        return {"th": th, "L": np.full(th.shape[0], np.nan), "mean": np.concatenate(means),
                "spread": np.concatenate(spreads), "pos": 0, "band": self.gate.band_now()}

    def _confident_reject(self, pool, i, L_min):
        return (pool["mean"] is not None and pool["spread"][i] <= self.gate.tau
                and pool["mean"][i] < self.gate.reject_below(L_min, pool["band"]))

    def _next_valid(self, pool, L_min):
        """Index of the next proposal of the pool with exact logL > L_min,
        or None when the pool is used up."""
        th, L = pool["th"], pool["L"]
        while pool["pos"] < th.shape[0]:
            i = pool["pos"]
            if not np.isnan(L[i]):
                pool["pos"] += 1
                if L[i] > L_min:
                    return i
                continue
            if self._confident_reject(pool, i, L_min):
                L[i] = -np.inf
                pool["pos"] += 1
                self.stats["n_gate_rejected"] += 1
                if self.audit_frac > 0 and self.audit_rng.uniform() < self.audit_frac:
                    # judged in full batches at the end, with what the gate saw
                    fl, cp = pool.get("band") or (np.nan, np.nan)
                    self._audits.append((th[i].copy(), (L_min, float(pool["mean"][i]),
                                                        float(pool["spread"][i]), fl, cp, self._it)))
                continue
            # evaluate exactly, in one call, the rest of the pool that the gate is unsure of
            idx = [j for j in range(i, th.shape[0])
                   if np.isnan(L[j]) and not self._confident_reject(pool, j, L_min)]
            L[idx] = self._exact(th[idx])
            if pool["mean"] is not None:
                # the surrogate's error where it was confident (spread <= tau) but
                # not below the threshold, so the point went to the exact call
                conf = [j for j in idx if pool["spread"][j] <= self.gate.tau]
                if conf:
                    err = np.abs(pool["mean"][conf] - self.gate.censor(L[conf], pool.get("band")))
                    self.stats["n_conf_checked"] += len(conf)
                    self.stats["max_conf_err"] = max(self.stats["max_conf_err"], float(np.max(err)))
        return None

    def _save(self, path, st):
        """Everything run() needs to continue, in one .npz (no pickles:
        arrays, and the scalars as JSON)."""
        import json
        pool = st["pool"]
        arrays = dict(live=st["live"], live_L=st["live_L"], dead=np.array(st["dead"]).reshape(-1, self.d),
                      dead_L=np.array(st["dead_L"]), dead_lnw=np.array(st["dead_lnw"]),
                      audit_th=np.array([a for a, _ in self._audits]).reshape(-1, self.d),
                      audit_info=np.array([b for _, b in self._audits], dtype=np.float64).reshape(-1, 6))
        meta = dict(logz=float(st["logz"]), ln_x_prev=float(st["ln_x_prev"]), it=int(st["it"]),
                    elapsed=float(st["elapsed"]), t_train0=float(st["t_train0"]), stats=self.stats,
                    rng=self.rng.bit_generator.state, audit_rng=self.audit_rng.bit_generator.state,
                    pool=None if pool is None else dict(pos=int(pool["pos"]), gated=pool["mean"] is not None,
                                                        band=[float(v) for v in pool["band"]]
                                                        if pool.get("band") is not None else None))
        if pool is not None:
            arrays["pool_th"] = pool["th"]
            arrays["pool_L"] = pool["L"]
            if pool["mean"] is not None:
                arrays["pool_mean"] = pool["mean"]
                arrays["pool_spread"] = pool["spread"]
        if self.gate is not None:
            g_arrays, g_meta = self.gate.state()
            arrays.update({"gate_" + k: v for k, v in g_arrays.items()})
            meta["gate"] = g_meta
        arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
        np.savez(path, **arrays)

    def _load(self, path):
        import json
        z = np.load(path, allow_pickle=False)
        meta = json.loads(z["meta"].tobytes().decode())
        self.stats = meta["stats"]
        self.rng.bit_generator.state = meta["rng"]
        self.audit_rng.bit_generator.state = meta["audit_rng"]
        if "audit_info" in z.files:
            info = z["audit_info"]
        else:   # files written before the gate's view was kept: the threshold only
            info = np.full((z["audit_L"].shape[0], 6), np.nan)
            info[:, 0] = z["audit_L"]
        self._audits = [(z["audit_th"][k].copy(), tuple(float(v) for v in info[k])) for k in range(info.shape[0])]
        pool = None
        if meta["pool"] is not None:
            pool = {"th": z["pool_th"], "L": z["pool_L"].copy(), "pos": meta["pool"]["pos"],
                    "mean": z["pool_mean"] if meta["pool"]["gated"] else None,
                    "spread": z["pool_spread"] if meta["pool"]["gated"] else None,
                    "band": None if meta["pool"].get("band") is None else tuple(meta["pool"]["band"])}
        if self.gate is not None:
            self.gate.set_state({k[5:]: z[k] for k in z.files if k.startswith("gate_")}, meta["gate"])
        return dict(live=z["live"].copy(), live_L=z["live_L"].copy(), dead=list(z["dead"]),
                    dead_L=list(z["dead_L"]), dead_lnw=list(z["dead_lnw"]), logz=meta["logz"],
                    ln_x_prev=meta["ln_x_prev"], pool=pool, it=meta["it"], elapsed=meta["elapsed"],
                    t_train0=meta["t_train0"])

    def run(self, time_limit=None, checkpoint=None, resume=None):
        """The nested-sampling run as a Result; None if this call stopped
        after `time_limit` seconds of its own (its state then saved to
        `checkpoint`; every call makes at least one iteration)."""
        t_start = t_call = time.perf_counter()
        d, n = self.d, self.n_live
        if resume is not None:
            st = self._load(resume)
            live, live_L = st["live"], st["live_L"]
            dead, dead_L, dead_lnw = st["dead"], st["dead_L"], st["dead_lnw"]
            logz, ln_x_prev, pool, it = st["logz"], st["ln_x_prev"], st["pool"], st["it"]
            t_start -= st["elapsed"]
            t_train0 = st["t_train0"]
        else:
            live = self.lo + (self.hi - self.lo) * self.rng.uniform(size=(n, d))
            live_L = self._exact(live)
            dead, dead_L, dead_lnw = [], [], []
            logz = -np.inf
            ln_x_prev = 0.0
            pool = None
            self._audits = []
            it = 0
            t_train0 = self.gate.train_seconds if self.gate is not None else 0.0
            if self.gate is not None:
                self.gate.maybe_retrain(it, float(np.min(live_L)))
        it_call = self._it = it
        while it < self.max_iter:
            if time_limit is not None and it > it_call and time.perf_counter() - t_call > time_limit:
                self._save(checkpoint, dict(live=live, live_L=live_L, dead=dead, dead_L=dead_L,
                                            dead_lnw=dead_lnw, logz=logz, ln_x_prev=ln_x_prev, pool=pool,
                                            it=it, elapsed=time.perf_counter() - t_start, t_train0=t_train0))
                return None
            worst = int(np.argmin(live_L))
            L_min = float(live_L[worst])
            ln_x = -(it + 1) / n
            ln_w = L_min + _logsubexp(ln_x_prev, ln_x)
            logz = np.logaddexp(logz, ln_w)
            dead.append(live[worst].copy())
            dead_L.append(L_min)
            dead_lnw.append(ln_w)
            ln_x_prev = ln_x
            it += 1
            self._it = it
            # replacement: the next pooled proposal above the threshold
            j = None if pool is None else self._next_valid(pool, L_min)
            while j is None:
                pool = self._new_pool(live, L_min)
                j = self._next_valid(pool, L_min)
            live[worst] = pool["th"][j]
            live_L[worst] = pool["L"][j]
            if self.gate is not None:
                self.gate.maybe_retrain(it, float(np.min(live_L)))
            if self.progress and it % self.progress == 0:
                import sys
                print(f"ns: iteration {it} ln Z {logz:.3f} L_min {L_min:.3f} exact {self.stats['n_exact']} "
                      f"gate-rejected {self.stats['n_gate_rejected']} screened {self.stats['n_screened']} "
                      f"confident {self.stats['n_confident']} {time.perf_counter() - t_start:.1f}s",
                      file=sys.stderr, flush=True)
            # stop when the live points can no longer change ln Z by dlogz
            if np.logaddexp(logz, float(np.max(live_L)) + ln_x) - logz < self.dlogz:
                break
        # audits of gate rejections: exact logL against the threshold in force
        # when each was rejected (they change nothing in the run)
        log = [np.zeros((0, len(AUDIT_COLUMNS)))]
        for a in range(0, len(self._audits), self.batch):
            chunk = self._audits[a:a + self.batch]
            La = self._exact(np.stack([t for t, _ in chunk]))
            info = np.array([b for _, b in chunk], dtype=np.float64)
            self.stats["n_audited"] += len(chunk)
            self.stats["n_false_reject"] += int(np.count_nonzero(La > info[:, 0]))
            log.append(np.column_stack([La, info]))
        # the final live points share the remaining prior volume
        ln_wl = live_L + ln_x_prev - math.log(n)
        logz_final = np.logaddexp(logz, np.logaddexp.reduce(ln_wl))
        samples = np.concatenate([np.array(dead), live])
        logl = np.concatenate([np.array(dead_L), live_L])
        lnw = np.concatenate([np.array(dead_lnw), ln_wl])
        # information H = sum_i p_i ln(L_i / Z), live points included
        p = np.exp(lnw - logz_final)
        H = float(np.sum(p * (logl - logz_final)))
        st = self.stats
        return Result(logz=float(logz_final), logz_err=math.sqrt(max(H, 0.0) / n), information=H,
                      samples=samples, logl=logl, logw=lnw - logz_final, iterations=it,
                      n_exact=st["n_exact"], n_proposed=st["n_proposed"],
                      n_gate_rejected=st["n_gate_rejected"], n_audited=st["n_audited"],
                      n_false_reject=st["n_false_reject"],
                      n_retrain=self.gate.n_train if self.gate is not None else 0,
                      wall_s=time.perf_counter() - t_start, t_exact_s=st["t_exact"], t_gate_s=st["t_gate"],
                      t_train_s=(self.gate.train_seconds - t_train0) if self.gate is not None else 0.0,
                      n_conf_checked=st["n_conf_checked"], max_conf_err=st["max_conf_err"],
                      audit_log=np.concatenate(log))


class GatedLikelihood:
    """The surrogate gate for NestedSampler: keeps the exact evaluations it
    sees, (re)trains the surrogate on the most recent ones, and decides which
    proposals need an exact call. Until the first training (once
    `first_train` exact evaluations have been seen: the initial prior draws
    and the early proposals) every proposal is evaluated exactly.

    Nested-sampling rejections lie below the threshold L_min, so the
    surrogate must be accurate there. Two ways to train for it:

    - band=None: retraining uses the last `window` exact evaluations with
      logL >= L_min - margin, standardised on that window, starting from the
      previous parameters.
    - band=(below, above): the network is trained on the last `window` exact
      evaluations with logL censored to the band [L_ref - below, L_ref +
      above] around the threshold L_ref at training time. The gate's decision
      only asks whether a proposal lies below the threshold, and censoring
      keeps that answer wherever the band reaches: a proposal far below
      predicts the floor, which is below every later threshold. The flat
      parts are easy to fit, so the ensemble agrees there (small spread) even
      early in the run, when logL spans thousands of units over the live
      points and its uncensored fit could never reach a spread of tau. The
      band is re-centred by retraining once L_min has climbed half its upper
      width (at most once per `stale_gap` iterations), so early in the run,
      when the threshold climbs fast, it lies far above the band most of the
      time and every valid proposal's target is the band's top.

      A rejection is trusted only where the network places the proposal at
      the floor: mean < min(L_min, floor + reach). Predictions between the
      floor and the top are not trusted even below L_min: with a stale band
      they are where the network's gross errors land (valid points many
      units above the threshold read in the middle of the band), and such
      losses are not harmless: they fall on the lower part of the valid
      region, so the replacements drift inward, the threshold climbs too
      fast and ln Z comes out high. A point at the floor lies at least
      `below` - `reach` under every later threshold.

    surrogate: an object with train(theta, logL, ...) and gate(theta, L_min,
    tau) -> (mean, spread, decision) (paper_2501_12928_amd.Surrogate, or any
    stand-in with that interface)."""

    def __init__(self, surrogate, tau=0.05, first_train=100_000, retrain_every=0, window=100_000,
                 margin=np.inf, train_kwargs=None, retrain_kwargs=None, band=None, reach=0.2, stale_gap=250,
                 whiten=False, cold=False, seed=0):
        self.s = surrogate
        self.tau = float(tau)
        self.first_train = int(first_train)
        self.retrain_every = int(retrain_every)
        self.window = int(window)
        self.margin = float(margin)
        self.train_kwargs = train_kwargs or {}
        # warm retraining starts from the previous parameters and may use a
        # smaller budget than the first training
        self.retrain_kwargs = retrain_kwargs if retrain_kwargs is not None else self.train_kwargs
        self._th = []
        self._L = []
        self._count = 0
        self.trained = False
        self.n_train = 0
        self.train_seconds = 0.0
        self._last_iter = 0
        self.band = None if band is None else (float(band[0]), float(band[1]))
        self.reach = float(reach)
        self.stale_gap = int(stale_gap)
        self.L_ref = -np.inf   # threshold at the last training
        self.floor = -np.inf   # band the network was trained on
        self.cap = np.inf
        # whiten: the network sees z = (theta - mid) / half, with mid and half
        # from the bounding box of its training inputs (enlarged by a quarter),
        # so the live region, however small in the prior box, spans [-1, 1];
        # the surrogate's own box must then be [-1, 1]. cold: every training
        # starts from fresh He-normal weights (needed when the map changes).
        self.whiten = bool(whiten)
        self.cold = bool(cold)
        self.seed = int(seed)
        self.mid = None
        self.half = None

    def _map(self, th):
        return (th - self.mid) / self.half if self.whiten else th

    def _reinit(self):
        """Fresh He-normal weights N(0, 2 / fan_in), zero biases, for every
        member (the flat layout W1 [H, n_in], b1, W2 [H, H], b2, W3 [H], b3)."""
        rng = np.random.default_rng([self.seed, self.n_train])
        M, P = self.s.M, self.s.P
        n_in, H = self.s.n_in, self.s.H
        p = np.zeros((M, P), dtype=np.float32)
        for z in range(M):
            o = 0
            p[z, o:o + H * n_in] = rng.standard_normal(H * n_in) * math.sqrt(2.0 / n_in)
            o += H * n_in + H
            p[z, o:o + H * H] = rng.standard_normal(H * H) * math.sqrt(2.0 / H)
            o += H * H + H
            p[z, o:o + H] = rng.standard_normal(H) * math.sqrt(2.0 / H)
        self.s.set_params(p)

    def observe(self, th, L):
        ok = np.isfinite(L)
        self._th.append(np.asarray(th)[ok])
        self._L.append(np.asarray(L)[ok])
        self._count += int(ok.sum())

    def band_now(self):
        """(floor, cap) of the network's current training targets."""
        return (self.floor, self.cap)

    def censor(self, L, band=None):
        """logL on the scale the network was trained on (that of `band`,
        the (floor, cap) in force when the predictions were made)."""
        if self.band is None:
            return L
        lo, hi = band if band is not None else (self.floor, self.cap)
        return np.clip(L, lo, hi)

    def reject_below(self, L_min, band=None):
        """Line under which a confident prediction is rejected, for
        predictions made on `band` (the (floor, cap) in force when they were
        made; the current one by default): a pool screened before a retraining
        keeps the old network's predictions, on the old band's scale."""
        if self.band is None:
            return L_min
        floor = band[0] if band is not None else self.floor
        return min(L_min, floor + self.reach)

    def _train(self, L_min):
        th = np.concatenate(self._th)
        L = np.concatenate(self._L)
        keep = max(self.window * 4, self.first_train, 1)
        th, L = th[-keep:], L[-keep:]           # bounded history
        self._th, self._L = [th], [L]
        # the first training takes every evaluation made so far (first_train
        # of them), later ones the last `window`
        use = self.window if self.trained else max(self.window, self.first_train)
        if self.band is None:
            near = L >= L_min - self.margin
            if np.count_nonzero(near) >= 256:
                th, L = th[near], L[near]
            th, y = th[-use:], L[-use:]
        else:
            self.floor, self.cap = L_min - self.band[0], L_min + self.band[1]
            th, y = th[-use:], np.clip(L[-use:], self.floor, self.cap)
        t0 = time.perf_counter()
        if self.whiten:
            lo, hi = th.min(axis=0), th.max(axis=0)
            self.mid = 0.5 * (lo + hi)
            self.half = np.maximum(0.625 * (hi - lo), 1e-12)
        if self.cold and self.trained:
            self._reinit()
        self.s.train(self._map(th), y, **(self.retrain_kwargs if self.trained and not self.cold
                                           else self.train_kwargs))
        self.train_seconds += time.perf_counter() - t0
        self.trained = True
        self.n_train += 1
        self.L_ref = L_min

    def maybe_retrain(self, it, L_min):
        """Called at every iteration with the threshold in force: the first
        training, the periodic retraining and the band's re-centring."""
        if not self.trained:
            if self._count >= self.first_train:
                self._last_iter = it
                self._train(L_min)
            return
        due = self.retrain_every > 0 and it - self._last_iter >= self.retrain_every
        stale = (self.band is not None and it - self._last_iter >= self.stale_gap
                 and L_min > self.L_ref + 0.5 * self.band[1])
        if due or stale:
            self._last_iter = it
            self._train(L_min)

    def state(self):
        """(arrays, scalars) of the gate for a checkpoint, the surrogate's
        parameters and standardisation included."""
        th = np.concatenate(self._th) if self._th else np.zeros((0, 0))
        L = np.concatenate(self._L) if self._L else np.zeros(0)
        arrays = {"th": th, "L": L}
        meta = dict(count=self._count, trained=self.trained, n_train=self.n_train,
                    train_seconds=self.train_seconds, last_iter=self._last_iter, L_ref=float(self.L_ref),
                    floor=float(self.floor), cap=float(self.cap),
                    mid=None if self.mid is None else self.mid.tolist(),
                    half=None if self.half is None else self.half.tolist())
        if self.trained:
            p = self.s.get_params()
            arrays["params"] = p.cpu().numpy() if hasattr(p, "cpu") else np.asarray(p)
            meta["standardisation"] = [float(v) for v in self.s.standardisation()]
        return arrays, meta

    def set_state(self, arrays, meta):
        self._th = [arrays["th"].copy()] if arrays["th"].size else []
        self._L = [arrays["L"].copy()] if arrays["L"].size else []
        self._count = int(meta["count"])
        self.trained = bool(meta["trained"])
        self.n_train = int(meta["n_train"])
        self.train_seconds = float(meta["train_seconds"])
        self._last_iter = int(meta["last_iter"])
        self.L_ref, self.floor, self.cap = float(meta["L_ref"]), float(meta["floor"]), float(meta["cap"])
        self.mid = None if meta.get("mid") is None else np.array(meta["mid"])
        self.half = None if meta.get("half") is None else np.array(meta["half"])
        if self.trained:
            self.s.set_params(arrays["params"])
            self.s.standardisation(np.array(meta["standardisation"]))

    def predict(self, th):
        """(mean, spread) of the ensemble for a pool of proposals, or None
        before the first training."""
        if not self.trained:
            return None
        m, sp, _ = self.s.gate(np.ascontiguousarray(self._map(th)), -np.inf, self.tau)
        as_np = (lambda x: x.cpu().numpy()) if hasattr(m, "cpu") else np.asarray
        return as_np(m), as_np(sp)


def exact_gpu(ctx):
    """loglike(theta numpy [B, d]) -> numpy [B] through eor_loglike_batch."""
    import torch

    def f(th):
        L, _ = ctx.loglike_batch(torch.from_numpy(np.ascontiguousarray(th)).cuda())
        return L.cpu().numpy()
    return f


def run_plain_and_gated(ctx, n_dim, lo, hi, surrogate, n_live=500, seed=0, tau=0.05, first_train=100_000,
                        retrain_every=0, window=100_000, margin=np.inf, train_cfg=None, batch=512, dlogz=0.01,
                        audit_frac=0.01, pool_factor=1, progress=0, retrain_cfg=None, band=None, reach=0.2,
                        stale_gap=250, whiten=False, cold=False):
    """The same nested-sampling run without and with the surrogate gate
    (same seed), and the comparison: evidence, per-bin posterior mean and
    standard deviation, exact calls avoided and wall-clock speedup. With
    whiten, the surrogate's own input box must be [-1, 1]."""
    loglike = exact_gpu(ctx)
    plain = NestedSampler(loglike, n_dim, lo, hi, n_live=n_live, dlogz=dlogz, batch=batch, seed=seed,
                          progress=progress).run()
    gate = GatedLikelihood(surrogate, tau=tau, first_train=first_train, retrain_every=retrain_every,
                           window=window, margin=margin,
                           train_kwargs={"cfg": train_cfg} if train_cfg is not None else {},
                           retrain_kwargs={"cfg": retrain_cfg} if retrain_cfg is not None else None,
                           band=band, reach=reach, stale_gap=stale_gap, whiten=whiten, cold=cold, seed=seed)
    gated = NestedSampler(loglike, n_dim, lo, hi, n_live=n_live, dlogz=dlogz, batch=batch, seed=seed,
                          gate=gate, audit_frac=audit_frac, pool_factor=pool_factor, progress=progress).run()
    return plain, gated, compare_runs(plain, gated, n_live)


def compare_runs(plain, gated, n_live):
    """Agreement and cost of a gated run against the plain one: evidence
    (tolerance 3 sqrt(H / n_live)), per-bin posterior means in posterior
    standard deviations, exact calls avoided, wall-clock speedup."""
    m1, s1 = plain.posterior_moments()
    m2, s2 = gated.posterior_moments()
    return {
        "logz_plain": plain.logz, "logz_gated": gated.logz,
        "logz_tolerance": 3.0 * math.sqrt(plain.information / n_live),
        "max_dmean_over_sigma": float(np.max(np.abs(m1 - m2) / s1)),
        "proposals_plain": plain.n_proposed, "proposals_gated": gated.n_proposed,
        "proposals_per_s_plain": plain.n_proposed / plain.wall_s,
        "proposals_per_s_gated": gated.n_proposed / gated.wall_s,
        "max_dstd_rel": float(np.max(np.abs(s2 / s1 - 1.0))),
        "exact_calls_plain": plain.n_exact, "exact_calls_gated": gated.n_exact,
        "exact_calls_avoided_frac": 1.0 - gated.n_exact / plain.n_exact,
        "gate_rejected": gated.n_gate_rejected, "audited": gated.n_audited,
        "false_rejections": gated.n_false_reject,
        "wall_plain_s": plain.wall_s, "wall_gated_s": gated.wall_s,
        "speedup": plain.wall_s / gated.wall_s,
        "train_s": gated.t_train_s, "gate_s": gated.t_gate_s, "retrains": gated.n_retrain,
        "iterations_plain": plain.iterations, "iterations_gated": gated.iterations,
        "confident_checked": gated.n_conf_checked, "confident_max_err": gated.max_conf_err,
    }
