"""Writes the stored fixtures under tests/golden/.

Inputs come from `synth` (seeded); every expected value comes from `oracle`
only. Run from the repository root:

    python tests/golden/make_golden.py digests
    python tests/golden/make_golden.py c1 [n_sample]
    python tests/golden/make_golden.py c3 [n_sample]
    python tests/golden/make_golden.py c2
    python tests/golden/make_golden.py stress [n_sample]

For the 20000 x 4096 workload the fixture also holds theta chosen outside the
batch (`extra_theta`): the corners and edges of the prior box [-1, 3]^12,
points beyond it, the theta the data were drawn at, and seeded uniform draws.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digests():
    with open(os.path.join(HERE, "c0_digest.txt"), "w") as f:
        f.write(synth.gen(0).digest() + "  synth.gen(0)\n")


def extra_theta(n_k, lo, hi, theta_true, n_random=11, seed=3003):
    """Theta beyond the batch's uniform draws: the box corners, alternating
    corners, ramps, one bin at the other end of the box, points outside the
    box, the data's theta and seeded uniform draws."""
    mid = 0.5 * (lo + hi)
    alt = np.where(np.arange(n_k) % 2 == 0, lo, hi)
    rows = [np.full(n_k, lo), np.full(n_k, hi), alt, lo + hi - alt, np.asarray(theta_true, float),
            np.full(n_k, mid), np.linspace(lo, hi, n_k), np.linspace(hi, lo, n_k),
            np.full(n_k, lo - 3.0), np.full(n_k, hi + 4.0)]
    for b, base, val in ((0, lo, hi), (n_k - 1, lo, hi), (n_k // 2, hi, lo)):
        r = np.full(n_k, base)
        r[b] = val
        rows.append(r)
    rng = np.random.default_rng(seed)
    rows.extend(rng.uniform(lo, hi, size=(n_random, n_k)))
    return np.ascontiguousarray(np.array(rows, dtype=np.float64))


def sampled(config_id, n_sample, with_extra=False):
    """Oracle logL at an evenly spaced sample of the config's theta batch
    (and, with_extra, at extra_theta)."""
    import oracle
    orc = oracle.get()
    inst = synth.gen(config_id)
    B = inst.theta.shape[0]
    idx = np.unique(np.linspace(0, B - 1, n_sample).round().astype(int))
    t0 = time.time()
    A, dbar, c, K0 = orc.precompute(inst.T, inst.noise_var, inst.d)
    t1 = time.time()
    print(f"precompute {t1 - t0:.1f} s", flush=True)
    logL, info, terms = orc.loglike(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var,
                                    inst.bin_scale, inst.theta[idx], terms=True)
    t2 = time.time()
    out = {
        "config": config_id,
        "digest": inst.digest(),
        "m": inst.m, "n": inst.n, "n_k": inst.n_k, "B": B,
        "c": c, "K0": K0,
        "dbar_head": [[float(z.real), float(z.imag)] for z in dbar[:8]],
        "A_samples": [[int(j), int(k), float(A[j, k].real), float(A[j, k].imag)]
                      for j, k in [(0, 0), (1, 0), (5, 3), (inst.n - 1, 0), (inst.n - 1, inst.n - 1),
                                   (inst.n // 2, inst.n // 3), (inst.n - 2, inst.n // 2)]],
        "index": idx.tolist(),
        "logL": logL.tolist(),
        "info": info.tolist(),
        "terms": terms.tolist(),
        "oracle_seconds": {"precompute": t1 - t0, "loglike": t2 - t1},
    }
    if with_extra:
        th = extra_theta(inst.n_k, inst.lo, inst.hi, inst.theta_true)
        xl, xi, xt = orc.loglike(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var,
                                 inst.bin_scale, th, terms=True)
        out["extra_theta"] = th.tolist()
        out["extra_logL"] = xl.tolist()
        out["extra_info"] = xi.tolist()
        out["extra_terms"] = xt.tolist()
        out["oracle_seconds"]["extra"] = time.time() - t2
    with open(os.path.join(HERE, f"c{config_id}_oracle_sample.json"), "w") as f:
        json.dump(out, f, indent=1)


def group_sampled(pick=(11, 17, 9), n_theta=2):
    """Oracle logL for the first theta of three of the 48 uneven sub-band
    instances (the smallest, the median and the largest n)."""
    import oracle
    orc = oracle.get()
    out = {"instances": {}}
    for idx, inst in enumerate(synth.gen_group()):
        if idx not in pick:
            continue
        t0 = time.time()
        logL, info = orc.loglike_instance(inst, theta=inst.theta[:n_theta])
        out["instances"][str(idx)] = {"n": inst.n, "m": inst.m, "n_k": inst.n_k,
                                      "B": int(inst.theta.shape[0]), "digest": inst.digest(),
                                      "logL": logL.tolist(), "info": info.tolist(),
                                      "oracle_seconds": time.time() - t0}
        print(idx, inst.n, time.time() - t0, flush=True)
    with open(os.path.join(HERE, "c2_oracle_sample.json"), "w") as f:
        json.dump(out, f, indent=1)


def stress_sampled(n_sample=8):
    """Oracle logL at an evenly spaced sample of the theta batch of each
    full-size ill-conditioned instance (synth.STRESS: T with singular values
    over four decades, with the usual foreground share and with a wide-field
    foreground model)."""
    import oracle
    orc = oracle.get()
    out = {"cases": {}}
    for name in sorted(synth.STRESS):
        inst = synth.gen_stress(name)
        B = inst.theta.shape[0]
        idx = np.unique(np.linspace(0, B - 1, n_sample).round().astype(int))
        t0 = time.time()
        logL, info = orc.loglike_instance(inst, theta=inst.theta[idx])
        out["cases"][name] = {"digest": inst.digest(), "m": inst.m, "n": inst.n, "n_k": inst.n_k, "B": B,
                              "index": idx.tolist(), "logL": logL.tolist(), "info": info.tolist(),
                              "oracle_seconds": time.time() - t0}
        print(name, time.time() - t0, flush=True)
    with open(os.path.join(HERE, "stress_oracle_sample.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "digests":
        digests()
    elif what == "c2":
        group_sampled()
    elif what == "stress":
        stress_sampled(int(sys.argv[2]) if len(sys.argv) > 2 else 8)
    else:
        cid = int(what[1:])
        sampled(cid, int(sys.argv[2]) if len(sys.argv) > 2 else 8, with_extra=(cid == 3))
