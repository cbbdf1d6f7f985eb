"""Gated nested sampling with the GPU likelihood and the GPU surrogate on
a small dataset: the gated run agrees with the plain run (same seed) in
evidence and posterior, every accepted point carries its exact logL, and
the surrogate rejects proposals without exact calls with a false-rejection
rate within 5% of the audited ones. (What the gate saves in time depends
on the cost of an exact call; the benchmark measures it at n = 4096.)

Agreement is the reading's: per-bin posterior means within 0.1 posterior
standard deviation and |d ln Z| within 3 sqrt(H / n_live). Once the gate is
trained the two runs draw different proposals, so they differ like two
independent runs; 1000 live points keep that difference well inside the
bar."""
import numpy as np
import pytest

import synth
from tests.gpu_util import have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]


def test_gated_sampler_agrees_with_plain(orc):
    import torch
    import paper_2501_12928_amd as eor
    from paper_2501_12928_amd.sampler import run_plain_and_gated
    inst = synth.small(seed=42, m=600, n=192, n_k=3, n_eor=168, n_theta=1)
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    sur = eor.Surrogate(inst.n_k, inst.lo, inst.hi, n_members=5, hidden=64, seed=1)
    cfg = eor.train_cfg(epochs=40, minibatch=256, patience=8, lr=1e-3, seed=5)
    print("gpu: plain and gated nested sampling, n=192, 3 bins", flush=True)
    plain, gated, cmp = run_plain_and_gated(ctx, inst.n_k, inst.lo, inst.hi, sur, n_live=1000, seed=3,
                                            tau=0.05, first_train=1500, retrain_every=250, window=3000,
                                            margin=30.0, train_cfg=cfg, batch=256, dlogz=0.05,
                                            audit_frac=0.05)
    print(cmp, flush=True)
    assert abs(cmp["logz_plain"] - cmp["logz_gated"]) < cmp["logz_tolerance"]
    assert cmp["max_dmean_over_sigma"] < 0.1
    assert cmp["gate_rejected"] > 0
    # what the trained network gains: exact calls the plain run makes and the gated one does not
    assert cmp["exact_calls_gated"] < cmp["exact_calls_plain"]
    assert cmp["false_rejections"] <= 0.05 * max(cmp["audited"], 1) + 1
    # accepted points carry exact logL: check a sample against the oracle
    idx = np.random.default_rng(0).choice(gated.samples.shape[0], 16, replace=False)
    ref, _ = orc.loglike_instance(inst, theta=gated.samples[idx])
    assert np.all(np.abs(gated.logl[idx] - ref) <= 1e-6 * np.abs(ref) + 1e-6)
    # the posterior concentrates near the truth the data were drawn at
    mean, std = gated.posterior_moments()
    assert np.all(np.abs(mean - inst.theta_true) < 5 * std + 0.2)
    sur.close()
    ctx.close()


def test_band_gate_agrees_with_plain(orc):
    """The gate as the benchmark runs it (targets censored to a band around
    the threshold, inputs mapped to the training box, fresh weights per
    training, rejections trusted only at the band's floor) against the plain
    run with the same seed: evidence and posterior agree, the gate rejects
    proposals, every audited rejection lies under the floor rule's line, and
    false rejections are rare."""
    import torch
    import paper_2501_12928_amd as eor
    from paper_2501_12928_amd.sampler import run_plain_and_gated
    inst = synth.small(seed=42, m=600, n=192, n_k=3, n_eor=168, n_theta=1)
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    sur = eor.Surrogate(inst.n_k, -1.0, 1.0, n_members=5, hidden=64, seed=1)
    cfg = eor.train_cfg(epochs=100, minibatch=256, patience=20, lr=1e-3, seed=5)
    print("gpu: plain and band-gated nested sampling, n=192, 3 bins", flush=True)
    plain, gated, cmp = run_plain_and_gated(ctx, inst.n_k, inst.lo, inst.hi, sur, n_live=1000, seed=3,
                                            tau=0.05, first_train=3000, retrain_every=500, window=3000,
                                            train_cfg=cfg, batch=256, dlogz=0.05, audit_frac=0.2,
                                            band=(0.5, 1.0), reach=0.2, stale_gap=100, whiten=True, cold=True)
    print(cmp, flush=True)
    assert abs(cmp["logz_plain"] - cmp["logz_gated"]) < cmp["logz_tolerance"]
    assert cmp["max_dmean_over_sigma"] < 0.1
    assert cmp["gate_rejected"] > 0 and cmp["audited"] > 0
    assert cmp["false_rejections"] <= 0.01 * cmp["audited"] + 1
    L, L_min, mean, spread, floor, cap, it = gated.audit_log.T
    assert np.all(mean < np.minimum(L_min, floor + 0.2)) and np.all(spread <= 0.05)
    idx = np.random.default_rng(1).choice(gated.samples.shape[0], 16, replace=False)
    ref, _ = orc.loglike_instance(inst, theta=gated.samples[idx])
    assert np.all(np.abs(gated.logl[idx] - ref) <= 1e-6 * np.abs(ref) + 1e-6)
    sur.close()
    ctx.close()
