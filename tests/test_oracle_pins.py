"""Pins of the CPU oracle against routes that do not share its arithmetic.

The oracle takes the Woodbury / determinant-lemma route (A, dbar, Cholesky).
Every pin here reaches the same number another way: dense data-space LU,
50-digit mpmath, closed forms for a diagonal instrument and a one-bin prior,
exact invariances of the model, and the sampling distribution of the data.
"""
import math

import numpy as np
import pytest

import synth
from tests import _pins


def test_generator_is_deterministic():
    a = synth.gen(0)
    b = synth.gen(0)
    assert a.digest() == b.digest()
    assert a.T.shape == (480, 200) and a.theta.shape == (64, 3)
    assert np.all(a.noise_var >= 0.5) and np.all(a.noise_var <= 2.0)
    assert (a.bin_of >= 0).sum() == 160 and (a.bin_of < 0).sum() == 40
    np.testing.assert_array_equal(np.bincount(a.bin_of[a.bin_of >= 0]), [54, 53, 53])


def test_generator_digest_pinned():
    # Written by tests/golden/make_golden.py from synth only; guards against a
    # change in numpy's generator or in the draw order.
    ref = open(_golden("c0_digest.txt")).read().split()[0]
    assert synth.gen(0).digest() == ref


def _golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


def test_brute_force_c0(orc):
    """D1 with a dense 480x480 C (LU) on the tiny workload, all 64 theta."""
    inst = synth.gen(0)
    logL, info = orc.loglike_instance(inst)
    assert np.all(info == 0)
    ref = np.array([_pins.brute_loglike(inst.T, inst.noise_var, inst.d, th, inst.bin_of,
                                        inst.fixed_var) for th in inst.theta])
    assert np.max(_pins.rel_err(logL, ref)) < 1e-12


def test_mpmath_50_digits(orc):
    """D1 at 50 digits on a tiny instance with EoR and foreground columns."""
    inst = synth.small(seed=7, m=18, n=8, n_k=2, n_eor=6, n_theta=2)
    logL, info = orc.loglike_instance(inst)
    assert np.all(info == 0)
    for t in range(inst.theta.shape[0]):
        ref = _pins.brute_loglike_mp(inst.T, inst.noise_var, inst.d, inst.theta[t],
                                     inst.bin_of, inst.fixed_var)
        assert abs(logL[t] - ref) <= 1e-12 * abs(ref)


def test_closed_form_diagonal_instrument(orc):
    """T = [I_n; 0]: logL is a sum of independent 1-D Gaussians."""
    rng = np.random.default_rng(11)
    m, n, n_k = 300, 220, 5
    T = np.zeros((m, n), dtype=np.complex128)
    T[np.arange(n), np.arange(n)] = 1.0
    inst = synth.make_instance(rng, m=m, n=n, n_k=n_k, n_eor=180, n_theta=6,
                               lo=-1.0, hi=3.0, T=T)
    logL, info = orc.loglike_instance(inst)
    assert np.all(info == 0)
    ref = [_pins.diagonal_closed_form(inst.noise_var, inst.d, th, inst.bin_of,
                                      inst.fixed_var, n) for th in inst.theta]
    assert np.max(_pins.rel_err(logL, ref)) < 1e-12


def test_closed_form_one_bin_eigen(orc):
    """One bin, no fixed columns: exact logL(theta) curve from eigh(A)."""
    rng = np.random.default_rng(12)
    m, n = 160, 96
    inst = synth.make_instance(rng, m=m, n=n, n_k=1, n_eor=n, n_theta=1, lo=-1, hi=3)
    grid = np.linspace(-3.0, 5.0, 9)
    logL, info = orc.loglike_instance(inst, theta=grid[:, None])
    assert np.all(info == 0)
    ref = _pins.eigen_closed_form(inst.T, inst.noise_var, inst.d, grid)
    assert np.max(_pins.rel_err(logL, ref)) < 1e-12


def test_bin_scale_matches_shifted_theta(orc):
    """phi = s_b 10^theta_b: a scale s_b equals a shift of theta_b by log10 s_b."""
    inst = synth.small(seed=3, m=40, n=24, n_k=3, n_theta=4)
    s = np.array([2.0, 0.25, 10.0])
    pre = orc.precompute(inst.T, inst.noise_var, inst.d)
    a, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, s, inst.theta)
    b, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, None,
                       inst.theta + np.log10(s)[None, :])
    np.testing.assert_allclose(a, b, rtol=1e-13)


def _unitary(rng, k):
    q, r = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_invariants(orc):
    """(I1) T -> T U, U unitary inside each bin and inside the equal-variance
    fixed block; (I2) column permutation with the bin map; (I3) T -> alpha T
    with s, v -> s/alpha^2, v/alpha^2; (I4) theta_b -> -40 equals deleting
    bin b's columns."""
    rng = np.random.default_rng(5)
    inst = synth.small(seed=5, m=60, n=32, n_k=3, n_theta=5)
    base, _ = orc.loglike_instance(inst)

    # I1
    T1 = inst.T.copy()
    for b in list(range(inst.n_k)) + [-1]:
        idx = np.flatnonzero(inst.bin_of == b)
        T1[:, idx] = T1[:, idx] @ _unitary(rng, idx.size)
    pre1 = orc.precompute(T1, inst.noise_var, inst.d)
    r1, _ = orc.loglike(*pre1, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta)
    np.testing.assert_allclose(r1, base, rtol=1e-12)

    # I2
    p = rng.permutation(inst.n)
    pre2 = orc.precompute(inst.T[:, p], inst.noise_var, inst.d)
    r2, _ = orc.loglike(*pre2, inst.n_k, inst.bin_of[p], inst.fixed_var[p], None, inst.theta)
    np.testing.assert_allclose(r2, base, rtol=1e-12)

    # I3
    alpha = 3.7
    pre3 = orc.precompute(alpha * inst.T, inst.noise_var, inst.d)
    r3, _ = orc.loglike(*pre3, inst.n_k, inst.bin_of, inst.fixed_var / alpha ** 2,
                        np.full(inst.n_k, 1.0 / alpha ** 2), inst.theta)
    np.testing.assert_allclose(r3, base, rtol=1e-12)

    # I4
    b = 1
    keep = inst.bin_of != b
    th = inst.theta.copy()
    th[:, b] = -40.0
    r4, _ = orc.loglike_instance(inst, theta=th)
    bins_k = inst.bin_of[keep].copy()
    bins_k[bins_k > b] -= 1
    th_k = np.delete(inst.theta, b, axis=1)
    pre4 = orc.precompute(inst.T[:, keep], inst.noise_var, inst.d)
    r4k, _ = orc.loglike(*pre4, inst.n_k - 1, bins_k, inst.fixed_var[keep], None, th_k)
    np.testing.assert_allclose(r4, r4k, rtol=1e-12)


def test_independent_blocks_add_under_mixing(orc):
    """(I6) Four independent problems with the same bins, stacked
    block-diagonally (data rows and noise concatenated) and mixed coefficient
    by coefficient with a random 4 x 4 unitary across the blocks: every mixed
    coefficient has the same prior variance, so the data covariance and the
    logL are those of the four problems side by side, the sum of their logL.
    The same construction checks the GPU path at sizes the oracle cannot
    reach; a block of T scaled by 1.01 must break it."""
    rng = np.random.default_rng(16384)
    n1, m1, n_k, n_eor, nb = 48, 70, 3, 40, 4
    parts = [synth.make_instance(rng, m=m1, n=n1, n_k=n_k, n_eor=n_eor, n_theta=1, lo=-1.0, hi=3.0)
             for _ in range(nb)]
    theta = np.ascontiguousarray(np.stack([parts[0].theta[0], np.full(n_k, -1.0), np.full(n_k, 3.0)]))
    U = np.stack([_unitary(rng, nb) for _ in range(n1)])
    T = np.empty((nb * m1, nb * n1), dtype=np.complex128)
    for r, p in enumerate(parts):
        for c in range(nb):
            T[r * m1:(r + 1) * m1, c * n1:(c + 1) * n1] = p.T * U[None, :, r, c]
    noise = np.concatenate([p.noise_var for p in parts])
    d = np.concatenate([p.d for p in parts])
    bins = np.concatenate([p.bin_of for p in parts])
    fixed = np.concatenate([p.fixed_var for p in parts])
    ref = sum(orc.loglike_instance(p, theta=theta)[0] for p in parts)
    got, _ = orc.loglike(*orc.precompute(T, noise, d), n_k, bins, fixed, None, theta)
    np.testing.assert_allclose(got, ref, rtol=1e-11)
    T[:m1, :n1] *= 1.01
    bad, _ = orc.loglike(*orc.precompute(T, noise, d), n_k, bins, fixed, None, theta)
    assert np.all(np.abs(bad - ref) > 1e-3)


def test_batch_position_independent(orc):
    """(I5) logL[b] does not depend on B or the order of the batch."""
    inst = synth.small(seed=9, m=50, n=30, n_k=4, n_theta=12)
    pre = orc.precompute(inst.T, inst.noise_var, inst.d)
    full, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta)
    p = np.random.default_rng(0).permutation(12)
    perm, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta[p])
    one, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta[3:4])
    assert np.array_equal(perm, full[p]) and one[0] == full[3]


def test_quadratic_form_is_gamma_m(orc):
    """At the true theta, d^H C^{-1} d ~ Gamma(m, 1) under the circular
    complex Gaussian convention (mean m, variance m): catches a factor-2
    convention error or a dropped weight."""
    m, n, n_k = 40, 16, 2
    vals = []
    for s in range(200):
        inst = synth.small(seed=100 + s, m=m, n=n, n_k=n_k, n_theta=1)
        _, info, terms = orc.loglike_instance(inst, theta=inst.theta_true[None, :], terms=True)
        pre = orc.precompute(inst.T, inst.noise_var, inst.d)
        c = pre[2]
        vals.append(c - terms[0, 1])
    vals = np.array(vals)
    assert abs(vals.mean() - m) < 4.0 * math.sqrt(m / len(vals))
    assert abs(vals.var() / m - 1.0) < 0.35


def test_score_has_zero_mean(orc):
    """E[d logL / d theta_b] = 0 at the true theta (finite differences of the
    oracle over independent data draws)."""
    m, n, n_k = 48, 24, 3
    h = 1e-5
    grads = []
    for s in range(150):
        inst = synth.small(seed=500 + s, m=m, n=n, n_k=n_k, n_eor=20, n_theta=1)
        th = np.repeat(inst.theta_true[None, :], 2 * n_k, axis=0)
        for b in range(n_k):
            th[2 * b, b] += h
            th[2 * b + 1, b] -= h
        L, _ = orc.loglike_instance(inst, theta=th)
        grads.append((L[0::2] - L[1::2]) / (2 * h))
    g = np.array(grads)
    se = g.std(axis=0, ddof=1) / math.sqrt(g.shape[0])
    assert np.all(np.abs(g.mean(axis=0)) < 4.0 * se)


def test_non_finite_and_non_hpd(orc):
    inst = synth.small(seed=2, m=30, n=16, n_k=2, n_theta=3)
    th = inst.theta.copy()
    th[1, 0] = np.nan
    logL, info = orc.loglike_instance(inst, theta=th)
    assert info[1] == -1 and logL[1] == -np.inf
    assert info[0] == 0 and np.isfinite(logL[0])
    A, dbar, c, K0 = orc.precompute(inst.T, inst.noise_var, inst.d)
    A = A.copy()
    A[5, 5] = -1e6   # corrupt the diagonal: Sigma is not positive definite
    logL, info = orc.loglike(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta)
    assert np.all(info == 6) and np.all(logL == -np.inf)


@pytest.mark.parametrize("mutant", list(range(1, 9)))
def test_planted_mistake_fails_a_pin(mutant, tmp_path):
    """Each planted mistake in the oracle (transposed operand, dropped weight,
    wrong constant, shifted bin index, dropped ln det Phi, flipped sign,
    inverted prior precision, missing conjugate) is caught by brute force."""
    import oracle
    mut = oracle.Oracle(mutant=mutant, out_dir=str(tmp_path))
    assert mut.lib.oracle_build_id() == b"oracle-mutant"
    inst = synth.small(seed=21, m=40, n=20, n_k=3, n_eor=16, n_theta=3)
    logL, _ = mut.loglike_instance(inst)
    ref = np.array([_pins.brute_loglike(inst.T, inst.noise_var, inst.d, th, inst.bin_of,
                                        inst.fixed_var) for th in inst.theta])
    assert np.max(_pins.rel_err(logL, ref)) > 1e-6


def test_stress_generator_is_host_independent_and_ill_conditioned():
    """The ill-conditioned instances are built with elementwise arithmetic
    only, so the stored full-size oracle values stay valid: their digests
    match the generator here. T's singular values spread over about the four
    decades of its column scales."""
    import json
    g = json.load(open(_golden("stress_oracle_sample.json")))["cases"]
    for name in sorted(synth.STRESS):
        assert synth.gen_stress(name).digest() == g[name]["digest"], name
    sv = np.linalg.svd(synth.stress(35, m=700, n=300, n_k=3).T, compute_uv=False)
    assert 3e3 < sv[0] / sv[-1] < 1e5
