"""Nested sampler (host logic) on closed-form problems: a Gaussian in a
uniform box has an analytic evidence; gating with a perfect surrogate must
keep the answer while avoiding exact calls; a gate that never rejects must
reproduce the ungated run exactly."""
import math

import numpy as np
from scipy.special import erf

from paper_2501_12928_amd.sampler import Ellipsoid, GatedLikelihood, NestedSampler

MU = np.array([0.3, -0.2, 1.0, 0.5])
SIG = 0.5
LO, HI = -5.0, 5.0


def gauss_loglike(th):
    th = np.atleast_2d(th)
    d = th.shape[1]
    return -0.5 * np.sum((th - MU[:d]) ** 2, axis=1) / SIG ** 2 - 0.5 * d * math.log(2 * math.pi * SIG ** 2)


def gauss_logz(d):
    """ln Z = ln( prod_k P(LO < x_k < HI) / (HI - LO)^d ) for the unit-mass Gaussian."""
    mass = 1.0
    for k in range(d):
        a = (LO - MU[k]) / (SIG * math.sqrt(2))
        b = (HI - MU[k]) / (SIG * math.sqrt(2))
        mass *= 0.5 * (erf(b) - erf(a))
    return math.log(mass) - d * math.log(HI - LO)


class PerfectSurrogate:
    """Stand-in with the surrogate interface: exact mean, zero spread."""

    def __init__(self, spread=0.0):
        self.spread = spread
        self.trained_on = 0

    def train(self, th, L):
        self.trained_on = th.shape[0]

    def gate(self, th, L_min, tau):
        m = gauss_loglike(th)
        s = np.full(th.shape[0], self.spread)
        dec = np.where((s <= tau) & (m < L_min), 0, 1).astype(np.int32)
        return m, s, dec


def test_gaussian_evidence_and_posterior():
    d = 4
    ns = NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=1)
    r = ns.run()
    truth = gauss_logz(d)
    assert abs(r.logz - truth) < 4 * r.logz_err + 0.02, (r.logz, truth, r.logz_err)
    mean, std = r.posterior_moments()
    assert np.all(np.abs(mean - MU) < 0.05)
    assert np.all(np.abs(std / SIG - 1) < 0.12)
    # information of a Gaussian in a wide box: H = ln(V / (2 pi e sigma^2)^(d/2)) approx.
    H_true = d * math.log(HI - LO) - 0.5 * d * math.log(2 * math.pi * math.e * SIG ** 2)
    assert abs(r.information - H_true) < 0.3
    # power recovery: theta ~ N(mu, sigma^2) gives E[10^theta] = 10^mu exp((sigma ln 10)^2 / 2),
    # median mu and 16-84% interval mu +- sigma
    k = np.array([0.1, 0.2, 0.5, 1.0])
    ps = r.power_summary(theta_true=MU[:d], k=k)
    expect = 10.0 ** MU[:d] * math.exp((SIG * math.log(10.0)) ** 2 / 2)
    np.testing.assert_allclose(ps["power_mean"], expect, rtol=0.12)
    # lognormal spread: std[10^theta] = E[10^theta] sqrt(exp((sigma ln 10)^2) - 1); eq. 2 scales
    # both moments by k^3 / (2 pi^2)
    sd_expect = expect * math.sqrt(math.exp((SIG * math.log(10.0)) ** 2) - 1.0)
    np.testing.assert_allclose(ps["power_std"], sd_expect, rtol=0.25)
    c = k ** 3 / (2 * math.pi ** 2)
    np.testing.assert_allclose(ps["delta2_mean"], c * expect, rtol=0.12)
    np.testing.assert_allclose(ps["delta2_std"], c * sd_expect, rtol=0.25)
    np.testing.assert_allclose(ps["delta2_true"], c * 10.0 ** MU[:d], rtol=1e-12)
    np.testing.assert_allclose(ps["theta_median"], MU[:d], atol=0.06)
    np.testing.assert_allclose(np.array(ps["theta_hi"]) - np.array(ps["theta_lo"]), 2 * SIG, rtol=0.12)
    assert np.all(np.abs(ps["theta_offset_sigma"]) < 0.15)


def test_gated_perfect_surrogate_keeps_answer_with_fewer_exact_calls():
    d = 4
    plain = NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=2).run()
    gate = GatedLikelihood(PerfectSurrogate(), tau=0.05, first_train=2000)
    gated = NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=2,
                          gate=gate, audit_frac=0.05).run()
    assert gate.n_train == 1
    assert abs(gated.logz - plain.logz) < 3 * math.sqrt(plain.logz_err ** 2 + gated.logz_err ** 2)
    m1, s1 = plain.posterior_moments()
    m2, s2 = gated.posterior_moments()
    assert np.all(np.abs(m1 - m2) < 0.15 * s1)
    assert gated.n_gate_rejected > 0 and gated.n_false_reject == 0 and gated.n_audited > 0
    assert gated.n_exact < 0.8 * plain.n_exact
    # every accepted sample carries its exact logL
    np.testing.assert_array_equal(gated.logl, gauss_loglike(gated.samples))


def test_gate_that_never_rejects_reproduces_plain_run():
    """With pools of one exact batch, a gate that is never confident leaves
    every decision to the exact likelihood: the run is the plain run."""
    d = 3
    plain = NestedSampler(gauss_loglike, d, LO, HI, n_live=100, dlogz=0.05, batch=128, seed=3).run()
    gate = GatedLikelihood(PerfectSurrogate(spread=1.0), tau=0.05, first_train=500)
    gated = NestedSampler(gauss_loglike, d, LO, HI, n_live=100, dlogz=0.05, batch=128, seed=3, gate=gate,
                          pool_factor=1).run()
    assert gated.n_gate_rejected == 0
    assert gated.logz == plain.logz
    np.testing.assert_array_equal(gated.samples, plain.samples)


def test_ellipsoid_bounds_and_volume():
    rng = np.random.default_rng(4)
    pts = rng.standard_normal((400, 3)) @ np.array([[1.0, 0.2, 0], [0, 0.5, 0.1], [0, 0, 2.0]])
    ell = Ellipsoid(pts, 1.5)
    Li = np.linalg.inv(ell.L)
    r = np.linalg.norm((pts - ell.mu) @ Li.T, axis=1)
    assert np.all(r <= 1.0 + 1e-9)
    # the enlarged ellipsoid's volume is 1.5 times the tight one's
    tight = Ellipsoid(pts, 1.0)
    ratio = abs(np.linalg.det(ell.L) / np.linalg.det(tight.L))
    assert abs(ratio - 1.5) < 1e-9
    x = ell.sample(rng, 20000)
    rx = np.linalg.norm((x - ell.mu) @ Li.T, axis=1)
    assert np.all(rx <= 1.0 + 1e-9)
    # uniform in the ball: P(r < 0.5) = 0.5^3
    assert abs(np.mean(rx < 0.5) - 0.125) < 0.01


class CensoredSurrogate:
    """Stand-in that learns the censoring band it is trained on: its mean is
    the exact logL clipped to [min(y), max(y)] of the last training targets,
    with zero spread; parameters are the band itself."""

    def __init__(self):
        self.lo, self.hi = -np.inf, np.inf
        self.n_trained = 0

    def train(self, th, y, **kw):
        self.lo, self.hi = float(np.min(y)), float(np.max(y))
        self.n_trained += 1

    def gate(self, th, L_min, tau):
        m = np.clip(gauss_loglike(th), self.lo, self.hi)
        s = np.zeros(th.shape[0])
        return m, s, np.where(m < L_min, 0, 1).astype(np.int32)

    def get_params(self):
        return np.array([[self.lo, self.hi]])

    def set_params(self, p):
        self.lo, self.hi = float(p[0][0]), float(p[0][1])

    def standardisation(self, mean_std=None):
        return np.array([0.0, 1.0]) if mean_std is None else mean_std


def test_censored_band_gate_keeps_the_answer():
    """Trained on logL censored to a band around the threshold, a surrogate
    that is exact on that scale rejects only proposals below the threshold
    (audits find no false rejection), keeps evidence and posterior, and
    avoids exact calls: the floor catches every proposal far below, whatever
    the distance."""
    d = 4
    plain = NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=5).run()
    sur = CensoredSurrogate()
    gate = GatedLikelihood(sur, tau=0.05, first_train=1500, retrain_every=2000, window=3000,
                           band=(2.0, 3.0), reach=1.5, stale_gap=10)
    gated = NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=5,
                          gate=gate, audit_frac=0.2).run()
    assert sur.n_trained > 3          # the band was re-centred as the threshold climbed
    assert gated.n_false_reject == 0 and gated.n_audited > 50
    assert abs(gated.logz - plain.logz) < 3 * math.sqrt(plain.logz_err ** 2 + gated.logz_err ** 2)
    m1, s1 = plain.posterior_moments()
    m2, _ = gated.posterior_moments()
    assert np.all(np.abs(m1 - m2) < 0.15 * s1)
    assert gated.n_exact < 0.9 * plain.n_exact   # only what lies below the floor + reach is saved
    np.testing.assert_array_equal(gated.logl, gauss_loglike(gated.samples))
    assert gated.n_conf_checked > 0
    # a rejection is trusted only at the floor: within `reach` of it, and below L_min
    assert gate.reject_below(gate.cap + 10.0) == gate.floor + 1.5
    assert gate.reject_below(gate.floor + 1.25) == gate.floor + 1.25
    # predictions made before a retraining are judged on their own band
    assert gate.reject_below(gate.cap + 10.0, band=(gate.floor - 7.0, gate.cap - 7.0)) == gate.floor - 5.5


def test_checkpoint_and_resume_reproduce_the_run(tmp_path):
    """A run stopped at a time limit and resumed from its checkpoint, over and
    over, ends with the same samples, weights and counters as the run made in
    one go (gated, with a deterministic stand-in surrogate)."""
    d = 3

    def make():
        gate = GatedLikelihood(CensoredSurrogate(), tau=0.05, first_train=600, retrain_every=500,
                               window=2000, band=(2.0, 3.0), reach=0.5, stale_gap=40)
        return NestedSampler(gauss_loglike, d, LO, HI, n_live=150, dlogz=0.05, batch=128, seed=9,
                             gate=gate, audit_frac=0.1)

    whole = make().run()
    path = str(tmp_path / "ns.npz")
    r, parts = make().run(time_limit=0.005, checkpoint=path), 1
    while r is None:
        r = make().run(time_limit=0.005, checkpoint=path, resume=path)
        parts += 1
    assert parts > 3
    np.testing.assert_array_equal(r.samples, whole.samples)
    np.testing.assert_array_equal(r.logw, whole.logw)
    assert r.logz == whole.logz and r.iterations == whole.iterations
    assert (r.n_exact, r.n_proposed, r.n_gate_rejected, r.n_audited, r.n_retrain) == \
        (whole.n_exact, whole.n_proposed, whole.n_gate_rejected, whole.n_audited, whole.n_retrain)
    # the audits keep what the gate saw across the checkpoints
    np.testing.assert_array_equal(r.audit_log, whole.audit_log)
    assert r.audit_log.shape == (whole.n_audited, 7) and np.all(np.isfinite(r.audit_log))


class GrossErrorSurrogate(CensoredSurrogate):
    """Exact on the censored scale except for a fixed pseudo-random fifth of
    the points, which read in the middle of the band with zero spread (the
    network's gross errors under a stale band: points far above the
    threshold placed inside the band)."""

    W = np.array([12.9898, 78.233, 37.719, 4.581])

    def gate(self, th, L_min, tau):
        m, s, _ = super().gate(th, L_min, tau)
        u = np.modf(np.abs(np.sin(th @ self.W[:th.shape[1]]) * 43758.5453))[0]
        m = np.where(u < 0.2, 0.5 * (self.lo + self.hi), m)
        return m, s, None


def test_floor_rule_never_trusts_mid_band_predictions():
    """A rejection is trusted only within `reach` of the band's floor: the
    gross errors of GrossErrorSurrogate never cause one (audits find no false
    rejection and the evidence matches the closed form), while a reach across
    the band, which trusts anything read below the threshold, rejects valid
    points that the audits then find."""
    d = 4
    truth = gauss_logz(d)

    def run(reach):
        gate = GatedLikelihood(GrossErrorSurrogate(), tau=0.05, first_train=1500, retrain_every=2000,
                               window=3000, band=(0.5, 1.0), reach=reach, stale_gap=50)
        return NestedSampler(gauss_loglike, d, LO, HI, n_live=300, dlogz=0.01, batch=256, seed=8,
                             gate=gate, audit_frac=0.2).run()

    safe, loose = run(0.2), run(1.5)
    assert safe.n_gate_rejected > 0 and safe.n_audited > 50 and safe.n_false_reject == 0
    assert abs(safe.logz - truth) < 4 * safe.logz_err + 0.02
    assert loose.n_false_reject > 0
    # every audited row records what the gate saw: rejected below its line
    L, L_min, mean, spread, floor, cap, it = safe.audit_log.T
    assert np.all(mean < np.minimum(L_min, floor + 0.2)) and np.all(spread <= 0.05)
    assert np.all(L <= L_min) and np.all(np.diff(it) >= 0)


def test_result_file_round_trip(tmp_path):
    """save_result / load_result keep every field, the audit log included
    (arrays and JSON scalars, no pickles), and files without an audit log
    load with audit_log None."""
    from paper_2501_12928_amd.sampler import AUDIT_COLUMNS, load_result, save_result
    d = 3
    gate = GatedLikelihood(CensoredSurrogate(), tau=0.05, first_train=600, retrain_every=500,
                           window=2000, band=(2.0, 3.0), reach=1.5, stale_gap=40)
    r = NestedSampler(gauss_loglike, d, LO, HI, n_live=150, dlogz=0.05, batch=128, seed=4,
                      gate=gate, audit_frac=0.2).run()
    assert r.audit_log.shape == (r.n_audited, len(AUDIT_COLUMNS)) and r.n_audited > 0
    path = str(tmp_path / "r.npz")
    save_result(path, r)
    back = load_result(path)
    for f in ("samples", "logl", "logw", "audit_log"):
        np.testing.assert_array_equal(getattr(back, f), getattr(r, f))
    assert (back.logz, back.iterations, back.n_exact, back.n_audited) == (r.logz, r.iterations, r.n_exact,
                                                                          r.n_audited)
    plain = NestedSampler(gauss_loglike, d, LO, HI, n_live=100, dlogz=0.05, batch=128, seed=4).run()
    plain.audit_log = None
    save_result(path, plain)
    assert load_result(path).audit_log is None
