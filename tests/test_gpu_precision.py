"""Reduced-precision A = W^H W (W = T / sigma): FP32 and split-BF16 on MFMA
with FP32 accumulation per 64-row chunk and FP64 across chunks.

Pins: the oracle's FP64 A, entry by entry, within a componentwise rounding
bound, and logL within the required tolerance; dbar and c stay FP64.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import have_gpu, run_instance, tol

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]

U32 = 2.0 ** -24   # unit roundoff of FP32
CHUNK = 64


def _export(inst, prec):
    import torch
    import paper_2501_12928_amd as eor
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var, prec=prec)
    A, dbar, c, K0 = ctx.export_precompute()
    out = A.cpu().numpy(), dbar.cpu().numpy(), c, K0
    ctx.close()
    return out


def _bound(inst):
    """Componentwise bound on |A_red - A| for either scheme:
    (rounding of W to FP32 or to three bfloat16 terms and the dropped
    cross products: below 8u per real product) + (FP32 accumulation over a
    64-row chunk: gamma_64 <= 65u), times the two real products that make
    each real or imaginary part: 2 (8 + 65) u sum_s |W_sj| |W_sk|."""
    W = np.abs(inst.T) / np.sqrt(inst.noise_var)[:, None]
    return 2.0 * (8 + CHUNK + 1) * U32 * (W.T @ W)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape", [(480, 200), (700, 300), (1030, 129)])
def test_reduced_precision_A_within_bound(orc, prec, shape):
    m, n = shape
    inst = synth.small(seed=m + 3 * n, m=m, n=n, n_k=3, n_theta=4)
    A64, dbar64, c64, K064 = orc.precompute(inst.T, inst.noise_var, inst.d)
    print(f"gpu: reduced precision {prec} m={m} n={n}", flush=True)
    A, dbar, c, K0 = _export(inst, prec)
    err = np.abs(A - A64)
    assert np.all(err <= _bound(inst)), f"max ratio {np.max(err / _bound(inst))}"
    rel = np.linalg.norm(A - A64) / np.linalg.norm(A64)
    assert rel < 1e-6, rel
    assert np.all(np.imag(np.diag(A)) == 0.0)
    np.testing.assert_array_equal(A, A.conj().T)
    # dbar, c and the constants stay FP64 in every precision
    assert np.max(np.abs(dbar - dbar64)) <= 1e-13 * np.max(np.abs(dbar64))
    assert abs(c - c64) <= 1e-13 * abs(c64) and abs(K0 - K064) <= 1e-13 * abs(K064)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_loglike(orc, prec):
    """logL from a reduced-precision A is NOT held to the FP64 tolerance:
    with foreground variance 1e4 the posterior mean x = Sigma^-1 dbar is
    large and logL moves by about x^H dA x - tr(Sigma^-1 dA). The pin is the
    oracle run on W rounded to complex64 (the first rounding both schemes
    make): the GPU's error may be at most 20 times the error that this
    rounding alone causes (the rest is FP32 accumulation and, for BF16x3,
    the dropped cross products)."""
    inst = synth.gen(0)
    ref, _ = orc.loglike_instance(inst)
    sig = np.sqrt(inst.noise_var)[:, None]
    W32 = (inst.T / sig).astype(np.complex64).astype(np.complex128)
    pre = orc.precompute(W32 * sig, inst.noise_var, inst.d)
    pre = (pre[0],) + tuple(orc.precompute(inst.T, inst.noise_var, inst.d)[1:])  # dbar, c in FP64
    emul, _ = orc.loglike(*pre, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta)
    print(f"gpu: reduced precision logL {prec}", flush=True)
    got, info = run_instance(inst, prec=prec)
    assert np.all(info == 0)
    err = np.abs(got - ref)
    bound = np.maximum(tol(ref), 20.0 * np.abs(emul - ref))
    assert np.all(err <= bound), (err.max(), np.abs(emul - ref).max())


# Ill-conditioned inputs: T with singular values over four decades, with the
# usual foreground share and with a wide-field foreground model (far more
# foreground than EoR coefficients).
STRESS_CASES = {
    "svd4": dict(m=700, n=300, n_k=3),
    "widefg": dict(m=700, n=300, n_k=3, n_eor=40),
}


@pytest.mark.parametrize("case", sorted(STRESS_CASES))
def test_stress_fp64_matches_oracle(orc, case):
    inst = synth.stress(seed=31 + len(case), n_theta=8, **STRESS_CASES[case])
    ref, rinfo = orc.loglike_instance(inst)
    print(f"gpu: stress {case} fp64", flush=True)
    got, info = run_instance(inst)
    np.testing.assert_array_equal(info, rinfo)
    ok = info == 0
    assert ok.any()
    assert np.all(np.abs(got[ok] - ref[ok]) <= tol(ref[ok])), np.max(np.abs(got[ok] - ref[ok]))
    assert np.all(got[~ok] == -np.inf)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", sorted(STRESS_CASES))
def test_stress_reduced_precision_reports_cleanly(orc, case, prec):
    """A reduced-precision A may lose positive definiteness on ill-conditioned
    inputs (the reason the factorisation stays FP64). Whatever happens, each
    theta either factors (finite logL, info 0) or reports its failing pivot
    (info in 1..n, logL = -inf); nothing non-finite escapes otherwise."""
    inst = synth.stress(seed=31 + len(case), n_theta=8, **STRESS_CASES[case])
    ref, _ = orc.loglike_instance(inst)
    print(f"gpu: stress {case} {prec}", flush=True)
    got, info = run_instance(inst, prec=prec)
    assert np.all((info == 0) | ((info >= 1) & (info <= inst.n)))
    assert np.all(np.isfinite(got[info == 0]))
    assert np.all(got[info != 0] == -np.inf)
    ok = info == 0
    if ok.any():
        print(f"  {case} {prec}: {int((~ok).sum())} of {info.size} failed; max |dlogL| "
              f"{np.max(np.abs(got[ok] - ref[ok])):.3g}", flush=True)
