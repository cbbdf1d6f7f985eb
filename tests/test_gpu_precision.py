"""Reduced-precision A = W^H W (W = T / sigma): FP32 and split-BF16 (three
or two terms) on MFMA with FP32 accumulation per 64-row chunk and FP64
across chunks.

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


# Rounding of one real product x y, in units of u = 2^-24, before the FP32
# accumulation: W to FP32 (or to three bfloat16 terms with the dropped
# cross products) stays below 8u. With two bfloat16 terms, x = h + l + d with
# |d| <= 2^-16 |x|, and the dropped l l' is at most 2^-16 (1 + 2^-8)^2 |x y|:
# about 3 2^-16 = 768u in all, 800u with the FP32 rounding of W.
SPLIT_U = {"fp32": 8, "bf16x3": 8, "bf16x2": 800}


def _bound(inst, prec):
    """Componentwise bound on |A_red - A|: (the product rounding of
    SPLIT_U) + (FP32 accumulation over a 64-row chunk: gamma_64 <= 65u),
    times the two real products that make each real or imaginary part:
    2 (SPLIT_U + 65) u sum_s |W_sj| |W_sk|."""
    W = np.abs(inst.T) / np.sqrt(inst.noise_var)[:, None]
    return 2.0 * (SPLIT_U[prec] + CHUNK + 1) * U32 * (W.T @ W)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x2"])
@pytest.mark.parametrize("shape", [(480, 200), (700, 300), (1030, 129)])
def test_reduced_precision_A_within_bound(orc, prec, shape):
    m, n = shape
    inst = synth.small(seed=m + 3 * n, m=m, n=n, n_k=3, n_theta=4)
    A64, dbar64, c64, K064 = orc.precompute(inst.T, inst.noise_var, inst.d)
    print(f"gpu: reduced precision {prec} m={m} n={n}", flush=True)
    A, dbar, c, K0 = _export(inst, prec)
    err = np.abs(A - A64)
    bound = _bound(inst, prec)
    assert np.all(err <= bound), f"max ratio {np.max(err / bound)}"
    rel = np.linalg.norm(A - A64) / np.linalg.norm(A64)
    assert rel < (1e-4 if prec == "bf16x2" else 1e-6), rel
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


def _bf16_nearest(x32):
    """The bfloat16 value nearest each float32 (ties to even), as float32."""
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _split2(x32):
    """x32 (float32) split into two bfloat16 terms h + l: (h + l, l) in FP64."""
    h = _bf16_nearest(x32)
    low = _bf16_nearest((x32 - h).astype(np.float32))
    return h.astype(np.float64) + low.astype(np.float64), low.astype(np.float64)


def test_bf16x2_loglike(orc):
    """The two-term split moves logL far more than the other schemes: every
    real product drops l l', which on the diagonal of A (l_r^2 + l_i^2) is
    never negative, so the error is systematic. The pin is the oracle run on
    what the scheme defines: with W split as H + L (each real and imaginary
    part its two bfloat16 terms), the kept products hh' + hl' + lh' form
    (H + L)^H (H + L) - L^H L, computed here in FP64. The GPU differs from
    it only by its FP32 accumulation, and may be at most 20 times the
    largest logL error of that run over the batch."""
    inst = synth.gen(0)
    ref, _ = orc.loglike_instance(inst)
    sig = np.sqrt(inst.noise_var)[:, None]
    W32 = (inst.T / sig).astype(np.complex64)
    sr, lr = _split2(np.ascontiguousarray(W32.real))
    si, li = _split2(np.ascontiguousarray(W32.imag))
    A2 = (orc.precompute((sr + 1j * si) * sig, inst.noise_var, inst.d)[0]
          - orc.precompute((lr + 1j * li) * sig, inst.noise_var, inst.d)[0])
    rest = orc.precompute(inst.T, inst.noise_var, inst.d)[1:]
    emul, _ = orc.loglike(A2, *rest, inst.n_k, inst.bin_of, inst.fixed_var, None, inst.theta)
    print("gpu: reduced precision logL bf16x2", flush=True)
    got, info = run_instance(inst, prec="bf16x2")
    assert np.all(info == 0)
    err = np.abs(got - ref)
    scale = np.max(np.abs(emul - ref))
    assert scale > 0.0
    assert np.all(err <= np.maximum(tol(ref), 20.0 * scale)), (err.max(), scale)
    # and the GPU is close to that run itself: FP32 accumulation is the rest
    assert np.max(np.abs(got - emul)) <= 0.5 * scale, (np.max(np.abs(got - emul)), scale)


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


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x2"])
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


@pytest.mark.parametrize("case", sorted(synth.STRESS))
def test_stress_full_size_sampled(case):
    """The ill-conditioned instances at full size (8000 x 2048, 8 bins,
    B = 256 in one call, singular values of T over four decades; wide-field:
    256 EoR against 1792 foreground coefficients), FP64: 8 theta of the batch
    against oracle values stored by tests/golden/make_golden.py, failure codes
    included, and every other theta finite or reported."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "stress_oracle_sample.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))["cases"][case]
    inst = synth.gen_stress(case)
    assert inst.digest() == g["digest"], "synthetic inputs differ from the ones the oracle saw"
    print(f"gpu: stress {case} full size m={inst.m} n={inst.n} B={inst.theta.shape[0]}", flush=True)
    got, info = run_instance(inst)
    idx = np.array(g["index"])
    ref, rinfo = np.array(g["logL"]), np.array(g["info"])
    np.testing.assert_array_equal(info[idx], rinfo)
    ok = rinfo == 0
    assert ok.any()
    assert np.all(np.abs(got[idx][ok] - ref[ok]) <= tol(ref[ok])), np.max(np.abs(got[idx][ok] - ref[ok]))
    assert np.all(got[idx][~ok] == -np.inf)
    assert np.all(np.isfinite(got[info == 0])) and np.all(got[info != 0] == -np.inf)
