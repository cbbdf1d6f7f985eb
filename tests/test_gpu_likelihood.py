"""GPU parity of the batched FP64 likelihood against the CPU oracle.

Bar: |dlogL| <= 1e-6 |logL| + 1e-6 for every theta (the required tolerance);
the kernels are also held to a tighter internal 1e-10 relative bound, which
FP64 with a different summation order meets with a wide margin.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests import _pins
from tests.gpu_util import have_gpu, run_instance, tol

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)


def _check(got, ref, rel=1e-10):
    err = np.abs(got - ref)
    assert np.all(err <= tol(ref)), f"max |dlogL| {err.max()}"
    assert np.all(err <= rel * np.maximum(np.abs(ref), 1.0)), f"max rel {np.max(err / np.abs(ref))}"


def test_tiny_workload_all_theta(orc):
    """480 x 200, 3 bins, 40 foreground coefficients, 64 theta (every theta)."""
    inst = synth.gen(0)
    ref, rinfo = orc.loglike_instance(inst)
    _say("gpu: tiny workload n=200 B=64")
    got, info = run_instance(inst)
    assert np.all(info == 0) and np.all(rinfo == 0)
    _check(got, ref)


def test_precompute_products(orc):
    import torch
    import paper_2501_12928_amd as eor
    inst = synth.gen(0)
    A, dbar, c, K0 = orc.precompute(inst.T, inst.noise_var, inst.d)
    _say("gpu: precompute export n=200")
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    gA, gd, gc, gK0 = ctx.export_precompute()
    gA = gA.cpu().numpy()
    gd = gd.cpu().numpy()
    ctx.close()
    assert np.max(np.abs(gA - A)) <= 1e-13 * np.max(np.abs(A))
    assert np.all(np.imag(np.diag(gA)) == 0.0)
    np.testing.assert_array_equal(gA, gA.conj().T)
    assert np.max(np.abs(gd - dbar)) <= 1e-13 * np.max(np.abs(dbar))
    assert abs(gc - c) <= 1e-13 * abs(c)
    assert abs(gK0 - K0) <= 1e-13 * abs(K0)


@pytest.mark.parametrize("ts", [64, 32])
@pytest.mark.parametrize("m,n,n_k,n_eor", [
    (5, 1, 1, 1),        # one coefficient
    (80, 63, 2, 50),     # just under one tile
    (80, 64, 2, 64),     # exactly one tile, no foreground
    (90, 65, 3, 60),     # one past a tile boundary
    (300, 130, 4, 100),  # three tiles, ragged
    (520, 257, 5, 220),  # five tiles, ragged by one
    (600, 384, 1, 384),  # six tiles, one bin
    (700, 300, 7, 0),    # every coefficient fixed (no bins used)
])
def test_ragged_shapes(orc, m, n, n_k, n_eor, ts):
    inst = synth.small(seed=m + n, m=m, n=n, n_k=n_k, n_eor=n_eor, n_theta=9)
    ref, rinfo = orc.loglike_instance(inst)
    _say(f"gpu: ragged m={m} n={n} n_k={n_k} n_eor={n_eor} tile {ts}")
    got, info = run_instance(inst, ts=ts)
    np.testing.assert_array_equal(info, rinfo)
    _check(got, ref)


def test_shell_bins_and_scales(orc):
    """Bins of unequal size (shell growth) and per-bin scales s_b."""
    inst = synth.small(seed=44, m=400, n=200, n_k=6, n_eor=170, n_theta=10, shells=True)
    inst.bin_scale = np.array([0.5, 2.0, 1.0, 3.0, 0.1, 7.0])
    ref, _ = orc.loglike_instance(inst)
    _say("gpu: shell bins with scales n=200")
    got, info = run_instance(inst)
    assert np.all(info == 0)
    _check(got, ref)


def test_terms_match_oracle(orc):
    inst = synth.small(seed=8, m=200, n=140, n_k=3, n_theta=6)
    ref, _, rterms = orc.loglike_instance(inst, terms=True)
    A, dbar, c, K0 = orc.precompute(inst.T, inst.noise_var, inst.d)
    _say("gpu: terms n=140")
    got, info, terms = run_instance(inst, terms=True)
    np.testing.assert_allclose(terms[:, 0], rterms[:, 0], rtol=1e-11)   # ln det Sigma
    np.testing.assert_allclose(terms[:, 1], rterms[:, 3], rtol=1e-11)   # ||L^-1 dbar||^2
    np.testing.assert_allclose(terms[:, 2], rterms[:, 2], rtol=1e-12)   # ln det Phi
    np.testing.assert_allclose(terms[:, 3], c, rtol=1e-13)


# Launch choices (prefetch stages, workgroups per CU, tiles per pass).
TUNINGS = [(4, 2, 1), (2, 2, 1), (4, 1, 1), (4, 1, 2), (2, 1, 2)]


@pytest.mark.parametrize("ts", [64, 32])
@pytest.mark.parametrize("m,n,n_k", [
    (300, 130, 4),   # 3 tiles of 64: 3, 2, 1 units per column (6 tiles of 32)
    (520, 257, 5),   # 5 tiles, ragged by one
    (900, 700, 6),   # 11 tiles (22 of 32)
])
def test_launch_choices_agree(orc, m, n, n_k, ts):
    """Every launch choice meets the bar, and all give the same bits: the
    tile updates sum in the same order whichever group computes them (with
    32-wide tiles, two or four groups per workgroup)."""
    inst = synth.small(seed=m + 3 * n, m=m, n=n, n_k=n_k, n_theta=12)
    ref, rinfo = orc.loglike_instance(inst)
    outs = []
    for t in TUNINGS:
        _say(f"gpu: n={n} tuning {t} tile {ts}")
        got, info = run_instance(inst, tuning=t, ts=ts)
        assert np.all(info == 0) and np.all(rinfo == 0)
        _check(got, ref)
        outs.append(got)
    for t, o in zip(TUNINGS[1:], outs[1:]):
        assert np.array_equal(o, outs[0]), t


def test_tuning_arguments():
    import paper_2501_12928_amd as eor
    ctx = eor.Context(0)
    assert ctx.tuning() == (4, 1, 2)
    assert ctx.tile_size() == 64
    for bad in (0, 16, 48, 128):
        with pytest.raises(eor.EorError):
            ctx.set_tile_size(bad)
    ctx.set_tile_size(32)
    assert ctx.tile_size() == 32
    for bad in [(3, 1, 1), (4, 3, 1), (4, 2, 2), (4, 1, 3), (0, 0, 0)]:
        with pytest.raises(eor.EorError):
            ctx.set_tuning(*bad)
    assert ctx.tuning() == (4, 1, 2)
    ctx.set_tuning(2, 1, 2)
    assert ctx.tuning() == (2, 1, 2)
    ctx.close()


@pytest.mark.parametrize("tuning,ts", [(None, 64), ((4, 2, 1), 64), (None, 32), ((2, 2, 1), 32)])
def test_failures_reported_per_theta(orc, tuning, ts):
    """Non-finite theta -> info -1; a NaN column of T -> pivot failure at
    that column (1-based), exactly as the oracle reports it; the rest of
    the batch is unaffected."""
    inst = synth.small(seed=12, m=150, n=100, n_k=3, n_theta=5)
    th = inst.theta.copy()
    th[1, 2] = np.nan
    th[3, 0] = np.inf
    th[4, 1] = 400.0     # 10^400 overflows: prior variance not finite
    ref, rinfo = orc.loglike_instance(inst, theta=th)
    _say(f"gpu: failure codes, tuning {tuning} tile {ts}")
    got, info = run_instance(inst, theta=th, tuning=tuning, ts=ts)
    np.testing.assert_array_equal(info, rinfo)
    np.testing.assert_array_equal(info, [0, -1, 0, -1, -1])
    assert np.all(got[info != 0] == -np.inf)
    _check(got[info == 0], ref[info == 0])

    bad = synth.small(seed=13, m=150, n=100, n_k=3, n_theta=3)
    bad.T = bad.T.copy()
    bad.T[:, 70] = np.nan
    ref, rinfo = orc.loglike_instance(bad)
    got, info = run_instance(bad, tuning=tuning, ts=ts)
    np.testing.assert_array_equal(rinfo, [71, 71, 71])
    np.testing.assert_array_equal(info, rinfo)
    assert np.all(got == -np.inf)


def test_deterministic_and_position_independent():
    inst = synth.small(seed=31, m=400, n=250, n_k=4, n_theta=40)
    _say("gpu: determinism n=250 B=40")
    a, _ = run_instance(inst)
    b, _ = run_instance(inst)
    assert np.array_equal(a, b)
    p = np.random.default_rng(1).permutation(40)
    c, _ = run_instance(inst, theta=inst.theta[p])
    assert np.array_equal(c, a[p])
    d, _ = run_instance(inst, theta=inst.theta[7:8])
    assert d[0] == a[7]


def test_diagonal_instrument_closed_form():
    """T = [I_n; 0] at n = 1000 (16 tiles): closed form, no oracle needed."""
    rng = np.random.default_rng(77)
    m, n = 1100, 1000
    T = np.zeros((m, n), dtype=np.complex128)
    T[np.arange(n), np.arange(n)] = 1.0
    inst = synth.make_instance(rng, m=m, n=n, n_k=6, n_eor=900, n_theta=8, lo=-1, hi=3, T=T)
    ref = np.array([_pins.diagonal_closed_form(inst.noise_var, inst.d, th, inst.bin_of,
                                               inst.fixed_var, n) for th in inst.theta])
    _say("gpu: diagonal closed form n=1000")
    got, info = run_instance(inst)
    assert np.all(info == 0)
    _check(got, ref, rel=1e-12)


def test_one_bin_eigen_closed_form():
    """One bin, dense T at n = 512: exact curve from eigh(A)."""
    rng = np.random.default_rng(78)
    m, n = 700, 512
    inst = synth.make_instance(rng, m=m, n=n, n_k=1, n_eor=n, n_theta=1, lo=-1, hi=3)
    grid = np.linspace(-2.0, 4.0, 13)[:, None]
    ref = _pins.eigen_closed_form(inst.T, inst.noise_var, inst.d, grid[:, 0])
    _say("gpu: one-bin eigen closed form n=512")
    got, info = run_instance(inst, theta=grid)
    assert np.all(info == 0)
    _check(got, ref)


def _sampled(config_id, tuning=None):
    path = os.path.join(GOLDEN, f"c{config_id}_oracle_sample.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))
    inst = synth.gen(config_id)
    assert inst.digest() == g["digest"], "synthetic inputs differ from the ones the oracle saw"
    _say(f"gpu: full workload {config_id}: m={inst.m} n={inst.n} B={inst.theta.shape[0]} tuning {tuning}")
    got, info = run_instance(inst, tuning=tuning)
    idx = np.array(g["index"])
    assert np.all(info == 0)
    _check(got[idx], np.array(g["logL"]))
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("tuning", [None, (4, 2, 1)])
def test_plain_batched_workload_sampled(tuning):
    """8000 x 2048, 8 bins, B = 256 in one call; 16 theta checked against
    oracle values stored by tests/golden/make_golden.py."""
    _sampled(1, tuning)


@pytest.mark.slow
def test_metric_workload():
    """20000 x 4096, 12 bins, B = 512 in one call (the benchmark's launch).
    Every one of the 512 logL is the same bits under the default launch
    (two tiles per pass in eight-wave workgroups, where each group reads
    tiles of L the other group wrote), under two four-wave workgroups per CU
    and as a one-instance group launch. Against stored oracle values: 16 theta
    of the batch and 24 theta outside it (the corners and edges of the prior
    box, points beyond it, the data's theta and seeded draws), element by
    element."""
    import torch
    import paper_2501_12928_amd as eor
    path = os.path.join(GOLDEN, "c3_oracle_sample.json")
    g = json.load(open(path))
    inst = synth.gen(3)
    assert inst.digest() == g["digest"], "synthetic inputs differ from the ones the oracle saw"
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    th = torch.from_numpy(inst.theta).cuda()
    runs = {}
    for t in [(4, 1, 2), (4, 2, 1)]:
        _say(f"gpu: metric workload 20000 x 4096 B=512, tuning {t}")
        ctx.set_tuning(*t)
        L, info = ctx.loglike_batch(th)
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        runs[t] = L.cpu().numpy()
    _say("gpu: metric workload as a one-instance group")
    grp = eor.Group([ctx])
    outs, infos = grp.loglike([th])
    torch.cuda.synchronize()
    assert np.all(infos[0].cpu().numpy() == 0)
    runs["group"] = outs[0].cpu().numpy()
    grp.close()
    base = runs[(4, 1, 2)]
    assert np.all(np.isfinite(base))
    for k, v in runs.items():
        assert np.array_equal(v, base), (k, np.max(np.abs(v - base)))
    idx = np.array(g["index"])
    assert len(idx) >= 16
    _check(base[idx], np.array(g["logL"]))
    xt = np.array(g["extra_theta"])
    assert xt.shape == (24, inst.n_k)
    _say("gpu: metric workload, 24 theta outside the batch")
    ctx.set_tuning(4, 1, 2)
    L, info = ctx.loglike_batch(torch.from_numpy(xt).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(info.cpu().numpy(), np.array(g["extra_info"]))
    _check(L.cpu().numpy(), np.array(g["extra_logL"]))
    # 32-wide tiles: the same batch, the same 40 oracle values
    _say("gpu: metric workload with 32-wide tiles")
    ctx.set_tile_size(32)
    L32, info = ctx.loglike_batch(th)
    Lx, infox = ctx.loglike_batch(torch.from_numpy(xt).cuda())
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and np.all(infox.cpu().numpy() == 0)
    L32 = L32.cpu().numpy()
    _check(L32[idx], np.array(g["logL"]))
    _check(Lx.cpu().numpy(), np.array(g["extra_logL"]))
    assert np.max(np.abs(L32 - base) / np.abs(base)) < 1e-11
    ctx.close()


def test_precompute_rejects_bad_leading_dimension():
    """ldT < n, and the other argument errors of eor_precompute, come back as
    EOR_ERR_ARG before any device work; the context stays usable."""
    import torch
    import paper_2501_12928_amd as eor
    inst = synth.small(seed=5, m=90, n=70, n_k=2, n_theta=3)
    T = torch.from_numpy(inst.T).cuda()
    nv = torch.from_numpy(inst.noise_var).cuda()
    d = torch.from_numpy(inst.d).cuda()
    bins = np.ascontiguousarray(inst.bin_of, dtype=np.int32)
    fv = np.ascontiguousarray(inst.fixed_var)
    ctx = eor.Context(0)
    L = eor.lib()
    args = lambda m, n, ld, nk=inst.n_k: (ctx.handle, m, n, T.data_ptr(), ld, nv.data_ptr(), d.data_ptr(), nk,
                                          bins.ctypes.data, fv.ctypes.data, None, 0, None)
    _say("gpu: precompute argument errors")
    assert L.eor_precompute(*args(90, 70, 69)) == eor.EOR_ERR_ARG
    assert b"ldT" in L.eor_last_error()
    assert L.eor_precompute(*args(90, 70, 0)) == eor.EOR_ERR_ARG
    assert L.eor_precompute(*args(0, 70, 70)) == eor.EOR_ERR_ARG
    assert L.eor_precompute(*args(90, 70, 70, nk=1)) == eor.EOR_ERR_ARG   # bin 1 out of range
    assert L.eor_loglike_batch(ctx.handle, 3, None, None, None, None) == eor.EOR_ERR_STATE
    assert L.eor_precompute(*args(90, 70, 70)) == eor.EOR_OK
    got, info = ctx.loglike_batch(torch.from_numpy(inst.theta).cuda())
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    ctx.close()


def test_workspace_limit(orc):
    """A workspace budget caps the theta in flight without changing a bit;
    a budget below one theta's slot returns EOR_ERR_OOM before any launch
    (the outputs stay as they were)."""
    import torch
    import paper_2501_12928_amd as eor
    inst = synth.small(seed=17, m=500, n=300, n_k=4, n_theta=40)
    ref, _ = orc.loglike_instance(inst)
    n_pad = 320
    # one slot: N (N + 1) / 2 packed tiles of 64 x 64 complex128, plus the solve vector
    N = n_pad // 64
    slot = N * (N + 1) // 2 * 64 * 64 * 16 + 16 * n_pad
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    th = torch.from_numpy(inst.theta).cuda()
    _say("gpu: workspace limit, no limit")
    a, _ = ctx.loglike_batch(th)
    torch.cuda.synchronize()
    a = a.cpu().numpy()
    for k in (3, 1):
        _say(f"gpu: workspace limit of {k} slots")
        ctx.set_workspace_limit(k * slot)
        b, info = ctx.loglike_batch(th)
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        assert np.array_equal(b.cpu().numpy(), a)
    assert np.all(np.abs(a - ref) <= tol(ref))
    ctx.set_workspace_limit(slot - 1)
    out = torch.full((40,), 7.0, dtype=torch.float64, device="cuda")
    inf = torch.full((40,), 9, dtype=torch.int32, device="cuda")
    L = eor.lib()
    st = L.eor_loglike_batch(ctx.handle, 40, th.data_ptr(), out.data_ptr(), inf.data_ptr(), None)
    assert st == eor.EOR_ERR_OOM, st
    assert b"workspace" in L.eor_last_error()
    torch.cuda.synchronize()
    assert torch.all(out == 7.0) and torch.all(inf == 9)
    ctx.set_workspace_limit(0)
    c, _ = ctx.loglike_batch(th)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), a)
    ctx.close()


def test_calls_on_two_streams(orc):
    """Back-to-back calls on one context from two streams share the task
    counter and the workspace: the second waits for the first, and both
    give the bits of calls made one after the other on one stream. The same
    for a group call on a third stream right after a context call."""
    import torch
    import paper_2501_12928_amd as eor
    inst = synth.small(seed=23, m=700, n=520, n_k=5, n_theta=300)
    ctx = eor.Context(0)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
    th1 = torch.from_numpy(inst.theta[:300]).cuda()
    th2 = torch.from_numpy(inst.theta[::-1].copy()).cuda()
    _say("gpu: one stream")
    r1, _ = ctx.loglike_batch(th1)
    r2, _ = ctx.loglike_batch(th2)
    torch.cuda.synchronize()
    r1, r2 = r1.cpu().numpy(), r2.cpu().numpy()
    assert np.array_equal(r2, r1[::-1])
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    grp = eor.Group([ctx])
    for rep in range(3):
        _say(f"gpu: two streams, repeat {rep}")
        torch.cuda.synchronize()
        a, _ = ctx.loglike_batch(th1, stream=s1)
        b, _ = ctx.loglike_batch(th2, stream=s2)
        outs, _ = grp.loglike([th1], stream=s3)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), r1)
        assert np.array_equal(b.cpu().numpy(), r2)
        assert np.array_equal(outs[0].cpu().numpy(), r1)
    grp.close()
    ctx.close()


def test_largest_shape_block_rotation():
    """n = 8192 (128 tiles per side), beyond any shape the oracle finishes
    quickly, through a property that holds at any size: two independent
    4096-coefficient problems with the same bins, stacked block-diagonally and
    then mixed pair by pair (coefficient j of each with a random 2 x 2
    unitary; both have the same prior variance, so the likelihood is
    unchanged while A becomes dense), must give the sum of the two logL. The
    4096-coefficient path is itself held to the oracle elsewhere."""
    rng = np.random.default_rng(8192)
    n1, m1, n_k, n_eor = 4096, 4400, 6, 3584
    p1 = synth.make_instance(rng, m=m1, n=n1, n_k=n_k, n_eor=n_eor, n_theta=4, lo=-1.0, hi=3.0)
    p2 = synth.make_instance(rng, m=m1, n=n1, n_k=n_k, n_eor=n_eor, n_theta=4, lo=-1.0, hi=3.0)
    assert np.array_equal(p1.bin_of, p2.bin_of)
    n, m = 2 * n1, 2 * m1
    T = np.zeros((m, n), dtype=np.complex128)
    # pair rotation: columns j and j + n1 of blockdiag(T1, T2) mixed by U_j
    a = rng.standard_normal(n1) + 1j * rng.standard_normal(n1)
    b = rng.standard_normal(n1) + 1j * rng.standard_normal(n1)
    nrm = np.sqrt(np.abs(a) ** 2 + np.abs(b) ** 2)
    a, b = a / nrm, b / nrm
    # U_j = [[a, -conj(b)], [b, conj(a)]] (unitary); T' = blockdiag(T1, T2) U
    T[:m1, :n1] = p1.T * a[None, :]
    T[m1:, :n1] = p2.T * b[None, :]
    T[:m1, n1:] = p1.T * (-np.conj(b))[None, :]
    T[m1:, n1:] = p2.T * np.conj(a)[None, :]
    big = synth.Instance(T=T, noise_var=np.concatenate([p1.noise_var, p2.noise_var]),
                         d=np.concatenate([p1.d, p2.d]), n_k=n_k,
                         bin_of=np.concatenate([p1.bin_of, p2.bin_of]),
                         fixed_var=np.concatenate([p1.fixed_var, p2.fixed_var]),
                         bin_scale=p1.bin_scale, theta=p1.theta, theta_true=p1.theta_true,
                         lo=p1.lo, hi=p1.hi)
    _say("gpu: n=4096 halves")
    l1, i1 = run_instance(p1)
    l2, i2 = run_instance(p2, theta=p1.theta)
    _say("gpu: n=8192 mixed, 4 theta (about 2.5 s each on one CU)")
    lb, ib = run_instance(big)
    assert np.all(i1 == 0) and np.all(i2 == 0) and np.all(ib == 0)
    ref = l1 + l2
    assert np.all(np.abs(lb - ref) <= tol(ref)), np.max(np.abs(lb - ref))


def test_n16384_four_block_rotation():
    """n = 16384 (256 tiles per side; each theta's factor is 4.3 GB, so its
    byte offsets pass 2^32), by the same property with four blocks: four
    independent 4096-coefficient problems with the same bins, stacked
    block-diagonally and mixed four columns at a time (coefficient j of each
    block by a random 4 x 4 unitary; all four have the same prior variance),
    must give the sum of the four logL, at a random theta and at the two
    corners of the prior box. Each 4096-coefficient problem is of the size
    held to the oracle elsewhere."""
    rng = np.random.default_rng(16384)
    n1, m1, n_k, n_eor, nb = 4096, 4400, 6, 3584, 4
    parts = [synth.make_instance(rng, m=m1, n=n1, n_k=n_k, n_eor=n_eor, n_theta=1, lo=-1.0, hi=3.0)
             for _ in range(nb)]
    for p in parts[1:]:
        assert np.array_equal(p.bin_of, parts[0].bin_of)
        assert np.array_equal(p.fixed_var, parts[0].fixed_var)
        assert np.array_equal(p.bin_scale, parts[0].bin_scale)
    theta = np.ascontiguousarray(np.stack([parts[0].theta[0], np.full(n_k, -1.0), np.full(n_k, 3.0)]))
    # U[j] (4 x 4 unitary per coefficient): Q of a complex Gaussian matrix
    g = rng.standard_normal((n1, nb, nb)) + 1j * rng.standard_normal((n1, nb, nb))
    U = np.linalg.qr(g)[0]
    assert np.allclose(np.einsum("jrc,jrd->jcd", U.conj(), U), np.eye(nb)[None], atol=1e-12)
    n, m = nb * n1, nb * m1
    # T' = blockdiag(T_0 .. T_3) U: block (r, c) is T_r scaled column-wise by U[:, r, c]
    T = np.empty((m, n), dtype=np.complex128)
    for r, p in enumerate(parts):
        for c in range(nb):
            T[r * m1:(r + 1) * m1, c * n1:(c + 1) * n1] = p.T * U[None, :, r, c]
    big = synth.Instance(T=T, noise_var=np.concatenate([p.noise_var for p in parts]),
                         d=np.concatenate([p.d for p in parts]), n_k=n_k,
                         bin_of=np.concatenate([p.bin_of for p in parts]),
                         fixed_var=np.concatenate([p.fixed_var for p in parts]),
                         bin_scale=parts[0].bin_scale, theta=theta, theta_true=parts[0].theta_true,
                         lo=parts[0].lo, hi=parts[0].hi)
    del T
    _say("gpu: four n=4096 blocks, 3 theta")
    ref = np.zeros(len(theta))
    for p in parts:
        lp, ip = run_instance(p, theta=theta)
        assert np.all(ip == 0)
        ref += lp
    _say("gpu: n=16384 mixed, 3 theta (one theta per CU)")
    lb, ib = run_instance(big)
    assert np.all(ib == 0)
    err = np.abs(lb - ref)
    _say(f"n=16384: max |dlogL| {err.max():.3e}, relative {np.max(err / np.abs(ref)):.3e}")
    assert np.all(err <= tol(ref)), err.max()


def test_fp64_mfma_probe():
    """The measured FP64 matrix peak is positive and below the part's
    specification (78.6 TFLOP/s at 2.4 GHz); bad arguments are refused."""
    import paper_2501_12928_amd as eor
    tf, ms = eor.probe_fp64_mfma(20000)
    assert 10.0 < tf <= 80.0 and ms > 0.0, (tf, ms)
    with pytest.raises(eor.EorError):
        eor.probe_fp64_mfma(0)


def test_empty_batches(orc):
    """Zero theta is a valid call everywhere: the batched path, a group with
    an empty instance beside a full one (and a group call with every
    instance empty), the surrogate's gate and the out-of-core path."""
    import torch
    import paper_2501_12928_amd as eor
    a = synth.small(seed=81, m=300, n=130, n_k=3, n_theta=5)
    b = synth.small(seed=82, m=200, n=70, n_k=2, n_theta=4)
    ctxs = []
    for inst in (a, b):
        c = eor.Context(0)
        c.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                     torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var)
        ctxs.append(c)
    print("gpu: empty batches", flush=True)
    L, info = ctxs[0].loglike_batch(torch.empty((0, a.n_k), dtype=torch.float64, device="cuda"))
    assert L.shape == (0,) and info.shape == (0,)
    lib = eor.lib()
    assert lib.eor_loglike_batch(ctxs[0]._h, 0, None, None, None, None) == eor.EOR_OK
    g = eor.Group(ctxs)
    outs, infos = g.loglike([torch.empty((0, a.n_k), dtype=torch.float64, device="cuda"),
                             torch.from_numpy(b.theta).cuda()])
    torch.cuda.synchronize()
    ref, _ = orc.loglike_instance(b)
    got = outs[1].cpu().numpy()
    assert outs[0].shape == (0,) and np.all(infos[1].cpu().numpy() == 0)
    assert np.all(np.abs(got - ref) <= tol(ref))
    outs, _ = g.loglike([torch.empty((0, a.n_k), dtype=torch.float64, device="cuda"),
                         torch.empty((0, b.n_k), dtype=torch.float64, device="cuda")])
    torch.cuda.synchronize()
    assert outs[0].shape == (0,) and outs[1].shape == (0,)
    g.close()
    s = eor.Surrogate(3, -1.0, 3.0, n_members=2, hidden=16, seed=1)
    rng = np.random.default_rng(3)
    th = rng.uniform(-1.0, 3.0, size=(256, 3))
    s.train(th, -np.sum(th ** 2, axis=1), cfg=eor.train_cfg(epochs=2, minibatch=64))
    m, sp, dec = s.gate(torch.empty((0, 3), dtype=torch.float64, device="cuda"), 0.0, 0.05)
    assert m.shape == (0,) and dec.shape == (0,)
    A, dbar, c, K0 = orc.precompute(a.T, a.noise_var, a.d)
    got, inf = eor.loglike_host(A, dbar, c, K0, a.n_k, a.bin_of, a.fixed_var, None, np.empty((0, a.n_k)), 1 << 26)
    assert got.shape == (0,) and inf.shape == (0,)
    A = np.ascontiguousarray(A, dtype=np.complex128)
    dbar = np.ascontiguousarray(dbar, dtype=np.complex128)
    bins = np.ascontiguousarray(a.bin_of, dtype=np.int32)
    fv = np.ascontiguousarray(a.fixed_var, dtype=np.float64)
    assert lib.eor_loglike_host(0, a.n, A.ctypes.data, a.n, dbar.ctypes.data, c, K0, a.n_k, bins.ctypes.data,
                                fv.ctypes.data, None, 0, None, 1 << 26, 0, None, None) == eor.EOR_OK
    for ctx in ctxs:
        ctx.close()
