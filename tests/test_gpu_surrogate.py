"""Surrogate network kernels against the FP64 oracle (oracle/mlp.py):
forward, hand-derived backward, Adam, ensemble statistics, the gate and the
stable compaction; and training that actually learns."""
import numpy as np
import pytest

from oracle import mlp
from tests.gpu_util import have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]


def _sur(n_in=12, M=3, H=256, seed=0, lo=-1.0, hi=3.0):
    import paper_2501_12928_amd as eor
    return eor.Surrogate(n_in, lo, hi, n_members=M, hidden=H, seed=seed)


def _params(rng, M, n_in, H):
    ps = []
    for _ in range(M):
        p = mlp.he_init(rng, n_in, H)
        P = mlp.n_params(n_in, H)
        # nonzero biases so that every gradient block is exercised
        W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, H)
        b1[:] = rng.standard_normal(H) * 0.1
        b2[:] = rng.standard_normal(H) * 0.1
        b3[:] = 0.3
        assert p.size == P
        ps.append(p)
    return np.stack(ps)


@pytest.mark.parametrize("H,nb", [(256, 1024), (64, 333), (36, 50), (512, 70)])
def test_loss_and_gradient_match_oracle(H, nb):
    """FP32 kernels vs the FP64 oracle on the same parameters and batch:
    relative error of every gradient block within 1e-4 of its norm."""
    rng = np.random.default_rng(H + nb)
    n_in, M = 12, 3
    s = _sur(n_in, M, H)
    p64 = _params(rng, M, n_in, H)
    p32 = p64.astype(np.float32)
    x = rng.uniform(-1, 1, size=(M, nb, n_in)).astype(np.float32)
    y = rng.standard_normal((M, nb)).astype(np.float32)
    s.set_params(p32)
    print(f"gpu: surrogate loss/grad H={H} nb={nb}", flush=True)
    loss, grad = s.loss_grad(x, y)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy()
    for z in range(M):
        l_ref, g_ref = mlp.loss_and_grad(p32[z].astype(np.float64), x[z].astype(np.float64),
                                         y[z].astype(np.float64), n_in, H)
        assert abs(loss[z] - l_ref) <= 1e-5 * abs(l_ref)
        blocks = mlp.unpack(np.arange(g_ref.size), n_in, H)
        for blk in blocks:
            ix = np.asarray(blk).ravel()
            err = np.linalg.norm(grad[z][ix] - g_ref[ix])
            assert err <= 1e-4 * np.linalg.norm(g_ref[ix]) + 1e-7, (z, ix[:2], err)
    s.close()


@pytest.mark.parametrize("n_in,M,H,nb", [(64, 1, 4, 1), (1, 2, 8, 17), (13, 3, 128, 16), (5, 2, 132, 33)])
def test_loss_and_gradient_edge_shapes(n_in, M, H, nb):
    """Edge shapes of the fused kernels: the widest input (64), one input,
    hidden widths of 4 (almost all padding), 128 (exactly one 128-unit
    block) and 132 (just past it), a batch of one sample, batches that end
    on and just past a 16-sample block, and a single member."""
    rng = np.random.default_rng(n_in * 100 + H)
    s = _sur(n_in, M, H)
    p32 = _params(rng, M, n_in, H).astype(np.float32)
    x = rng.uniform(-1, 1, size=(M, nb, n_in)).astype(np.float32)
    y = rng.standard_normal((M, nb)).astype(np.float32)
    s.set_params(p32)
    print(f"gpu: surrogate loss/grad n_in={n_in} M={M} H={H} nb={nb}", flush=True)
    loss, grad = s.loss_grad(x, y)
    loss = loss.cpu().numpy()
    grad = grad.cpu().numpy()
    for z in range(M):
        l_ref, g_ref = mlp.loss_and_grad(p32[z].astype(np.float64), x[z].astype(np.float64),
                                         y[z].astype(np.float64), n_in, H)
        assert abs(loss[z] - l_ref) <= 1e-5 * abs(l_ref) + 1e-7
        for blk in mlp.unpack(np.arange(g_ref.size), n_in, H):
            ix = np.asarray(blk).ravel()
            err = np.linalg.norm(grad[z][ix] - g_ref[ix])
            assert err <= 1e-4 * np.linalg.norm(g_ref[ix]) + 1e-7, (z, ix[:2], err)
    s.close()


def test_adam_step_matches_oracle():
    import paper_2501_12928_amd as eor
    rng = np.random.default_rng(4)
    n_in, M, H, nb = 12, 2, 64, 256
    s = _sur(n_in, M, H)
    p32 = _params(rng, M, n_in, H).astype(np.float32)
    x = rng.uniform(-1, 1, size=(M, nb, n_in)).astype(np.float32)
    y = rng.standard_normal((M, nb)).astype(np.float32)
    s.set_params(p32)
    cfg = eor.train_cfg(lr=1e-2)
    _, g1 = s.loss_grad(x, y)
    s.adam_step(cfg)
    _, g2 = s.loss_grad(x, y)
    s.adam_step(cfg)
    got = s.get_params().cpu().numpy()
    for z in range(M):
        p = p32[z].astype(np.float64)
        m = np.zeros_like(p)
        v = np.zeros_like(p)
        p, m, v = mlp.adam_step(p, g1.cpu().numpy()[z].astype(np.float64), m, v, 1, lr=1e-2)
        p, m, v = mlp.adam_step(p, g2.cpu().numpy()[z].astype(np.float64), m, v, 2, lr=1e-2)
        np.testing.assert_allclose(got[z], p, rtol=1e-5, atol=1e-6)
    s.close()


@pytest.mark.parametrize("n_in,H,B", [(12, 256, 70001), (64, 132, 70001), (12, 256, (1 << 20) + 4097)])
def test_inference_matches_oracle_ensemble(n_in, H, B):
    """Member outputs against the oracle on sampled points, and the ensemble
    statistics against the members' outputs on every point; the last case
    spans two launches of 2^20 points."""
    import torch
    rng = np.random.default_rng(5 + H)
    M = 5
    s = _sur(n_in, M, H)
    p32 = _params(rng, M, n_in, H).astype(np.float32)
    s.set_params(p32)
    s.standardisation(np.array([-1.5e4, 250.0]))
    th = rng.uniform(-1, 3, size=(B, n_in))
    print(f"gpu: surrogate inference {B} points n_in={n_in} H={H}", flush=True)
    mean, spread, mem = s.infer(torch.from_numpy(th).cuda(), members=True)
    mean = mean.cpu().numpy()
    spread = spread.cpu().numpy()
    mem = mem.cpu().numpy()
    idx = np.unique(np.concatenate([rng.choice(B, 2000, replace=False), np.arange(B - 64, B)]))
    rm, rs = mlp.ensemble([p.astype(np.float64) for p in p32], th[idx], -1.0, 3.0, -1.5e4, 250.0, n_in, H)
    # FP32 network outputs: |error| of a member output ~ 1e-6 relative to its scale
    assert np.max(np.abs(mean[idx] - rm)) <= 250.0 * 1e-4
    assert np.max(np.abs(spread[idx] - rs)) <= 250.0 * 1e-4
    # mean and spread are exactly the FP64 statistics of the members' FP32 outputs
    pred = -1.5e4 + 250.0 * mem.astype(np.float64)
    np.testing.assert_allclose(mean, pred.mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(spread, pred.std(axis=0, ddof=0), rtol=1e-9, atol=1e-9)
    s.close()


def test_gate_decisions_and_compaction():
    import torch
    import paper_2501_12928_amd as eor
    rng = np.random.default_rng(6)
    n_in, M, H = 4, 5, 32
    s = _sur(n_in, M, H, lo=0.0, hi=1.0)
    p = _params(rng, M, n_in, H).astype(np.float32)
    p[:, -1] = 0.0
    s.set_params(p)
    s.standardisation(np.array([0.0, 0.05]))
    th = torch.from_numpy(rng.uniform(0, 1, size=(10000, n_in))).cuda()
    mean, spread = s.infer(th)
    L_min = float(np.median(mean.cpu().numpy()))
    tau = float(np.median(spread.cpu().numpy()))
    m2, s2, dec = s.gate(th, L_min, tau)
    ref = mlp.gate(m2.cpu().numpy(), s2.cpu().numpy(), L_min, tau)
    np.testing.assert_array_equal(dec.cpu().numpy(), ref)
    assert 0 < int((dec == 0).sum()) < 10000
    rows, idx, c = eor.compact_rows(dec, th)
    keep = np.flatnonzero(ref)
    assert c == keep.size
    np.testing.assert_array_equal(idx.cpu().numpy(), keep)
    np.testing.assert_array_equal(rows.cpu().numpy(), th.cpu().numpy()[keep])
    # edge cases: nothing kept, everything kept
    _, idx0, c0 = eor.compact_rows(torch.zeros(777, dtype=torch.int32, device="cuda"))
    _, idx1, c1 = eor.compact_rows(torch.ones(777, dtype=torch.int32, device="cuda"))
    assert c0 == 0 and c1 == 777 and np.array_equal(idx1.cpu().numpy(), np.arange(777))
    s.close()


def _smooth_target(th):
    # a logL-like surface: a broad quadratic bowl plus a gentle nonlinearity
    c = np.linspace(0.3, 1.7, th.shape[1])
    return -50.0 * np.sum((th - c) ** 2 / (1.0 + 0.3 * np.abs(th)), axis=1) + 10.0 * np.sin(th[:, 0])


def test_training_learns_and_is_deterministic():
    import torch
    import paper_2501_12928_amd as eor
    rng = np.random.default_rng(7)
    n_in = 12
    th = rng.uniform(-1, 3, size=(20000, n_in))
    y = _smooth_target(th)
    cfg = eor.train_cfg(epochs=60, minibatch=512, patience=10, lr=1e-3, seed=11)
    print("gpu: surrogate training 20000 samples", flush=True)
    s = _sur(n_in, 5, 256, seed=3)
    ep, val = s.train(torch.from_numpy(th).cuda(), torch.from_numpy(y).cuda(), cfg)
    assert 1 <= ep <= 60 and np.all(val < 0.01)     # validation MSE in standardised units
    test = rng.uniform(-1, 3, size=(4000, n_in))
    mean, spread = s.infer(torch.from_numpy(test).cuda())
    err = np.abs(mean.cpu().numpy() - _smooth_target(test))
    assert np.median(err) < 0.05 * np.std(y)
    p1 = s.get_params().cpu().numpy()
    s2 = _sur(n_in, 5, 256, seed=3)
    s2.train(torch.from_numpy(th).cuda(), torch.from_numpy(y).cuda(), cfg)
    assert np.array_equal(p1, s2.get_params().cpu().numpy())
    s.close()
    s2.close()


def test_surrogate_argument_errors():
    import ctypes
    import paper_2501_12928_amd as eor
    L = eor.lib()
    out = ctypes.c_void_p()
    lo = np.zeros(3)
    hi = np.ones(3)
    assert L.eor_surrogate_create(0, 3, 0, 8, 0, lo.ctypes.data, hi.ctypes.data, ctypes.byref(out)) == eor.EOR_ERR_ARG
    assert L.eor_surrogate_create(0, 3, 2, 8, 0, hi.ctypes.data, lo.ctypes.data, ctypes.byref(out)) == eor.EOR_ERR_ARG
    # hidden width: a multiple of 4 up to 512; inputs: up to 64
    assert L.eor_surrogate_create(0, 3, 2, 37, 0, lo.ctypes.data, hi.ctypes.data, ctypes.byref(out)) == eor.EOR_ERR_ARG
    assert L.eor_surrogate_create(0, 3, 2, 516, 0, lo.ctypes.data, hi.ctypes.data, ctypes.byref(out)) == eor.EOR_ERR_ARG
    lo65, hi65 = np.zeros(65), np.ones(65)
    assert L.eor_surrogate_create(0, 65, 2, 8, 0, lo65.ctypes.data, hi65.ctypes.data,
                                  ctypes.byref(out)) == eor.EOR_ERR_ARG
    s = _sur(3, 2, 8, lo=0.0, hi=1.0)
    # untrained surrogate: inference is refused
    assert L.eor_surrogate_infer(s._h, 4, 1, None, None, None, None) == eor.EOR_ERR_STATE
    s.close()
