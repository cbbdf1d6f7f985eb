"""The allocation-free gate (eor_surrogate_gate_noalloc) against the gate it
varies (eor_surrogate_gate): the same means, spreads, member outputs and
decisions, on two calls in a row (the second smaller, so it runs on what the
first left in the fixed scratch), through the C ABI; a batch beyond the
scratch is refused before any launch."""
import numpy as np
import pytest

from oracle import mlp
from tests.gpu_util import have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="no GPU")]


def _gate(lib, fn, s, th, L_min, tau, M):
    import torch
    B = th.shape[0]
    mean = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
    spread = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
    mem = torch.full((M, B), np.nan, dtype=torch.float32, device="cuda")
    dec = torch.full((B,), -7, dtype=torch.int32, device="cuda")
    st = getattr(lib, fn)(s._h, B, th.data_ptr(), L_min, tau, mean.data_ptr(), spread.data_ptr(),
                          mem.data_ptr(), dec.data_ptr(), None)
    assert st == 0, lib.eor_last_error()
    torch.cuda.synchronize()
    return mean.cpu().numpy(), spread.cpu().numpy(), mem.cpu().numpy(), dec.cpu().numpy()


def test_gate_noalloc_matches_gate():
    import torch
    import paper_2501_12928_amd as eor
    lib = eor.lib()
    n_in, M, H = 12, 5, 256
    rng = np.random.default_rng(11)
    s = eor.Surrogate(n_in, -1.0, 3.0, n_members=M, hidden=H, seed=4)
    th = rng.uniform(-1.0, 3.0, size=(3000, n_in))
    y = -0.5 * np.sum((th - 1.0) ** 2, axis=1) * 40.0
    print("gpu: no-alloc gate, training a 5-member surrogate", flush=True)
    s.train(th, y, cfg=eor.train_cfg(epochs=30, minibatch=256, patience=5, seed=2))
    ymean, ystd = s.standardisation()
    tau = float(ystd)  # trained members agree within one target sd: decisions follow the mean
    for B in (70001, 777):
        print(f"gpu: no-alloc gate vs gate, B={B}", flush=True)
        t = torch.from_numpy(rng.uniform(-1.0, 3.0, size=(B, n_in))).cuda()
        L_min = float(np.median(y))
        a = _gate(lib, "eor_surrogate_gate", s, t, L_min, tau, M)
        b = _gate(lib, "eor_surrogate_gate_noalloc", s, t, L_min, tau, M)
        for x, z in zip(a, b):
            assert np.array_equal(x, z)
        assert np.all(np.isfinite(a[0])) and set(np.unique(a[3])) <= {0, 1}
        assert 0 < np.sum(a[3] == 0) < B
        # the oracle's gate rule on the kernel's mean and spread
        np.testing.assert_array_equal(b[3], mlp.gate(b[0], b[1], L_min, tau))
    # beyond the fixed scratch: refused, outputs untouched
    Bmax = (1 << 22) // M
    big = torch.zeros((Bmax + 1, n_in), dtype=torch.float64, device="cuda")
    out = torch.full((Bmax + 1,), 5.0, dtype=torch.float64, device="cuda")
    st = lib.eor_surrogate_gate_noalloc(s._h, Bmax + 1, big.data_ptr(), 0.0, 0.05, out.data_ptr(), None, None,
                                        None, None)
    assert st == eor.EOR_ERR_ARG and b"scratch" in lib.eor_last_error()
    torch.cuda.synchronize()
    assert torch.all(out == 5.0)
    assert lib.eor_surrogate_gate_noalloc(s._h, 0, None, 0.0, 0.05, None, None, None, None, None) == eor.EOR_OK
    s.close()
