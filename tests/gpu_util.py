"""Helpers of the GPU tests: move a synth.Instance through the C ABI."""
import numpy as np


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def run_instance(inst, theta=None, prec="fp64", terms=False, tuning=None, ts=None):
    import torch
    import paper_2501_12928_amd as eor
    ctx = eor.Context(0)
    if tuning is not None:
        ctx.set_tuning(*tuning)
    if ts is not None:
        ctx.set_tile_size(ts)
    ctx.precompute(torch.from_numpy(inst.T).cuda(), torch.from_numpy(inst.noise_var).cuda(),
                   torch.from_numpy(inst.d).cuda(), inst.n_k, inst.bin_of, inst.fixed_var,
                   inst.bin_scale, prec=prec)
    th = torch.from_numpy(np.ascontiguousarray(inst.theta if theta is None else theta)).cuda()
    if terms:
        logL, info, tm = ctx.loglike_terms(th)
        torch.cuda.synchronize()
        out = (logL.cpu().numpy(), info.cpu().numpy(), tm.cpu().numpy())
    else:
        logL, info = ctx.loglike_batch(th)
        torch.cuda.synchronize()
        out = (logL.cpu().numpy(), info.cpu().numpy())
    ctx.close()
    return out


def tol(ref):
    """The required parity bound: |dlogL| <= 1e-6 |logL| + 1e-6."""
    return 1e-6 * np.abs(ref) + 1e-6
