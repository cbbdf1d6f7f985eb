"""Batched FP64 marginal likelihood of the 21-cm power spectrum on AMD MI355X.

Thin Python binding over the C ABI in ``include/eor.h`` (``libeor.so``,
HIP for gfx950). Every step of the computation runs in the library's HIP
kernels; this module only marshals arguments. PyTorch supplies device memory
and streams: tensors are passed by ``data_ptr()`` and the current stream.

If the library has not been built, importing works but the first call raises
``RuntimeError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeor.so")

EOR_OK = 0
EOR_ERR_ARG = -1
EOR_ERR_OOM = -2
EOR_ERR_HIP = -3
EOR_ERR_STATE = -4

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x2": 3}

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


class TrainCfg(ctypes.Structure):
    """eor_train_cfg."""
    _fields_ = [("epochs", ctypes.c_int32), ("minibatch", ctypes.c_int32), ("patience", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("val_frac", ctypes.c_float), ("seed", ctypes.c_uint64)]


def train_cfg(epochs=500, minibatch=1024, patience=20, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              val_frac=0.1, seed=0) -> TrainCfg:
    return TrainCfg(epochs, minibatch, patience, lr, beta1, beta2, eps, val_frac, seed)


class EorError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"eor status {status}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libeor.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2501_12928_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        L.eor_last_error.restype = ctypes.c_char_p
        L.eor_version.restype = ctypes.c_char_p
        L.eor_create.argtypes = [ctypes.c_int, ctypes.POINTER(_P)]
        L.eor_destroy.argtypes = [_P]
        L.eor_destroy.restype = None
        L.eor_precompute.argtypes = [_P, _I64, _I64, _P, _I64, _P, _P, _I32, _P, _P, _P, ctypes.c_int, _P]
        L.eor_loglike_batch.argtypes = [_P, _I64, _P, _P, _P, _P]
        L.eor_loglike_terms.argtypes = [_P, _I64, _P, _P, _P, _P, _P]
        L.eor_export_precompute.argtypes = [_P, _P, _I64, _P, _P, _P]
        L.eor_shape.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)]
        L.eor_group_create.argtypes = [_I32, ctypes.POINTER(_P), ctypes.POINTER(_P)]
        L.eor_group_destroy.argtypes = [_P]
        L.eor_group_destroy.restype = None
        L.eor_group_loglike.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                        ctypes.POINTER(_P), _P]
        L.eor_group_set_graph.argtypes = [_P, _I32]
        L.eor_group_tuning.argtypes = [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                       ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
        L.eor_group_set_tuning.argtypes = [_P, _I32, _I32, _I32]
        L.eor_set_tuning.argtypes = [_P, _I32, _I32, _I32]
        L.eor_set_workspace_limit.argtypes = [_P, ctypes.c_size_t]
        L.eor_set_tile_size.argtypes = [_P, _I32]
        L.eor_get_tile_size.argtypes = [_P, ctypes.POINTER(_I32)]
        L.eor_group_set_tile_sizes.argtypes = [_P, _P]
        L.eor_group_tile_sizes.argtypes = [_P, _P]
        L.eor_get_tuning.argtypes = [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]
        L.eor_autotune.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_P), ctypes.c_char_p, _I32, _P]
        L.eor_surrogate_create.argtypes = [ctypes.c_int, _I32, _I32, _I32, ctypes.c_uint64, _P, _P,
                                           ctypes.POINTER(_P)]
        L.eor_surrogate_destroy.argtypes = [_P]
        L.eor_surrogate_destroy.restype = None
        L.eor_surrogate_size.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32)]
        L.eor_surrogate_params.argtypes = [_P, _P, _P, _P]
        L.eor_surrogate_standardisation.argtypes = [_P, _P, _P]
        L.eor_surrogate_train.argtypes = [_P, _I64, _P, _P, ctypes.POINTER(TrainCfg), _P]
        L.eor_surrogate_report.argtypes = [_P, ctypes.POINTER(_I32), _P]
        L.eor_surrogate_loss_grad.argtypes = [_P, _I64, _P, _P, _P, _P, _P]
        L.eor_surrogate_adam_step.argtypes = [_P, ctypes.POINTER(TrainCfg), _P]
        L.eor_surrogate_infer.argtypes = [_P, _I64, _P, _P, _P, _P, _P]
        L.eor_surrogate_gate.argtypes = [_P, _I64, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P]
        L.eor_surrogate_gate_noalloc.argtypes = [_P, _I64, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                                 _P, _P]
        L.eor_compact_rows.argtypes = [_I64, _I32, _P, _P, _P, _P, _P, _P]
        L.eor_probe_fp64_mfma.argtypes = [ctypes.c_int, _I64, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
        L.eor_loglike_host.argtypes = [ctypes.c_int, _I64, _P, _I64, _P, ctypes.c_double, ctypes.c_double, _I32,
                                       _P, _P, _P, _I64, _P, ctypes.c_size_t, _I32, _P, _P]
        L.eor_loglike_host_plan.argtypes = [_I64, _I32, ctypes.c_size_t, _I32, _P, _P, _P, _P]
        L.eor_forward_model.argtypes = [_I64, _I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, ctypes.c_double,
                                        _P, _I64, _P]
        for name in ("eor_create", "eor_precompute", "eor_loglike_batch", "eor_loglike_terms",
                     "eor_export_precompute", "eor_shape", "eor_group_create", "eor_group_loglike",
                     "eor_group_set_graph", "eor_group_tuning", "eor_group_set_tuning", "eor_set_tuning",
                     "eor_set_workspace_limit", "eor_set_tile_size", "eor_get_tile_size",
                     "eor_group_set_tile_sizes", "eor_group_tile_sizes",
                     "eor_get_tuning", "eor_autotune", "eor_surrogate_create",
                     "eor_surrogate_size", "eor_surrogate_params", "eor_surrogate_standardisation",
                     "eor_surrogate_train", "eor_surrogate_report", "eor_surrogate_loss_grad",
                     "eor_surrogate_adam_step", "eor_surrogate_infer", "eor_surrogate_gate",
                     "eor_surrogate_gate_noalloc",
                     "eor_compact_rows", "eor_probe_fp64_mfma", "eor_forward_model", "eor_loglike_host",
                     "eor_loglike_host_plan"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != EOR_OK:
        raise EorError(status, lib().eor_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    import torch
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    if not t.is_cuda:
        t = t.cuda()
    t = t.to(dtype)
    return t.contiguous()


class Context:
    """One dataset on one GPU: precompute once, then logL for theta batches."""

    def __init__(self, device: int = 0):
        self._h = _P()
        check(lib().eor_create(int(device), ctypes.byref(self._h)))
        self.device = device
        self.n_k = 0

    def close(self):
        if self._h:
            lib().eor_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def precompute(self, T, noise_var, d, n_k, bin_of, fixed_var=None, bin_scale=None,
                   prec: str = "fp64", stream=None):
        """T [m, n] complex128, noise_var [m], d [m] (device tensors or
        arrays); bin_of [n] int, fixed_var [n], bin_scale [n_k] on the host."""
        import torch
        T = _dev(T, torch.complex128)
        noise_var = _dev(noise_var, torch.float64)
        d = _dev(d, torch.complex128)
        m, n = T.shape
        bin_of = np.ascontiguousarray(bin_of, dtype=np.int32)
        fv = None if fixed_var is None else np.ascontiguousarray(fixed_var, dtype=np.float64)
        bs = None if bin_scale is None else np.ascontiguousarray(bin_scale, dtype=np.float64)
        check(lib().eor_precompute(self._h, m, n, T.data_ptr(), n, noise_var.data_ptr(), d.data_ptr(),
                                   int(n_k), bin_of.ctypes.data,
                                   None if fv is None else fv.ctypes.data,
                                   None if bs is None else bs.ctypes.data,
                                   PREC[prec], _stream(stream)))
        self.n_k = int(n_k)
        self.m, self.n = int(m), int(n)
        return self

    def loglike_batch(self, theta, stream=None, out=None, info=None):
        """logL [B] float64 and info [B] int32 (device tensors) for theta [B, n_k]."""
        import torch
        theta = _dev(theta, torch.float64)
        B = theta.shape[0] if theta.dim() > 0 else 0
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        if info is None:
            info = torch.empty(B, dtype=torch.int32, device=theta.device)
        check(lib().eor_loglike_batch(self._h, B, theta.data_ptr(), out.data_ptr(), info.data_ptr(),
                                      _stream(stream)))
        return out, info

    def loglike_terms(self, theta, stream=None):
        """logL, info and terms [B, 4] = (ln det Sigma, dbar^H Sigma^-1 dbar, ln det Phi, c)."""
        import torch
        theta = _dev(theta, torch.float64)
        B = theta.shape[0]
        out = torch.empty(B, dtype=torch.float64, device=theta.device)
        info = torch.empty(B, dtype=torch.int32, device=theta.device)
        terms = torch.empty((B, 4), dtype=torch.float64, device=theta.device)
        check(lib().eor_loglike_terms(self._h, B, theta.data_ptr(), out.data_ptr(), info.data_ptr(),
                                      terms.data_ptr(), _stream(stream)))
        return out, info, terms

    def set_tuning(self, stages, wg_per_cu, tiles_per_pass=1):
        """Launch choices of loglike_batch / loglike_terms (see eor_set_tuning)."""
        check(lib().eor_set_tuning(self._h, stages, wg_per_cu, tiles_per_pass))

    def set_workspace_limit(self, nbytes: int):
        """Device-memory budget of the per-theta workspace (0 = none); see
        eor_set_workspace_limit."""
        check(lib().eor_set_workspace_limit(self._h, int(nbytes)))

    def set_tile_size(self, ts: int):
        """Side of the factorisation tiles, 64 or 32 (eor_set_tile_size)."""
        check(lib().eor_set_tile_size(self._h, int(ts)))

    def tile_size(self) -> int:
        v = _I32()
        check(lib().eor_get_tile_size(self._h, ctypes.byref(v)))
        return v.value

    def tuning(self):
        """(prefetch stages, workgroups per CU, tiles per pass)."""
        s, w, t = _I32(), _I32(), _I32()
        check(lib().eor_get_tuning(self._h, ctypes.byref(s), ctypes.byref(w), ctypes.byref(t)))
        return s.value, w.value, t.value

    def export_precompute(self, stream=None):
        """(A [n, n] complex128 full Hermitian, dbar [n], c, K0)."""
        import torch
        A = torch.empty((self.n, self.n), dtype=torch.complex128, device=f"cuda:{self.device}")
        dbar = torch.empty(self.n, dtype=torch.complex128, device=A.device)
        sc = (ctypes.c_double * 2)()
        check(lib().eor_export_precompute(self._h, A.data_ptr(), self.n, dbar.data_ptr(), sc,
                                          _stream(stream)))
        return A, dbar, sc[0], sc[1]


class Group:
    """Several precomputed contexts evaluated in one persistent launch."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        n = len(self.contexts)
        arr = (_P * n)(*[c.handle for c in self.contexts])
        self._h = _P()
        check(lib().eor_group_create(n, arr, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().eor_group_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _arrays(self, thetas):
        import torch
        n = len(self.contexts)
        if len(thetas) != n:
            raise ValueError("one theta batch per context")
        th = [_dev(t, torch.float64) for t in thetas]
        B = (_I64 * n)(*[t.shape[0] for t in th])
        tp = (_P * n)(*[t.data_ptr() for t in th])
        return th, B, tp

    def loglike(self, thetas, stream=None, with_info=True, outs=None, infos=None):
        """Lists of logL (and info) device tensors, one per context. Passing
        the previous call's `outs`/`infos` keeps the pointers unchanged, so
        the captured graph is replayed as is."""
        import torch
        th, B, tp = self._arrays(thetas)
        if outs is None:
            outs = [torch.empty(t.shape[0], dtype=torch.float64, device=t.device) for t in th]
        if infos is None:
            infos = [torch.empty(t.shape[0], dtype=torch.int32, device=t.device) for t in th]
        n = len(th)
        op = (_P * n)(*[o.data_ptr() for o in outs])
        ip = (_P * n)(*[i.data_ptr() for i in infos]) if with_info else None
        check(lib().eor_group_loglike(self._h, B, tp, op, ip, _stream(stream)))
        return (outs, infos) if with_info else outs

    def set_graph(self, enable: bool):
        check(lib().eor_group_set_graph(self._h, 1 if enable else 0))

    def tuning(self):
        """(prefetch stages, workgroups per CU, tiles per pass, graph launches, graph captures)."""
        s, w, t, r, c = _I32(), _I32(), _I32(), _I64(), _I64()
        check(lib().eor_group_tuning(self._h, ctypes.byref(s), ctypes.byref(w), ctypes.byref(t),
                                     ctypes.byref(r), ctypes.byref(c)))
        return s.value, w.value, t.value, r.value, c.value

    def set_tuning(self, stages, wg_per_cu, tiles_per_pass=1):
        check(lib().eor_group_set_tuning(self._h, stages, wg_per_cu, tiles_per_pass))

    def set_tile_sizes(self, ts_per_bucket):
        """Tile side (32 or 64) per size bucket of n: <= 512, <= 1024, <= 2048,
        <= 4096, larger."""
        v = np.ascontiguousarray(ts_per_bucket, dtype=np.int32)
        if v.shape != (5,):
            raise ValueError("five tile sides, one per size bucket")
        check(lib().eor_group_set_tile_sizes(self._h, v.ctypes.data))

    def tile_sizes(self):
        v = np.zeros(5, dtype=np.int32)
        check(lib().eor_group_tile_sizes(self._h, v.ctypes.data))
        return v.tolist()

    def autotune(self, thetas, cache_path=None, force=False, stream=None):
        """Time every launch choice on this batch, keep the fastest and return
        it as (stages, workgroups per CU, tiles per pass)."""
        th, B, tp = self._arrays(thetas)
        cp = None if cache_path is None else str(cache_path).encode()
        check(lib().eor_autotune(self._h, B, tp, cp, 1 if force else 0, _stream(stream)))
        return self.tuning()[:3]


class Surrogate:
    """Ensemble of MLP surrogates of logL(theta) (FP32, trained on the GPU)."""

    def __init__(self, n_in, lo, hi, n_members=5, hidden=256, seed=0, device=0):
        lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, dtype=np.float64), (n_in,)))
        hi = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, dtype=np.float64), (n_in,)))
        self._h = _P()
        check(lib().eor_surrogate_create(int(device), int(n_in), int(n_members), int(hidden), int(seed),
                                         lo.ctypes.data, hi.ctypes.data, ctypes.byref(self._h)))
        self.n_in, self.M, self.H, self.device = int(n_in), int(n_members), int(hidden), device
        P = _I64()
        check(lib().eor_surrogate_size(self._h, ctypes.byref(P), None))
        self.P = P.value

    def close(self):
        if self._h:
            lib().eor_surrogate_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import torch
        out = torch.empty((self.M, self.P), dtype=torch.float32, device=f"cuda:{self.device}")
        check(lib().eor_surrogate_params(self._h, out.data_ptr(), None, _stream()))
        return out

    def set_params(self, p):
        import torch
        p = _dev(p, torch.float32).reshape(self.M, self.P).contiguous()
        check(lib().eor_surrogate_params(self._h, None, p.data_ptr(), _stream()))

    def standardisation(self, mean_std=None):
        out = np.zeros(2)
        st = None if mean_std is None else np.ascontiguousarray(mean_std, dtype=np.float64)
        check(lib().eor_surrogate_standardisation(self._h, out.ctypes.data,
                                                  None if st is None else st.ctypes.data))
        return out if st is None else st

    def train(self, theta, logL, cfg=None, stream=None):
        import torch
        theta = _dev(theta, torch.float64)
        logL = _dev(logL, torch.float64)
        cfg = cfg or train_cfg()
        check(lib().eor_surrogate_train(self._h, theta.shape[0], theta.data_ptr(), logL.data_ptr(),
                                        ctypes.byref(cfg), _stream(stream)))
        ep = _I32()
        val = np.zeros(self.M)
        check(lib().eor_surrogate_report(self._h, ctypes.byref(ep), val.ctypes.data))
        return ep.value, val

    def loss_grad(self, x, y):
        import torch
        x = _dev(x, torch.float32)
        y = _dev(y, torch.float32)
        nb = y.shape[-1]
        loss = torch.empty(self.M, dtype=torch.float32, device=x.device)
        grad = torch.empty((self.M, self.P), dtype=torch.float32, device=x.device)
        check(lib().eor_surrogate_loss_grad(self._h, nb, x.data_ptr(), y.data_ptr(), loss.data_ptr(),
                                            grad.data_ptr(), _stream()))
        return loss, grad

    def adam_step(self, cfg):
        check(lib().eor_surrogate_adam_step(self._h, ctypes.byref(cfg), _stream()))

    def infer(self, theta, members=False):
        import torch
        theta = _dev(theta, torch.float64)
        B = theta.shape[0]
        mean = torch.empty(B, dtype=torch.float64, device=theta.device)
        spread = torch.empty(B, dtype=torch.float64, device=theta.device)
        mem = torch.empty((self.M, B), dtype=torch.float32, device=theta.device) if members else None
        check(lib().eor_surrogate_infer(self._h, B, theta.data_ptr(), mean.data_ptr(), spread.data_ptr(),
                                        None if mem is None else mem.data_ptr(), _stream()))
        return (mean, spread, mem) if members else (mean, spread)

    def gate(self, theta, L_min, tau):
        """(mean, spread, decision): decision 1 = evaluate exactly, 0 = reject."""
        import torch
        theta = _dev(theta, torch.float64)
        B = theta.shape[0]
        mean = torch.empty(B, dtype=torch.float64, device=theta.device)
        spread = torch.empty(B, dtype=torch.float64, device=theta.device)
        dec = torch.empty(B, dtype=torch.int32, device=theta.device)
        check(lib().eor_surrogate_gate(self._h, B, theta.data_ptr(), float(L_min), float(tau), mean.data_ptr(),
                                       spread.data_ptr(), None, dec.data_ptr(), _stream()))
        return mean, spread, dec


def compact_rows(keep, rows=None):
    """(rows_out, index_out, count) for the rows with keep != 0, in order."""
    import torch
    keep = _dev(keep, torch.int32)
    n = keep.shape[0]
    n_cols = 0 if rows is None else (rows.shape[1] if rows.dim() > 1 else 1)
    if rows is not None:
        rows = _dev(rows, torch.float64)
    out = torch.empty((max(n, 1), max(n_cols, 1)), dtype=torch.float64, device=keep.device) if rows is not None else None
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=keep.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=keep.device)
    check(lib().eor_compact_rows(n, n_cols, keep.data_ptr(), None if rows is None else rows.data_ptr(),
                                 None if out is None else out.data_ptr(), idx.data_ptr(), cnt.data_ptr(), _stream()))
    c = int(cnt.item())
    return (None if out is None else out[:c]), idx[:c], c


def loglike_host(A, dbar, c, K0, n_k, bin_of, fixed_var, bin_scale, theta, device_bytes, device=0, lanes=0):
    """(logL [B], info [B]) of eor_loglike_host: A (complex128 [n, n], host,
    lower triangle read) and the rest in host memory; the device uses at most
    `device_bytes` (Sigma factored out of core, `lanes` theta at a time, 0 =
    the library's choice)."""
    A = np.asarray(A, dtype=np.complex128)
    if not A.flags.c_contiguous:
        A = np.ascontiguousarray(A)
    dbar = np.ascontiguousarray(dbar, dtype=np.complex128)
    bin_of = np.ascontiguousarray(bin_of, dtype=np.int32)
    fixed_var = np.ascontiguousarray(fixed_var, dtype=np.float64)
    bs = None if bin_scale is None else np.ascontiguousarray(bin_scale, dtype=np.float64)
    theta = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
    n, B = A.shape[0], theta.shape[0]
    logL = np.empty(B)
    info = np.empty(B, dtype=np.int32)
    check(lib().eor_loglike_host(int(device), n, A.ctypes.data, A.shape[1], dbar.ctypes.data, float(c), float(K0),
                                 int(n_k), bin_of.ctypes.data, fixed_var.ctypes.data,
                                 None if bs is None else bs.ctypes.data, B, theta.ctypes.data, int(device_bytes),
                                 int(lanes), logL.ctypes.data, info.ctypes.data))
    return logL, info


def loglike_host_plan(n, n_k, device_bytes, lanes=0):
    """The schedule eor_loglike_host follows (host only): dict of lanes,
    cols_per_pass, window_tiles and link_bytes (host <-> device per theta)."""
    lo = ctypes.c_int32()
    J, W, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().eor_loglike_host_plan(int(n), int(n_k), int(device_bytes), int(lanes), ctypes.byref(lo),
                                      ctypes.byref(J), ctypes.byref(W), ctypes.byref(nb)))
    return {"lanes": lo.value, "cols_per_pass": J.value, "window_tiles": W.value, "link_bytes": nb.value}


def forward_model(freq, bl, lm, beam, uv, Z, norm, out=None):
    """T [F n_bl, n_eta n_uv] complex128 on the GPU from the instrument
    (freq [F] Hz, bl [n_bl, 2] m, lm [n_pix, 2], beam [F, n_pix]), the model
    cells uv [n_uv, 2] and spectral modes Z [F, n_eta] (complex): the
    visibility equation of eor_forward_model."""
    import torch
    freq = _dev(freq, torch.float64)
    bl = _dev(bl, torch.float64)
    lm = _dev(lm, torch.float64)
    beam = _dev(beam, torch.float64)
    uv = _dev(uv, torch.float64)
    Z = _dev(Z, torch.complex128)
    F, n_bl, n_pix, n_uv, n_eta = freq.shape[0], bl.shape[0], lm.shape[0], uv.shape[0], Z.shape[1]
    if out is None:
        out = torch.empty((F * n_bl, n_eta * n_uv), dtype=torch.complex128, device=freq.device)
    check(lib().eor_forward_model(F, n_bl, n_pix, n_uv, n_eta, freq.data_ptr(), bl.data_ptr(), lm.data_ptr(),
                                  beam.data_ptr(), uv.data_ptr(), Z.data_ptr(), float(norm), out.data_ptr(),
                                  out.stride(0), _stream()))
    return out


def version() -> str:
    return lib().eor_version().decode()


def probe_fp64_mfma(iters: int, device: int = 0):
    """(TFLOP/s, ms) of back-to-back FP64 MFMAs on every CU for `iters`
    rounds: the device's measured FP64 matrix peak over a run that long."""
    t = ctypes.c_double()
    ms = ctypes.c_double()
    check(lib().eor_probe_fp64_mfma(device, int(iters), ctypes.byref(t), ctypes.byref(ms)))
    return t.value, ms.value
