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

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


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
        L.eor_group_tuning.argtypes = [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                                       ctypes.POINTER(_I64)]
        L.eor_autotune.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_P), ctypes.c_char_p, _I32, _P]
        for name in ("eor_create", "eor_precompute", "eor_loglike_batch", "eor_loglike_terms",
                     "eor_export_precompute", "eor_shape", "eor_group_create", "eor_group_loglike",
                     "eor_group_set_graph", "eor_group_tuning", "eor_autotune"):
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
        """(prefetch stages, workgroups per CU, graph launches, graph captures)."""
        s, w, r, c = _I32(), _I32(), _I64(), _I64()
        check(lib().eor_group_tuning(self._h, ctypes.byref(s), ctypes.byref(w), ctypes.byref(r),
                                     ctypes.byref(c)))
        return s.value, w.value, r.value, c.value

    def autotune(self, thetas, cache_path=None, force=False, stream=None):
        th, B, tp = self._arrays(thetas)
        cp = None if cache_path is None else str(cache_path).encode()
        check(lib().eor_autotune(self._h, B, tp, cp, 1 if force else 0, _stream(stream)))
        return self.tuning()[:2]


def version() -> str:
    return lib().eor_version().decode()
