"""CPU FP64 oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library neither links nor
calls it, and it imports nothing from the product package.

``oracle.c`` holds the marginal likelihood (plain C, FP64, no BLAS); this
module builds it with gcc and calls it through ctypes. ``mlp.py`` holds the
surrogate network's forward/backward/Adam, the ensemble statistics and the
gate rule in numpy FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c99",
          "-fPIC", "-shared", "-Wall"]


def lib_path(mutant: int = 0, out_dir: str | None = None) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mut{mutant}.so"
    return os.path.join(out_dir or _HERE, name)


def build(mutant: int = 0, out_dir: str | None = None, force: bool = True) -> str:
    """Compile oracle.c (optionally a planted-mistake mutant) with gcc."""
    out = lib_path(mutant, out_dir)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    cmd = ["gcc", *CFLAGS, _SRC, "-o", out + ".tmp", "-lm"]
    if mutant:
        cmd.insert(1, f"-DORACLE_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_P = ctypes.c_void_p
_I64 = ctypes.c_int64


class Oracle:
    """ctypes view of one build of oracle.c."""

    def __init__(self, mutant: int = 0, out_dir: str | None = None):
        path = build(mutant, out_dir, force=False)
        self.lib = ctypes.CDLL(path)
        self.lib.oracle_precompute.argtypes = [_I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, ctypes.c_int]
        self.lib.oracle_precompute.restype = ctypes.c_int
        self.lib.oracle_loglike.argtypes = [_I64, _P, _P, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32, _P, _P, _P, _I64, _P, _P, _P, _P,
                                            ctypes.c_int]
        self.lib.oracle_loglike.restype = ctypes.c_int
        self.lib.oracle_build_id.restype = ctypes.c_char_p

    def precompute(self, T, noise_var, d, nthreads: int = 0):
        """A (n x n full Hermitian), dbar, c, K0 from T, sigma^2, d."""
        T = np.ascontiguousarray(T, dtype=np.complex128)
        noise_var = np.ascontiguousarray(noise_var, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.complex128)
        m, n = T.shape
        A = np.empty((n, n), dtype=np.complex128)
        dbar = np.empty(n, dtype=np.complex128)
        c = ctypes.c_double()
        K0 = ctypes.c_double()
        rc = self.lib.oracle_precompute(m, n, T.ctypes.data, n, noise_var.ctypes.data,
                                        d.ctypes.data, A.ctypes.data, dbar.ctypes.data,
                                        ctypes.byref(c), ctypes.byref(K0), nthreads)
        if rc != 0:
            raise ValueError("oracle_precompute rejected its arguments")
        return A, dbar, c.value, K0.value

    def loglike(self, A, dbar, c, K0, n_k, bin_of, fixed_var, bin_scale, theta,
                nthreads: int = 0, terms: bool = False):
        """logL[B], info[B] (and terms[B,4] if asked) for theta[B, n_k]."""
        A = np.ascontiguousarray(A, dtype=np.complex128)
        dbar = np.ascontiguousarray(dbar, dtype=np.complex128)
        bin_of = np.ascontiguousarray(bin_of, dtype=np.int32)
        fixed_var = np.ascontiguousarray(fixed_var, dtype=np.float64)
        theta = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        n = A.shape[0]
        B = theta.shape[0]
        bs = None if bin_scale is None else np.ascontiguousarray(bin_scale, dtype=np.float64)
        logL = np.empty(B, dtype=np.float64)
        info = np.empty(B, dtype=np.int32)
        tm = np.empty((B, 4), dtype=np.float64)
        rc = self.lib.oracle_loglike(n, A.ctypes.data, dbar.ctypes.data, float(c), float(K0),
                                     int(n_k), bin_of.ctypes.data, fixed_var.ctypes.data,
                                     None if bs is None else bs.ctypes.data, B,
                                     theta.ctypes.data, logL.ctypes.data, info.ctypes.data,
                                     tm.ctypes.data, nthreads)
        if rc != 0:
            raise ValueError("oracle_loglike rejected its arguments")
        return (logL, info, tm) if terms else (logL, info)

    def loglike_instance(self, inst, theta=None, nthreads: int = 0, terms: bool = False,
                         pre=None):
        """Full path on a synth.Instance: precompute then per-theta logL."""
        if pre is None:
            pre = self.precompute(inst.T, inst.noise_var, inst.d, nthreads)
        A, dbar, c, K0 = pre
        th = inst.theta if theta is None else theta
        return self.loglike(A, dbar, c, K0, inst.n_k, inst.bin_of, inst.fixed_var,
                            inst.bin_scale, th, nthreads=nthreads, terms=terms)


_default: Oracle | None = None


def get() -> Oracle:
    """The normal (non-mutant) oracle build, loaded once."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
