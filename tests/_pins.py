"""Independent routes to the marginal likelihood, used to pin the oracle.

None of these goes through A = T^H N^{-1} T or a Cholesky factor: they work
on the data-space covariance C = N + T Phi T^H (brute force), on a diagonal
instrument (closed form), or on an eigendecomposition (closed form for a
single-bin prior).
"""
from __future__ import annotations

import math

import numpy as np


def prior_var(theta, bin_of, fixed_var, bin_scale=None):
    """phi_j = s_b 10^theta_b for bin b >= 0, else the fixed variance."""
    theta = np.asarray(theta, dtype=np.float64)
    b = np.asarray(bin_of)
    s = np.ones(int(b.max()) + 1 if b.max() >= 0 else 1) if bin_scale is None else np.asarray(bin_scale)
    out = np.array(fixed_var, dtype=np.float64, copy=True)
    sel = b >= 0
    out[sel] = s[b[sel]] * 10.0 ** theta[b[sel]]
    return out


def brute_loglike(T, noise_var, d, theta, bin_of, fixed_var, bin_scale=None):
    """D1 directly: -m ln pi - ln det C - d^H C^{-1} d, C = N + T Phi T^H,
    with LU (slogdet, solve) on the m x m matrix."""
    m = T.shape[0]
    phi = prior_var(theta, bin_of, fixed_var, bin_scale)
    C = np.diag(np.asarray(noise_var, dtype=np.complex128)) + (T * phi[None, :]) @ T.conj().T
    sign, logdet = np.linalg.slogdet(C)
    assert abs(sign - 1.0) < 1e-8
    quad = np.real(np.vdot(d, np.linalg.solve(C, d)))
    return -m * math.log(math.pi) - logdet - quad


def brute_loglike_mp(T, noise_var, d, theta, bin_of, fixed_var, dps=50):
    """D1 in mpmath at `dps` digits (tiny sizes only)."""
    import mpmath as mp
    mp.mp.dps = dps
    m, n = T.shape
    phi = [mp.mpf(10) ** mp.mpf(float(theta[b])) if b >= 0 else mp.mpf(float(v))
           for b, v in zip(bin_of, fixed_var)]
    Tm = [[mp.mpc(complex(T[i, j])) for j in range(n)] for i in range(m)]
    C = mp.matrix(m, m)
    for i in range(m):
        for k in range(m):
            s = mp.mpc(0)
            for j in range(n):
                s += Tm[i][j] * phi[j] * mp.conj(Tm[k][j])
            C[i, k] = s + (mp.mpf(float(noise_var[i])) if i == k else 0)
    dv = mp.matrix([mp.mpc(complex(x)) for x in d])
    x = mp.lu_solve(C, dv)
    quad = mp.re(sum(mp.conj(dv[i]) * x[i] for i in range(m)))
    logdet = mp.re(mp.log(mp.det(C)))
    return float(-m * mp.log(mp.pi) - logdet - quad)


def diagonal_closed_form(noise_var, d, theta, bin_of, fixed_var, n, bin_scale=None):
    """T = [I_n; 0]: C is diagonal, sigma_j^2 + phi_j for j < n, sigma_i^2 after."""
    phi = prior_var(theta, bin_of, fixed_var, bin_scale)
    v = np.asarray(noise_var, dtype=np.float64).copy()
    v[:n] += phi
    return float(np.sum(-math.log(math.pi) - np.log(v) - np.abs(d) ** 2 / v))


def eigen_closed_form(T, noise_var, d, thetas, scale=1.0):
    """One bin, no fixed coefficients: Sigma = A + 10^-theta/s I, so with
    A = V diag(lam) V^H (numpy ZGEMM + ZHEEVD),
    ln det Sigma = sum ln(lam + 10^-theta/s),
    dbar^H Sigma^{-1} dbar = sum |V^H dbar|^2 / (lam + 10^-theta/s)."""
    m, n = T.shape
    W = T / np.sqrt(noise_var)[:, None]
    A = W.conj().T @ W
    dbar = W.conj().T @ (d / np.sqrt(noise_var))
    c = float(np.sum(np.abs(d) ** 2 / noise_var))
    K0 = -m * math.log(math.pi) - float(np.sum(np.log(noise_var)))
    lam, V = np.linalg.eigh(A)
    g = np.abs(V.conj().T @ dbar) ** 2
    out = []
    for th in np.atleast_1d(thetas):
        mu = 10.0 ** (-th) / scale
        ldS = float(np.sum(np.log(lam + mu)))
        quad = float(np.sum(g / (lam + mu)))
        ldP = n * (th * math.log(10.0) + math.log(scale))
        out.append(K0 - ldP - ldS - (c - quad))
    return np.array(out)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)
