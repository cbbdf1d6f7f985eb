"""FP64 oracle of the instrument forward model (test infrastructure only).

The likelihood works on a dense complex matrix T that takes the model's
coefficients (a Fourier-domain sky cube of EoR and foreground modes) to
visibilities. The paper builds T from the primary-beam response of a
baseline and the uv sampling of the data (section "Running BayesEoR") but
prints no formula for it. The reading used here is the textbook visibility
equation on a pixelised sky:

    V_b(nu) = sum_p A(l_p, m_p, nu) I(l_p, m_p, nu) exp(-2 pi i (u_b(nu) l_p + v_b(nu) m_p)),
    u_b(nu) = x_b nu / c,  v_b(nu) = y_b nu / c   (baseline (x_b, y_b) in metres),

with the sky expanded in the model's basis, a 2-D Fourier mode (u_k, v_k)
on the sky times a spectral mode Z[f, e] along frequency:

    I(l, m, nu_f) = norm sum_{e, k} a_{e k} Z[f, e] exp(+2 pi i (u_k l + v_k m)).

Hence

    T[f n_bl + b, e n_uv + k] = norm Z[f, e] sum_p exp(-2 pi i (u_b(nu_f) l_p + v_b(nu_f) m_p))
                                               A[f, p] exp(+2 pi i (u_k l_p + v_k m_p)).

Rows are frequency-major (channel f, then baseline b); columns are
spectral-mode-major (mode e, then uv cell k). This module writes the sum out
as it stands; it imports nothing from the product package.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0  # m / s


def forward_model(freq, bl, lm, beam, uv, Z, norm):
    """T [F n_bl, n_eta n_uv] complex128.

    freq [F] Hz; bl [n_bl, 2] metres; lm [n_pix, 2] direction cosines;
    beam [F, n_pix] real; uv [n_uv, 2] wavelengths; Z [F, n_eta] complex;
    norm: scalar."""
    freq = np.asarray(freq, dtype=np.float64)
    bl = np.asarray(bl, dtype=np.float64)
    lm = np.asarray(lm, dtype=np.float64)
    beam = np.asarray(beam, dtype=np.float64)
    uv = np.asarray(uv, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.complex128)
    F, n_bl, n_uv, n_eta = freq.size, bl.shape[0], uv.shape[0], Z.shape[1]
    # the sky-side Fourier modes do not depend on frequency
    sky = np.exp(2j * np.pi * (np.outer(lm[:, 0], uv[:, 0]) + np.outer(lm[:, 1], uv[:, 1])))  # [n_pix, n_uv]
    T = np.empty((F * n_bl, n_eta * n_uv), dtype=np.complex128)
    for f in range(F):
        u = bl[:, 0] * freq[f] / C_LIGHT
        v = bl[:, 1] * freq[f] / C_LIGHT
        vis = np.exp(-2j * np.pi * (np.outer(u, lm[:, 0]) + np.outer(v, lm[:, 1])))  # [n_bl, n_pix]
        G = (vis * beam[f][None, :]) @ sky                                          # [n_bl, n_uv]
        for e in range(n_eta):
            T[f * n_bl:(f + 1) * n_bl, e * n_uv:(e + 1) * n_uv] = norm * Z[f, e] * G
    return T


def forward_model_entry(freq, bl, lm, beam, uv, Z, norm, row, col):
    """One entry T[row, col] by the sum over pixels, for spot checks at any size."""
    n_bl, n_uv = bl.shape[0], uv.shape[0]
    f, b = divmod(int(row), n_bl)
    e, k = divmod(int(col), n_uv)
    u = bl[b, 0] * freq[f] / C_LIGHT
    v = bl[b, 1] * freq[f] / C_LIGHT
    ph = np.exp(-2j * np.pi * (u * lm[:, 0] + v * lm[:, 1])) * np.exp(2j * np.pi * (uv[k, 0] * lm[:, 0] + uv[k, 1] * lm[:, 1]))
    return norm * Z[f, e] * np.sum(beam[f] * ph)
