"""Pins of the forward-model oracle (oracle/forward_model.py) against closed
forms that do not go through its sum: the discrete Fourier orthogonality of
a regular pixel grid, and the geometric-series value of the pixel sum for a
beam that is a product of cosines, at several channels, baselines, uv cells
and spectral modes (so that signs, the frequency scaling of the baseline,
the normalisation and the row and column order are all exercised)."""
import numpy as np

from oracle import forward_model as fm


def _grid(N, delta, l0=None):
    """Pixel centres of an N x N grid with spacing delta, lm [N*N, 2]
    (l varies fastest), and the 1-D coordinates."""
    x = (np.arange(N) - N // 2) * delta if l0 is None else l0 + np.arange(N) * delta
    L, M = np.meshgrid(x, x, indexing="xy")
    return np.stack([L.ravel(), M.ravel()], axis=1), x


def _dirichlet(x, coords):
    """sum_i exp(2 pi i x c_i) over an arithmetic progression c_i = c_0 + i d,
    by the geometric series."""
    c0, d, N = coords[0], coords[1] - coords[0], coords.size
    x = np.asarray(x, dtype=np.float64)
    r = np.exp(2j * np.pi * x * d)
    out = np.empty(x.shape, dtype=np.complex128)
    near = np.abs(r - 1.0) < 1e-12
    out[near] = N
    out[~near] = (1.0 - r[~near] ** N) / (1.0 - r[~near])
    return np.exp(2j * np.pi * x * c0) * out


def test_orthogonal_grid_selects_the_matching_uv_cell():
    """Uniform beam, one channel, baselines and model cells on the grid's
    Fourier lattice: the pixel sum is N^2 where the cells coincide and zero
    elsewhere, so T is norm Z times N^2 times a selection."""
    rng = np.random.default_rng(11)
    N, delta = 12, 0.01
    lm, _ = _grid(N, delta)
    du = 1.0 / (N * delta)
    nu = 150e6
    cells = [(kx, ky) for kx in range(-3, 3) for ky in range(-2, 2)]
    uv = np.array([(kx * du, ky * du) for kx, ky in cells])
    pick = rng.choice(len(cells), 7, replace=False)
    # baseline (x, y) metres such that x nu / c = kx du
    bl = np.array([(cells[i][0] * du * fm.C_LIGHT / nu, cells[i][1] * du * fm.C_LIGHT / nu) for i in pick])
    beam = np.ones((1, N * N))
    Z = (rng.standard_normal((1, 3)) + 1j * rng.standard_normal((1, 3)))
    norm = 0.37
    T = fm.forward_model([nu], bl, lm, beam, uv, Z, norm)
    expect = np.zeros_like(T)
    for b, i in enumerate(pick):
        for e in range(3):
            expect[b, e * len(cells) + i] = norm * Z[0, e] * N * N
    np.testing.assert_allclose(T, expect, atol=1e-9 * N * N)


def test_cosine_beam_matches_geometric_series():
    """Beam A_f(l, m) = cos(2 pi s_f l) cos(2 pi t_f m) on a regular grid:
    the pixel sum factorises into two 1-D sums, each half the sum of two
    geometric series, at arbitrary (non-lattice) baselines and cells."""
    rng = np.random.default_rng(12)
    N, delta, l0 = 9, 0.013, -0.05
    lm, x = _grid(N, delta, l0)
    freq = np.array([140e6, 151.5e6, 163e6])
    s = np.array([1.7, 2.3, 0.4])
    t = np.array([0.9, 3.1, 1.2])
    beam = np.stack([np.cos(2 * np.pi * s[f] * lm[:, 0]) * np.cos(2 * np.pi * t[f] * lm[:, 1])
                     for f in range(3)])
    bl = rng.uniform(-40.0, 40.0, size=(5, 2))
    uv = rng.uniform(-20.0, 20.0, size=(4, 2))
    Z = rng.standard_normal((3, 2)) + 1j * rng.standard_normal((3, 2))
    norm = 1.0 / (N * N)
    T = fm.forward_model(freq, bl, lm, beam, uv, Z, norm)
    for f in range(3):
        for b in range(5):
            du = uv[:, 0] - bl[b, 0] * freq[f] / fm.C_LIGHT
            dv = uv[:, 1] - bl[b, 1] * freq[f] / fm.C_LIGHT
            Sl = 0.5 * (_dirichlet(du + s[f], x) + _dirichlet(du - s[f], x))
            Sm = 0.5 * (_dirichlet(dv + t[f], x) + _dirichlet(dv - t[f], x))
            for e in range(2):
                got = T[f * 5 + b, e * 4:(e + 1) * 4]
                np.testing.assert_allclose(got, norm * Z[f, e] * Sl * Sm, rtol=1e-10, atol=1e-13)


def test_entry_function_agrees_with_the_matrix():
    rng = np.random.default_rng(13)
    lm = rng.uniform(-0.2, 0.2, size=(50, 2))
    freq = np.array([150e6, 155e6])
    bl = rng.uniform(-30, 30, size=(6, 2))
    beam = rng.uniform(0.1, 1.0, size=(2, 50))
    uv = rng.uniform(-10, 10, size=(5, 2))
    Z = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    T = fm.forward_model(freq, bl, lm, beam, uv, Z, 0.5)
    for row, col in [(0, 0), (7, 14), (11, 3), (5, 9)]:
        assert abs(fm.forward_model_entry(freq, bl, lm, beam, uv, Z, 0.5, row, col) - T[row, col]) <= 1e-12 * abs(T).max()
