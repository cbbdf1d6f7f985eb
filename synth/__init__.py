"""Seeded synthetic inputs shaped like the paper's likelihood workloads.

This module is the only code shared by the CPU oracle and the GPU path. It
draws random numbers and lays them out; it holds none of the likelihood's
arithmetic (no A, no d-bar, no Cholesky, no log-determinant).

Data model (statement of need: joint EoR + foreground coefficients seen through
a forward-modelled instrument; eq. 1: one power value per spherical k-shell):

    d = T a + e,   a ~ CN(0, Phi(theta*)),   e ~ CN(0, diag(sigma^2))

with T an m x n dense complex matrix, Phi diagonal with phi_j = s_b 10^theta_b
for an EoR coefficient j in k-bin b and a fixed variance for foreground
coefficients.

Draw order per config, from ``numpy.random.default_rng(1000 + config_id)``:
T, sigma^2, (bin map: no draw), a, e, theta batch.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

FG_VAR = 1.0e4  # fixed prior variance of every foreground coefficient


@dataclasses.dataclass
class Instance:
    """One dataset: instrument matrix, noise, data, bin map and theta batch."""

    T: np.ndarray          # complex128 (m, n), C-contiguous (row-major)
    noise_var: np.ndarray  # float64 (m,), > 0
    d: np.ndarray          # complex128 (m,)
    n_k: int
    bin_of: np.ndarray     # int32 (n,), -1 marks a fixed-variance coefficient
    fixed_var: np.ndarray  # float64 (n,), read where bin_of < 0
    bin_scale: np.ndarray  # float64 (n_k,), s_b (1 unless stated)
    theta: np.ndarray      # float64 (B, n_k), row-major
    theta_true: np.ndarray  # float64 (n_k,), the theta* the data were drawn at
    lo: float = -1.0       # prior box of theta
    hi: float = 3.0

    @property
    def m(self) -> int:
        return int(self.T.shape[0])

    @property
    def n(self) -> int:
        return int(self.T.shape[1])

    def digest(self) -> str:
        """SHA-256 over every array, in a fixed order."""
        h = hashlib.sha256()
        for a in (self.T, self.noise_var, self.d, self.bin_of, self.fixed_var,
                  self.bin_scale, self.theta, self.theta_true):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def balanced_bins(n_eor: int, n: int, n_k: int) -> np.ndarray:
    """Contiguous, balanced assignment of the first n_eor coefficients to
    n_k bins (b = floor(j n_k / n_eor)); the rest are foreground (-1)."""
    j = np.arange(n, dtype=np.int64)
    b = (j * n_k) // max(n_eor, 1)
    b[j >= n_eor] = -1
    return b.astype(np.int32)


def shell_bins(n_eor: int, n: int, n_k: int) -> np.ndarray:
    """Stress variant: bin b holds a share proportional to (b+1)^2 (shell
    volume growth), every bin at least one coefficient."""
    w = (np.arange(n_k) + 1.0) ** 2
    counts = np.maximum(1, np.floor(w / w.sum() * n_eor).astype(np.int64))
    counts[-1] += n_eor - counts.sum()
    if counts[-1] < 1:
        raise ValueError("n_eor too small for shell bins")
    b = np.repeat(np.arange(n_k), counts)
    out = np.full(n, -1, dtype=np.int32)
    out[:n_eor] = b
    return out


def _cn(rng: np.random.Generator, shape, var) -> np.ndarray:
    """Circular complex normal CN(0, var): real and imaginary parts i.i.d.
    N(0, var/2)."""
    z = rng.standard_normal(tuple(shape) + (2,))
    z = z.view(np.complex128).reshape(shape)
    return z * np.sqrt(np.asarray(var, dtype=np.float64) / 2.0)


def _matvec_rows(T: np.ndarray, a: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """T @ a by an elementwise product and numpy's pairwise row sum, in row
    chunks: no BLAS, so the rounding does not depend on the thread count."""
    out = np.empty(T.shape[0], dtype=np.complex128)
    for r0 in range(0, T.shape[0], chunk):
        out[r0:r0 + chunk] = (T[r0:r0 + chunk] * a[None, :]).sum(axis=1)
    return out


def make_instance(rng: np.random.Generator, m: int, n: int, n_k: int,
                  n_eor: int, n_theta: int, lo: float, hi: float,
                  theta_true=None, shells: bool = False,
                  T: np.ndarray | None = None, bin_of: np.ndarray | None = None) -> Instance:
    """Draw one instance in the fixed order T, sigma^2, a, e, theta."""
    if T is None:
        T = _cn(rng, (m, n), 1.0 / m)          # entries CN(0,1)/sqrt(m)
    noise_var = rng.uniform(0.5, 2.0, size=m)
    if bin_of is None:
        bin_of = shell_bins(n_eor, n, n_k) if shells else balanced_bins(n_eor, n, n_k)
    fixed_var = np.where(bin_of < 0, FG_VAR, 0.0).astype(np.float64)
    bin_scale = np.ones(n_k, dtype=np.float64)
    if theta_true is None:
        theta_true = np.linspace(0.5, 1.5, n_k)
    theta_true = np.asarray(theta_true, dtype=np.float64)
    phi = np.where(bin_of >= 0, 10.0 ** theta_true[np.maximum(bin_of, 0)], fixed_var)
    a = _cn(rng, (n,), phi)
    e = _cn(rng, (m,), noise_var)
    d = _matvec_rows(T, a) + e
    theta = rng.uniform(lo, hi, size=(n_theta, n_k))
    return Instance(T=np.ascontiguousarray(T), noise_var=noise_var, d=d,
                    n_k=n_k, bin_of=bin_of, fixed_var=fixed_var,
                    bin_scale=bin_scale, theta=np.ascontiguousarray(theta),
                    theta_true=theta_true, lo=lo, hi=hi)


# Workload shapes (paper's test dataset is not available; these stand in).
CONFIGS = {
    0: dict(m=480, n=200, n_k=3, n_eor=160, n_theta=64, lo=-1.0, hi=2.0,
            theta_true=(0.5, 1.0, 1.5)),
    1: dict(m=8000, n=2048, n_k=8, n_eor=1792, n_theta=256, lo=-1.0, hi=3.0),
    3: dict(m=20000, n=4096, n_k=12, n_eor=3584, n_theta=512, lo=-1.0, hi=3.0),
    4: dict(m=20000, n=4096, n_k=12, n_eor=3584, n_theta=0, lo=-1.0, hi=3.0),
}


def gen(config_id: int, seed: int | None = None, n_theta: int | None = None) -> Instance:
    """Instance for one of the fixed workloads (0, 1, 3, 4)."""
    cfg = dict(CONFIGS[config_id])
    if n_theta is not None:
        cfg["n_theta"] = n_theta
    rng = np.random.default_rng(1000 + config_id if seed is None else seed)
    return make_instance(rng, **cfg)


def gen_group(seed: int = 1002, n_inst: int = 48, n_lo: int = 256,
              n_hi: int = 4096, th_lo: int = 16, th_hi: int = 128,
              k_lo: int = 4, k_hi: int = 12, shapes_only: bool = False):
    """Uneven sub-band instances: n ~ U{n_lo..n_hi}, T (4n x n),
    n_theta ~ U{th_lo..th_hi}, n_k ~ U{k_lo..k_hi}, n_fg = n/8.

    Yields (n, n_theta, n_k) when shapes_only, else Instance objects, one at a
    time so a caller can upload and drop each before the next is drawn."""
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(n_lo, n_hi + 1)), int(rng.integers(th_lo, th_hi + 1)),
               int(rng.integers(k_lo, k_hi + 1))) for _ in range(n_inst)]
    if shapes_only:
        yield from shapes
        return
    for idx, (n, nth, nk) in enumerate(shapes):
        sub = np.random.default_rng([seed, idx])
        yield make_instance(sub, m=4 * n, n=n, n_k=nk, n_eor=n - n // 8,
                            n_theta=nth, lo=-1.0, hi=3.0)


def small(seed: int, m: int, n: int, n_k: int, n_eor: int | None = None,
          n_theta: int = 8, lo: float = -1.0, hi: float = 3.0,
          shells: bool = False) -> Instance:
    """Small instance of any shape for tests."""
    rng = np.random.default_rng(seed)
    return make_instance(rng, m=m, n=n, n_k=n_k,
                         n_eor=n - n // 8 if n_eor is None else n_eor,
                         n_theta=n_theta, lo=lo, hi=hi, shells=shells)


def stress_T(rng: np.random.Generator, m: int, n: int, decades: float = 4.0) -> np.ndarray:
    """Ill-conditioned instrument matrix T = G diag(s): the columns of a
    complex Gaussian G (entries CN(0, 1/m), so every column has norm about 1
    and G's own condition number is about (1 + sqrt(n/m)) / (1 - sqrt(n/m)))
    scaled by s log-spaced over `decades` decades, so that T's singular
    values spread over about as many. Elementwise arithmetic only: the same
    bits on any host (a QR or a matrix product would round differently
    with the host's BLAS)."""
    s = np.logspace(0.0, -decades, n)
    return np.ascontiguousarray(_cn(rng, (m, n), 1.0 / m) * s[None, :])


def stress(seed: int, m: int, n: int, n_k: int, n_eor: int | None = None, n_theta: int = 8,
           lo: float = -1.0, hi: float = 3.0, decades: float = 4.0) -> Instance:
    """Instance with the ill-conditioned instrument matrix of stress_T."""
    rng = np.random.default_rng(seed)
    T = stress_T(rng, m, n, decades)
    return make_instance(rng, m=m, n=n, n_k=n_k,
                         n_eor=n - n // 8 if n_eor is None else n_eor,
                         n_theta=n_theta, lo=lo, hi=hi, T=T)


# Stress workloads at the plain-batched sizes (reported, not a metric):
# singular values of T over four decades, and a wide-field foreground model
# with many more foreground than EoR coefficients on the same T.
STRESS = {
    "svd4": dict(m=8000, n=2048, n_k=8, n_eor=1792, n_theta=256, decades=4.0),
    "widefg": dict(m=8000, n=2048, n_k=8, n_eor=256, n_theta=256, decades=4.0),
}


def gen_stress(name: str, seed: int | None = None) -> Instance:
    cfg = dict(STRESS[name])
    base = 2000 + sorted(STRESS).index(name)
    return stress(base if seed is None else seed, **cfg)


def theta_batch(rng: np.random.Generator, B: int, n_k: int, lo: float, hi: float) -> np.ndarray:
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(B, n_k)))


# ---------------------------------------------------------------------------
# Synthetic instrument: the inputs of the forward model that builds T from a
# primary beam, the uv sampling and the model's Fourier basis. These are
# tables of the instrument and of the basis functions; the sum over pixels
# that turns them into T is not here.

C_LIGHT = 299792458.0


@dataclasses.dataclass
class Instrument:
    freq: np.ndarray      # float64 (F,), Hz
    bl: np.ndarray        # float64 (n_bl, 2), baseline east/north in metres
    lm: np.ndarray        # float64 (n_pix, 2), direction cosines of the sky pixels
    beam: np.ndarray      # float64 (F, n_pix), primary-beam response
    uv: np.ndarray        # float64 (n_uv, 2), model Fourier cells in wavelengths
    Z: np.ndarray         # complex128 (F, n_eta), spectral modes (foreground first)
    norm: float
    bin_of: np.ndarray    # int32 (n_eta n_uv,), k-shell of each coefficient, -1 for foreground modes
    n_k: int
    k_shell: np.ndarray   # float64 (n_k,), mean |(i_x, i_y, j)| of each shell's coefficients (lattice units)

    @property
    def m(self) -> int:
        return int(self.freq.size * self.bl.shape[0])

    @property
    def n(self) -> int:
        return int(self.Z.shape[1] * self.uv.shape[0])


def instrument(seed: int, F: int = 32, n_bl: int = 625, n_side: int = 64, kx: int = 16, ky: int = 8,
               n_fg: int = 4, n_eor_eta: int = 28, n_k: int = 12, nu0: float = 150e6,
               dnu: float = 100e3, dish: float = 14.0, fov: float = 0.3) -> Instrument:
    """Drawn from numpy.random.default_rng(seed): baselines uniform in a
    disc of radius 60 m (at least 14.6 m long). Fixed: channels nu0 + f dnu;
    an n_side x n_side pixel grid over a field of view `fov` (radians) centred
    on the pointing; a Gaussian primary beam of FWHM 1.03 lambda / dish; model
    cells on the grid's Fourier lattice, kx x ky cells around uv = 0; spectral
    modes: Legendre polynomials of degree 0..n_fg-1 over the band (foreground)
    and exp(2 pi i j f / F) for j = +-1 .. +-n_eor_eta/2 (EoR); norm 1/n_pix.
    EoR coefficients fall into n_k spherical shells of sqrt(ix^2 + iy^2 + j^2)
    with equal counts (ties kept together)."""
    rng = np.random.default_rng(seed)
    r = np.sqrt(rng.uniform((14.6 / 60.0) ** 2, 1.0, size=n_bl)) * 60.0
    ang = rng.uniform(0.0, 2.0 * np.pi, size=n_bl)
    bl = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    freq = nu0 + dnu * np.arange(F, dtype=np.float64)
    delta = fov / n_side
    x = (np.arange(n_side) - n_side // 2) * delta
    L, M = np.meshgrid(x, x, indexing="xy")
    lm = np.stack([L.ravel(), M.ravel()], axis=1)
    sigma = 1.03 * (C_LIGHT / freq) / dish / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    beam = np.exp(-(lm[None, :, 0] ** 2 + lm[None, :, 1] ** 2) / (2.0 * sigma[:, None] ** 2))
    du = 1.0 / (n_side * delta)
    ix, iy = np.meshgrid(np.arange(kx) - kx // 2, np.arange(ky) - ky // 2, indexing="ij")
    ix, iy = ix.ravel(), iy.ravel()
    uv = np.stack([ix * du, iy * du], axis=1).astype(np.float64)
    xf = 2.0 * np.arange(F) / max(F - 1, 1) - 1.0
    fg = np.stack([np.polynomial.legendre.legval(xf, np.eye(n_fg)[d]) for d in range(n_fg)], axis=1)
    js = np.concatenate([-np.arange(n_eor_eta // 2, 0, -1), np.arange(1, n_eor_eta // 2 + 1)])
    eor = np.exp(2j * np.pi * np.outer(np.arange(F), js) / F)
    Z = np.concatenate([fg.astype(np.complex128), eor], axis=1)
    n_uv = uv.shape[0]
    kk = np.sqrt(ix[None, :] ** 2 + iy[None, :] ** 2 + js[:, None] ** 2).ravel()  # EoR coefficients, mode-major
    order = np.argsort(kk, kind="stable")
    shell = np.empty(kk.size, dtype=np.int64)
    shell[order] = (np.arange(kk.size) * n_k) // kk.size
    # ties kept together: every coefficient takes the shell of the first with its |k|
    first = {}
    for idx in order:
        first.setdefault(kk[idx], shell[idx])
    shell = np.array([first[v] for v in kk], dtype=np.int64)
    bin_of = np.concatenate([np.full(n_fg * n_uv, -1, dtype=np.int64), shell]).astype(np.int32)
    used = np.unique(shell)
    remap = {b: i for i, b in enumerate(used)}
    bin_of = np.array([remap[b] if b >= 0 else -1 for b in bin_of], dtype=np.int32)
    eor_bins = bin_of[n_fg * n_uv:]
    k_shell = np.array([kk[eor_bins == b].mean() for b in range(used.size)])
    return Instrument(freq=freq, bl=bl, lm=np.ascontiguousarray(lm), beam=np.ascontiguousarray(beam),
                      uv=uv, Z=np.ascontiguousarray(Z), norm=1.0 / lm.shape[0], bin_of=bin_of,
                      n_k=int(used.size), k_shell=k_shell)


def instrument_instance(ins: Instrument, T: np.ndarray, seed: int, n_theta: int, lo: float = -1.0,
                        hi: float = 3.0) -> Instance:
    """Noise, data and theta batch for the forward-modelled T (drawn in the
    same order as make_instance), with the instrument's k-shells."""
    rng = np.random.default_rng(seed)
    inst = make_instance(rng, m=T.shape[0], n=T.shape[1], n_k=ins.n_k, n_eor=1, n_theta=n_theta, lo=lo, hi=hi,
                         T=T, bin_of=ins.bin_of)
    return inst
