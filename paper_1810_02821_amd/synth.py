"""Seeded synthetic inputs for the messenger-field method.

This module only *generates data*: a true signal drawn as a periodic Gaussian
random field, a heteroscedastic diagonal noise map, a mask of missing pixels
and the data vector d = s + n (the linear model of Sec. 1.1, Eq. 1, with
A = I).  It contains none of the messenger method's arithmetic; both the
CPU oracle and the GPU library receive the arrays it returns.

Conventions fixed here and used by both sides:

* wavenumbers are integer grid indices k_x, k_y in numpy ``fftfreq * N``
  order and |k| = sqrt(k_x^2 + k_y^2) ("grid units");
* the power spectrum is in the *synthesis* convention,
  s_x = sum_k s_k exp(+2 pi i k.x / N) with <|s_k|^2> = P(|k|)
  (the reading of Eq. 8-9 adopted by this project, see the design notes);
  the field is made as ifft2(sqrt(n P) * fft2(white)), so that modes that are
  not self-conjugate get real and imaginary parts of variance P/2 each and the
  Hermitian symmetry s_k^* = s_{-k} holds, as Sec. 3.2 prescribes;
* masked pixels carry noise variance +inf (the infinite-noise rule of Sec. 1.1)
  and data value 0;
* masks are made of grid-aligned 4x4 tiles, drawn without replacement.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

__all__ = [
    "Spectrum", "Problem", "spectrum_powerlaw", "spectrum_bands",
    "log_band_edges", "grf", "tile_mask", "make_problem",
    "config_small", "config_128", "config_uneven", "config_bands",
    "config_large", "philox_seed",
]


@dataclasses.dataclass
class Spectrum:
    """Isotropic power spectrum P(|k|) (Eq. 9).

    kind == "powerlaw": P(k) = amp * (k + k0) ** (-n)
    kind == "bands":    P(k) = amps[b] for edges[b] <= k < edges[b+1]
                        (the last band also includes k == edges[-1]).
    """
    kind: str
    amp: float = 1.0
    k0: float = 1.0
    n: float = 2.0
    edges: Optional[np.ndarray] = None
    amps: Optional[np.ndarray] = None

    def evaluate(self, kmag: np.ndarray) -> np.ndarray:
        """P(|k|) for synthesis of the true field (generator's own copy)."""
        if self.kind == "powerlaw":
            return self.amp * (kmag + self.k0) ** (-self.n)
        if self.kind == "bands":
            idx = np.searchsorted(self.edges, kmag, side="right") - 1
            idx = np.clip(idx, 0, len(self.amps) - 1)
            return np.asarray(self.amps, dtype=np.float64)[idx]
        raise ValueError(f"unknown spectrum kind {self.kind!r}")


def spectrum_powerlaw(amp: float = 1.0, k0: float = 1.0, n: float = 2.0) -> Spectrum:
    return Spectrum(kind="powerlaw", amp=float(amp), k0=float(k0), n=float(n))


def spectrum_bands(edges: Sequence[float], amps: Sequence[float]) -> Spectrum:
    edges = np.asarray(edges, dtype=np.float64)
    amps = np.asarray(amps, dtype=np.float64)
    if edges.ndim != 1 or amps.ndim != 1 or len(edges) != len(amps) + 1:
        raise ValueError("bands need len(edges) == len(amps) + 1")
    return Spectrum(kind="bands", edges=edges, amps=amps)


def log_band_edges(H: int, W: int, n_bands: int = 32) -> np.ndarray:
    """Band edges: 0, then n_bands log-spaced edges from 1 to k_max.

    k_max = sqrt((H/2)^2 + (W/2)^2) is the largest |k| on the grid, so every
    mode falls in some band; band 0 holds only k = 0.
    """
    kmax = math.hypot(H / 2.0, W / 2.0)
    e = [0.0] + [kmax ** ((b - 1) / (n_bands - 1)) for b in range(1, n_bands + 1)]
    return np.asarray(e, dtype=np.float64)


def _kmag(H: int, W: int) -> np.ndarray:
    ky = np.fft.fftfreq(H) * H
    kx = np.fft.fftfreq(W) * W
    return np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)


def grf(H: int, W: int, spectrum: Spectrum, rng: np.random.Generator) -> np.ndarray:
    """Real periodic Gaussian random field with synthesis spectrum P (Sec. 3.2)."""
    n = H * W
    amp = np.sqrt(n * spectrum.evaluate(_kmag(H, W)))
    white = rng.standard_normal((H, W))
    return np.fft.ifft2(amp * np.fft.fft2(white)).real


def tile_mask(H: int, W: int, frac: float, rng: np.random.Generator,
              tile: int = 4) -> np.ndarray:
    """Boolean mask (True = missing) of round(frac * #tiles) aligned tiles
    (sides that are not multiples of the tile end in partial tiles)."""
    th, tw = -(-H // tile), -(-W // tile)
    n_tiles = th * tw
    k = int(round(frac * n_tiles))
    chosen = rng.permutation(n_tiles)[:k]
    m = np.zeros((th, tw), dtype=bool)
    m.flat[chosen] = True
    return np.repeat(np.repeat(m, tile, axis=0), tile, axis=1)[:H, :W]


@dataclasses.dataclass
class Problem:
    """One image problem: data, diagonal noise variance, mask and spectrum."""
    H: int
    W: int
    d: np.ndarray            # float64 (H, W), 0 on masked pixels
    noise_var: np.ndarray    # float64 (H, W), +inf on masked pixels
    mask: np.ndarray         # bool (H, W), True = missing
    spectrum: Spectrum
    s_true: np.ndarray       # float64 (H, W), the generating field
    response: Optional[np.ndarray] = None  # float64 (H, W) diagonal A of d = A s + n, None = identity
    gamma: Optional[np.ndarray] = None     # complex128 (H, W) shear data of a mass-mapping problem

    @property
    def n(self) -> int:
        return self.H * self.W


def make_problem(H: int, W: int, spectrum: Spectrum, sigma: np.ndarray,
                 mask: np.ndarray, rng: np.random.Generator) -> Problem:
    s = grf(H, W, spectrum, rng)
    noise = sigma * rng.standard_normal((H, W))
    d = np.where(mask, 0.0, s + noise)
    nv = np.where(mask, np.inf, sigma ** 2)
    return Problem(H=H, W=W, d=d, noise_var=nv, mask=mask.copy(),
                   spectrum=spectrum, s_true=s)


def config_response(seed: int = 0, size: int = 128, dead: float = 0.01) -> Problem:
    """The paper-size recipe seen through a diagonal instrument response:
    d = A s + n with A_i ~ U[0.5, 1.5] (gain / exposure variation), a fraction
    `dead` of pixels with A_i = 0 (no response), and 25% masked 4x4 tiles."""
    rng = np.random.default_rng(seed)
    spec = spectrum_powerlaw(1.0, 2.0, 2.5)
    sigma = _uniform_sigma(size, size, 0.3, 3.0, rng)
    mask = tile_mask(size, size, 0.25, rng)
    A = rng.uniform(0.5, 1.5, size=(size, size))
    A[rng.random((size, size)) < dead] = 0.0
    s = grf(size, size, spec, rng)
    noise = sigma * rng.standard_normal((size, size))
    missing = mask | (A == 0.0)
    d = np.where(missing, 0.0, A * s + noise)
    nv = np.where(mask, np.inf, sigma ** 2)
    return Problem(H=size, W=size, d=d, noise_var=nv, mask=missing, spectrum=spec, s_true=s, response=A)


def shear_from_convergence(kappa: np.ndarray) -> np.ndarray:
    """The weak-lensing shear of a convergence map (Kaiser & Squires 1993):
    gamma_hat = (k_1 + i k_2)^2 / |k|^2 kappa_hat, with no shear from k = 0."""
    H, W = kappa.shape
    ky = (np.fft.fftfreq(H) * H)[:, None]
    kx = (np.fft.fftfreq(W) * W)[None, :]
    k2 = kx * kx + ky * ky
    k2[0, 0] = 1.0
    kernel = (kx + 1j * ky) ** 2 / k2
    kernel[0, 0] = 0.0
    return np.fft.ifft2(kernel * np.fft.fft2(kappa))


def config_shear(seed: int = 0, size: int = 128, b_ratio: float = 0.0, width: Optional[int] = None) -> Problem:
    """Mass mapping: convergence kappa = kappa_E + i kappa_B with
    P_E = (k+1)^-2 and P_B = b_ratio P_E, shear gamma = A kappa + n with
    sigma ~ U[0.3, 1.0] per component, 20% masked 4x4 tiles.  `spectrum` is P_E.
    size x size, or size x width."""
    rng = np.random.default_rng(seed)
    H, W = size, (size if width is None else width)
    spec = spectrum_powerlaw(1.0, 1.0, 2.0)
    sigma = _uniform_sigma(H, W, 0.3, 1.0, rng)
    mask = tile_mask(H, W, 0.20, rng)
    kE = grf(H, W, spec, rng)
    kB = np.sqrt(b_ratio) * grf(H, W, spec, rng) if b_ratio > 0 else np.zeros((H, W))
    kappa = kE + 1j * kB
    noise = sigma * (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W)))
    g = np.where(mask, 0.0, shear_from_convergence(kappa) + noise)
    nv = np.where(mask, np.inf, sigma ** 2)
    return Problem(H=H, W=W, d=np.zeros((H, W)), noise_var=nv, mask=mask, spectrum=spec,
                   s_true=kE, gamma=g)


def philox_seed(data_seed: int) -> int:
    """Seed of the sampler's random stream for a given data seed."""
    return int(data_seed) + 1000


# --------------------------------------------------------------------------
# Workload recipes (the paper's self-simulated data of Sec. 3.2 / Fig. 2,
# at the sizes this project measures).
# --------------------------------------------------------------------------

def _uniform_sigma(H, W, lo, hi, rng):
    return rng.uniform(lo, hi, size=(H, W))


def config_small(seed: int = 0, size: int = 32) -> Problem:
    """32x32, P=(k+1)^-2, sigma~U[0.5,2], 20% masked in 4x4 tiles."""
    rng = np.random.default_rng(seed)
    spec = spectrum_powerlaw(1.0, 1.0, 2.0)
    sigma = _uniform_sigma(size, size, 0.5, 2.0, rng)
    mask = tile_mask(size, size, 0.20, rng)
    return make_problem(size, size, spec, sigma, mask, rng)


def config_128(seed: int = 0, size: int = 128) -> Problem:
    """128x128 (the paper's image size), P=(k+2)^-2.5, sigma~U[0.3,3], 25% tiles."""
    rng = np.random.default_rng(seed)
    spec = spectrum_powerlaw(1.0, 2.0, 2.5)
    sigma = _uniform_sigma(size, size, 0.3, 3.0, rng)
    mask = tile_mask(size, size, 0.25, rng)
    return make_problem(size, size, spec, sigma, mask, rng)


def config_uneven(seed: int = 0, n_problems: int = 4096,
                  sizes: Sequence[int] = (64, 128, 256, 512),
                  weights: Sequence[float] = (0.4, 0.3, 0.2, 0.1)) -> List[Problem]:
    """Uneven batch: sizes drawn from `sizes` at `weights`, per-problem spectra."""
    rng = np.random.default_rng(seed)
    picks = rng.choice(len(sizes), size=n_problems, p=np.asarray(weights) / np.sum(weights))
    out = []
    for i in range(n_problems):
        N = int(sizes[picks[i]])
        k0 = rng.uniform(0.5, 4.0)
        nn = rng.uniform(1.5, 3.5)
        spec = spectrum_powerlaw(1.0, k0, nn)
        sigma = _uniform_sigma(N, N, 0.2, 4.0, rng)
        mask = tile_mask(N, N, rng.uniform(0.0, 0.4), rng)
        out.append(make_problem(N, N, spec, sigma, mask, rng))
    return out


def bands_from_powerlaw(H: int, W: int, n_bands: int, k0: float, n: float) -> Spectrum:
    """Log bands (log_band_edges) with amplitude (k + k0)^-n at the mean |k|
    of the modes in each band (the band midpoint for an empty band)."""
    edges = log_band_edges(H, W, n_bands)
    km = _kmag(H, W)
    idx = np.clip(np.searchsorted(edges, km, side="right") - 1, 0, n_bands - 1)
    amps = np.empty(n_bands)
    for b in range(n_bands):
        sel = km[idx == b]
        kc = sel.mean() if sel.size else 0.5 * (edges[b] + edges[b + 1])
        amps[b] = (kc + k0) ** (-n)
    return spectrum_bands(edges, amps)


def config_bands(seed: int = 0, size: int = 256, n_bands: int = 32, width: Optional[int] = None) -> Problem:
    """Band-amplitude spectrum for differentiation: 32 log bands seeded from
    P(k)=(k+1)^-2 at the mean |k| of each band, times U[0.8,1.2];
    sigma~U[0.5,2]; 30% masked tiles.  size x size, or size x width."""
    rng = np.random.default_rng(seed)
    H, W = size, (size if width is None else width)
    base = bands_from_powerlaw(H, W, n_bands, 1.0, 2.0)
    spec = spectrum_bands(base.edges, base.amps * rng.uniform(0.8, 1.2, size=n_bands))
    sigma = _uniform_sigma(H, W, 0.5, 2.0, rng)
    mask = tile_mask(H, W, 0.30, rng)
    return make_problem(H, W, spec, sigma, mask, rng)


def config_large(seed: int = 0, size: int = 2048, n_bands: int = 0) -> Problem:
    """Large map: P=(k+1)^-2.2; sigma = 2^(cos(2 pi x/N) cos(2 pi y/N)) in
    [0.5, 2]; observed central disk of radius 0.45 N (outside masked) with
    random radius-3 holes until 5% of the disk is masked.  n_bands > 0 gives
    the spectrum as that many log bands of the same power law (for gradients
    with respect to band amplitudes)."""
    rng = np.random.default_rng(seed)
    N = size
    spec = (bands_from_powerlaw(N, N, n_bands, 1.0, 2.2) if n_bands > 0
            else spectrum_powerlaw(1.0, 1.0, 2.2))
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    sigma = 2.0 ** (np.cos(2 * np.pi * x / N) * np.cos(2 * np.pi * y / N))
    c = (N - 1) / 2.0
    r2 = (x - c) ** 2 + (y - c) ** 2
    disk = r2 <= (0.45 * N) ** 2
    mask = ~disk
    target = 0.05 * disk.sum()
    holes = np.zeros_like(mask)
    R = 3
    dy, dx = np.mgrid[-R:R + 1, -R:R + 1]
    stamp = (dy ** 2 + dx ** 2) <= R * R
    disk_idx = np.flatnonzero(disk)
    count = 0
    while count < target:
        centres = rng.choice(disk_idx, size=256)
        for cidx in centres:
            cy, cx = divmod(int(cidx), N)
            ys = (cy + dy[stamp]) % N
            xs = (cx + dx[stamp]) % N
            new = disk[ys, xs] & ~holes[ys, xs]
            holes[ys[new], xs[new]] = True
            count += int(new.sum())
            if count >= target:
                break
    mask = mask | holes
    return make_problem(N, N, spec, sigma, mask, rng)
