"""Reduced-precision storage of the streamed field (FP64 CPU; test infrastructure).

Sec. 3.2 weighs the bit width of the arithmetic against the resources of the
dataflow engine.  The GPU analogue here keeps FP32 arithmetic but stores the
chain-pair field in HBM as 16-bit pairs (IEEE binary16 or bfloat16) between
the two kernels of a streamed sweep.  This module defines what that computes:
Algorithm 1 as in ``messenger``, with each 2D transform split into its row
and column passes (fft2(x) = fft(fft(x, axis=1), axis=0)) and the field
rounded to the nearest representable value, ties to even, wherever it is
stored:

  s      = round(s0)                                    (the start state)
  per sweep:
  t      = (1 - a) s + T b + sigma_t xi                 (pixel step)
  u      = round(fft(t, axis=1))                        (row transforms, stored)
  S_hat  = f fft(u, axis=0) + w eta                     (column transforms, Fourier step)
  v      = round(ifft(S_hat, axis=0) / W)               (inverse column transforms, stored)
  s      = W ifft(v, axis=1)                            (inverse row transforms)

Without rounding this is exactly ``messenger.sweep`` (the stored v carries the
1/W that the unnormalised inverse row pass undoes; rounding commutes with the
power-of-two scale away from underflow and overflow).  Samples are the s of a
sweep, before any rounding; the state a call returns is round(s) of its last
sweep.  Real and imaginary parts round independently.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import messenger, philox


def round_fp16(x: np.ndarray) -> np.ndarray:
    """Nearest binary16 value of each real and imaginary part (numpy's
    float16 conversion rounds to nearest even, with subnormals)."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return round_fp16(x.real) + 1j * round_fp16(x.imag)
    with np.errstate(over="ignore"):  # beyond 65504: inf, as the hardware conversion gives
        return x.astype(np.float16).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 value (8 significand bits, FP32 exponent range) of
    each real and imaginary part: the value is first rounded to FP32 (where
    the GPU holds it), then its 32-bit pattern is rounded to the upper 16
    bits, ties to even."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return round_bf16(x.real) + 1j * round_bf16(x.imag)
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


ROUNDERS = {"fp32": None, "fp16": round_fp16, "bf16": round_bf16}


def stored_sweep(s, b, c: messenger.Coefficients, rnd, xi=None, eta=None):
    """One sweep with the field rounded where the streamed kernels store it.
    Returns the new state s (unrounded)."""
    W = s.shape[1]
    t = messenger.pixel_step(s, b, c, xi)
    u = rnd(np.fft.fft(t, axis=1))
    s_hat = messenger.harmonic_step(np.fft.fft(u, axis=0), c, eta)
    v = rnd(np.fft.ifft(s_hat, axis=0) / W)
    return W * np.fft.ifft(v, axis=1)


def sample_pair_stored(problem, seed: int, problem_index: int, pair: int, burn_in: int, n_samples: int,
                       thin: int = 1, storage: str = "fp16", s0: Optional[np.ndarray] = None,
                       sweep_offset: int = 0):
    """``messenger.sample_pair`` with the field stored as `storage` between
    the kernels.  Returns (samples [2, n_samples, H, W], returned state)."""
    rnd = ROUNDERS[storage] or (lambda x: x)
    H, W = problem.H, problem.W
    c = messenger.coefficients(problem.noise_var, problem.spectrum, 1.0, None, messenger.response_of(problem))
    d = np.where(problem.mask, 0.0, problem.d)
    b = c.ninv * d
    s = np.zeros((H, W), dtype=np.complex128) if s0 is None else np.array(s0, dtype=np.complex128)
    s = rnd(s)
    out = np.empty((2, n_samples, H, W))
    emitted = 0
    for k in range(burn_in + n_samples * thin):
        g = sweep_offset + k
        xi = messenger.pair_normals(seed, philox.STAGE_PIXEL, g, problem_index, pair, H, W)
        eta = messenger.pair_normals(seed, philox.STAGE_HARMONIC, g, problem_index, pair, H, W)
        s = stored_sweep(s, b, c, rnd, xi, eta)
        if k >= burn_in and (k - burn_in + 1) % thin == 0:
            out[0, emitted] = s.real
            out[1, emitted] = s.imag
            emitted += 1
    return out, rnd(s)
