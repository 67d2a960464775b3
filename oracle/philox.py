"""Counter-based normal variates for the sampler (oracle side).

Philox4x32 with 10 rounds, implemented from its published definition
(J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a 2-word key;
each round multiplies words 0 and 2 by two fixed odd constants, keeps the
64-bit products' high and low halves, and mixes the high halves with the
other two counter words and the round key; the key is bumped by two Weyl
constants between rounds.

Normals come from the Box-Muller transform, which the paper's CPU code uses
to make one pair of unit normals at a time (Sec. 3.2).  The uniforms are taken
from the top 24 bits of each 32-bit word, so they are exact in FP32 and both
implementations see bit-identical uniforms:
    u1 = ((x >> 8) + 1) * 2^-24  in (0, 1]
    u2 = (x >> 8) * 2^-24        in [0, 1)
    z0 = sqrt(-2 ln u1) cos(2 pi u2),  z1 = sqrt(-2 ln u1) sin(2 pi u2).

Stream layout (one Philox call per two elements):
    key     = (seed mod 2^32, seed >> 32)
    counter = (elem >> 1, sweep, (problem << 8) | stage, pair)
    words (x0, x1) -> (z0, z1) of element 2j, words (x2, x3) -> element 2j+1
where `elem` is the row-major index of a pixel (stage 0, messenger draw) or
of a Fourier mode in unshifted FFT order (stage 1, signal draw), stage 2
is the dispersed initial state, and stage 3 holds the chi-square variates of
the power-spectrum draw (elem = flat index over the bands' degrees of
freedom, sweep = the Gibbs iteration).  For a chain pair, z0 feeds chain 2*pair and
z1 chain 2*pair+1 (stage 0, 2) or the real and imaginary parts of the mode's
complex variate (stage 1).
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
ROUNDS = 10

STAGE_PIXEL = 0
STAGE_HARMONIC = 1
STAGE_INIT = 2
STAGE_SPECTRUM = 3


def philox4x32(ctr, key, rounds: int = ROUNDS):
    """Vectorised Philox4x32-R.  `ctr` is 4 integer arrays (broadcastable),
    `key` two integers.  Returns four uint64 arrays holding 32-bit words."""
    m = np.uint64(MASK32)
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & m for c in ctr)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(key[0]) & MASK32
    k1 = int(key[1]) & MASK32
    sh = np.uint64(32)
    for _ in range(rounds):
        p0 = c0 * np.uint64(PHILOX_M0)        # < 2^64, exact in uint64
        p1 = c2 * np.uint64(PHILOX_M1)
        n0 = (p1 >> sh) ^ c1 ^ np.uint64(k0)
        n1 = p1 & m
        n2 = (p0 >> sh) ^ c3 ^ np.uint64(k1)
        n3 = p0 & m
        c0, c1, c2, c3 = n0, n1, n2, n3
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return c0, c1, c2, c3


def philox4x32_scalar(ctr, key, rounds: int = ROUNDS):
    """The same function on plain Python integers (one counter)."""
    c = [int(x) & MASK32 for x in ctr]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for _ in range(rounds):
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & MASK32, p1 & MASK32,
             ((p0 >> 32) ^ c[3] ^ k1) & MASK32, p0 & MASK32]
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return tuple(c)


def uniforms(xa, xb):
    """The two uniforms of one Box-Muller pair (exact 24-bit values)."""
    xa = np.asarray(xa, dtype=np.uint64)
    xb = np.asarray(xb, dtype=np.uint64)
    u1 = ((xa >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
    u2 = (xb >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    return u1, u2


def box_muller(xa, xb):
    """Two independent unit normals from two 32-bit words (FP64)."""
    u1, u2 = uniforms(xa, xb)
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def split_seed(seed: int):
    seed = int(seed)
    if seed < 0 or seed >= 2 ** 64:
        raise ValueError("seed must fit in 64 bits")
    return seed & MASK32, (seed >> 32) & MASK32


def stream_normals(seed: int, stage: int, sweep: int, problem: int, pair: int,
                   n_elem: int):
    """(z0, z1), each float64 of length n_elem, for one chain pair."""
    if n_elem % 2:
        raise ValueError("the stream pairs elements, n_elem must be even")
    if not (0 <= problem < 2 ** 24 and 0 <= stage < 256):
        raise ValueError("problem must be < 2^24 and stage < 256")
    j = np.arange(n_elem // 2, dtype=np.uint64)
    ctr = (j, np.uint64(sweep & MASK32),
           np.uint64(((problem << 8) | stage) & MASK32), np.uint64(pair & MASK32))
    x0, x1, x2, x3 = philox4x32(ctr, split_seed(seed))
    ze0, ze1 = box_muller(x0, x1)
    zo0, zo1 = box_muller(x2, x3)
    z0 = np.empty(n_elem)
    z1 = np.empty(n_elem)
    z0[0::2], z0[1::2] = ze0, zo0
    z1[0::2], z1[1::2] = ze1, zo1
    return z0, z1


def stream_normals_scalar(seed: int, stage: int, sweep: int, problem: int,
                          pair: int, elem: int):
    """(z0, z1) of one element, by scalar code (for cross-checks)."""
    ctr = (elem >> 1, sweep, (problem << 8) | stage, pair)
    w = philox4x32_scalar(ctr, split_seed(seed))
    xa, xb = (w[0], w[1]) if elem % 2 == 0 else (w[2], w[3])
    u1 = ((xa >> 8) + 1) * 2.0 ** -24
    u2 = (xb >> 8) * 2.0 ** -24
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)
