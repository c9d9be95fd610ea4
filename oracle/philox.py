"""Philox4x64-10 counter-based generator (test infrastructure).

The paper does not say how its random numbers are drawn; the sampler here draws every random
number from Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11), written from that paper's definition: ten rounds of
  (hi0, lo0) = mulhilo(M0, x0); (hi1, lo1) = mulhilo(M1, x2);
  x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
with the key bumped by the Weyl constants (W0, W1) between rounds.

Counter layout used by the sampler: (index, slice, sweep, tag); key = (seed, 0).
tag PATH: index = particle, one uniform per (particle, slice, sweep) for backward sampling.
tag GIBBS: index = site, one draw per (site, slice, sweep) for the field update.

Integer to float conversions:
  uniform in [0,1):  (x0 >> 11) * 2^-53
  Gaussian:          u1 = ((x0 >> 11) + 1) * 2^-53 in (0,1], u2 = (x1 >> 11) * 2^-53,
                     z = sqrt(-2 log u1) * cos(2 pi u2)            (Box-Muller)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

TAG_PATH = 0
TAG_GIBBS = 1

TWO_PI = 6.283185307179586  # the double nearest 2*pi
INV_2_53 = 1.0 / 9007199254740992.0


def _mulhilo(a: np.ndarray, m: np.uint64):
    """(hi, lo) 64-bit halves of the 128-bit product a*m, from 32-bit partial products."""
    a0 = a & _M32
    a1 = a >> _S32
    m0 = m & _M32
    m1 = m >> _S32
    p00 = a0 * m0
    p01 = a0 * m1
    p10 = a1 * m0
    p11 = a1 * m1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * m  # wraps modulo 2^64
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Vectorised Philox4x64: counters and keys broadcast as uint64 arrays; returns 4 arrays."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        x0, x1, x2, x3 = (v.copy() for v in (x0, x1, x2, x3))
        k0 = np.asarray(k0, dtype=np.uint64) + np.zeros_like(x0)
        k1 = np.asarray(k1, dtype=np.uint64) + np.zeros_like(x0)
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + W0
            k1 = k1 + W1
    return x0, x1, x2, x3


def uniform(x0: np.ndarray) -> np.ndarray:
    """53-bit uniform in [0, 1)."""
    return (x0 >> np.uint64(11)).astype(np.float64) * INV_2_53


def gaussian(x0: np.ndarray, x1: np.ndarray) -> np.ndarray:
    """Box-Muller standard normal from two 64-bit words."""
    u1 = ((x0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * INV_2_53
    u2 = (x1 >> np.uint64(11)).astype(np.float64) * INV_2_53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(TWO_PI * u2)


def draw_words(seed: int, index, slc, sweep, tag):
    return philox4x64(index, slc, sweep, tag, np.uint64(seed), np.uint64(0))


def path_uniforms(seed: int, particles: np.ndarray, slc: int, sweep: int) -> np.ndarray:
    x0, _, _, _ = draw_words(seed, particles, slc, sweep, TAG_PATH)
    return uniform(x0)
