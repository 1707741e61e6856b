"""Philox4x64-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with the
multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157, a word permutation and
a key xor, with the Weyl key bump (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
between rounds.

Vectorised over counters with numpy uint64; the 128-bit products are formed
from 32-bit halves.

The per-trajectory draw of the sampler: key (seed, 0), counter (s, 0, 0, 0)
for trajectory s; the top 24 bits of output words 0 and 1 scaled by 2^-24 give
two uniforms in [0, 1) that are exact in float32 and float64.
"""
import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.uint64, b: np.ndarray):
    """(hi, lo) words of the 128-bit product a*b, elementwise."""
    b = b.astype(np.uint64)
    a0 = a & _LO32
    a1 = a >> _S32
    b0 = b & _LO32
    b1 = b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(counter, key):
    """counter: 4 arrays (or scalars) of uint64; key: 2 uint64 scalars or
    arrays.  Returns the 4 output words as uint64 arrays."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = [np.asarray(c, dtype=np.uint64) for c in counter]
        k0, k1 = [np.asarray(k, dtype=np.uint64) for k in key]
        for r in range(10):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, c0)
            hi1, lo1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def trajectory_uniforms(seed: int, sample_ids: np.ndarray):
    """Two 24-bit uniforms per trajectory (float64, exact)."""
    s = np.asarray(sample_ids, dtype=np.uint64)
    z = np.zeros_like(s)
    out = philox4x64_10((s, z, z, z), (np.uint64(seed), np.uint64(0)))
    u1 = (out[0] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    u2 = (out[1] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    return u1, u2
