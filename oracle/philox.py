"""Philox4x64-10 counter-based generator and the sampler's uniform (oracle side).

Test infrastructure only: this module belongs to the FP64 oracle and is used
by the tests and the CPU-baseline leg of the benchmark, never by the product
path.

The paper draws one uniform threshold per sample at every measurement
(Section 3.3.1, Algorithm 1: ``threshold = repeat(rand(N2), d)``) but names no
generator.  Reading taken: one FP64 uniform per (chain, sample, site) from
Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written here from that published
definition:

* state: four 64-bit counter words and two 64-bit key words;
* round: (hi0, lo0) = M0 * x0 and (hi1, lo1) = M1 * x2 as full 128-bit
  products; the new words are (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0);
* before every round after the first the key is bumped by the Weyl
  constants W0, W1 (mod 2^64).

key = (seed, mps_id), counter = (n, k, 0, 0) with n the global sample index
and k the site, first output word x0, u = ((x0 >> 12) + 0.5) * 2^-52, which
lies in the open interval (0, 1): every step is exact in FP64, the smallest
value is 2^-53 and the largest 1 - 2^-53.  (With 53 bits, (2^53 - 1) + 0.5 is
not representable and rounds up to 2^53, so that mapping can return 1.0.)
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B


def philox4x64(ctr: tuple[int, int, int, int], key: tuple[int, int], rounds: int = 10):
    """Scalar Philox4x64-R on Python integers (the definition, unoptimised)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
    return x0, x1, x2, x3


def _mulhilo(a: np.ndarray, b: int):
    """Full 64x64 -> 128-bit product on uint64 arrays, via 32-bit limbs."""
    lo32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    b = np.uint64(b)
    a0, a1 = a & lo32, a >> s32
    b0, b1 = b & lo32, b >> s32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> s32) + (p01 & lo32) + (p10 & lo32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    lo = a * b  # wraps mod 2^64
    return hi, lo


def philox4x64_np(c0, c1, c2, c3, k0: int, k1: int, rounds: int = 10):
    """Vectorised Philox4x64-R over uint64 counter arrays (same definition)."""
    x0 = np.asarray(c0, dtype=np.uint64).copy()
    x1 = np.asarray(c1, dtype=np.uint64).copy()
    x2 = np.asarray(c2, dtype=np.uint64).copy()
    x3 = np.asarray(c3, dtype=np.uint64).copy()
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    x0, x1, x2, x3 = (x.copy() for x in (x0, x1, x2, x3))
    k0 = int(k0) & MASK64
    k1 = int(k1) & MASK64
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = (k0 + W0) & MASK64
                k1 = (k1 + W1) & MASK64
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
    return x0, x1, x2, x3


def bits_to_uniform(x) -> np.ndarray:
    """u = ((x >> 12) + 0.5) * 2^-52 in FP64; never 0 or 1."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def uniforms(seed: int, mps_id: int, n, k) -> np.ndarray:
    """U(seed, mps_id, n, k) for broadcastable arrays of sample index n and site k."""
    n = np.asarray(n, dtype=np.uint64)
    k = np.asarray(k, dtype=np.uint64)
    n, k = np.broadcast_arrays(n, k)
    z = np.zeros(n.shape, dtype=np.uint64)
    x0, _, _, _ = philox4x64_np(n, k, z, z, seed, mps_id)
    return bits_to_uniform(x0)
