"""Counter-based start block X0 ~ N(0,1) (oracle; test infrastructure).

Algorithm 3 opens with a random block X; a solve given no start block draws
it on the device.  This is an independent host implementation of the same
generator, written from its published definition, so that the device block
can be compared entry by entry:

  Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011, section 4): ten rounds on a counter of four
  32-bit words (c0, c1, c2, c3) under a key (k0, k1).  One round forms the
  two 64-bit products M0 c0 and M1 c2 (M0 = 0xD2511F53, M1 = 0xCD9E8D57) and
  outputs (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
  after each round the key is bumped by the Weyl constants (0x9E3779B9,
  0xBB67AE85) modulo 2^32.

Entry (i, j) of the block uses counter (i mod 2^32, j, i div 2^32, 0) and key
(seed mod 2^32, seed div 2^32).  The four output words give two uniforms with
53 random bits each, u = ((w_a >> 5) 2^26 + (w_b >> 6) + 1/2) 2^-53, which lie
strictly inside (0, 1), and the Box-Muller transform (Box and Muller, 1958)
turns them into the pair sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) of
independent N(0,1) numbers.  A real block takes the first of the pair; a
complex block takes both as real and imaginary part, times sqrt(1/2).

Pins (tests/test_oracle_rng.py): the published known-answer vectors of
Philox-4x32-10, the closed-form extremes of the uniform map, and the normal
distribution of the block (Kolmogorov-Smirnov against scipy, moments,
independence of the real and imaginary parts).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(counter, key):
    """Philox-4x32-10 of counters ``counter`` (array (..., 4) of words) under
    the key (k0, k1); returns the four output words as uint32, shape (..., 4)."""
    c = np.asarray(counter, dtype=np.uint64) & _LO
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0                     # < 2^64: exact in uint64
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ np.uint64(k0), p1 & _LO,
                          (p0 >> _S32) ^ c3 ^ np.uint64(k1), p0 & _LO)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniform53(wa, wb):
    """Two 32-bit words -> a uniform in (0, 1) with 53 random bits:
    ((wa >> 5) 2^26 + (wb >> 6) + 1/2) 2^-53, computed exactly in float64."""
    a = (np.asarray(wa, dtype=np.uint64) >> np.uint64(5)).astype(np.float64)
    b = (np.asarray(wb, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b + 0.5) * 2.0 ** -53


def start_block(n: int, ncols: int, seed: int, complex_: bool) -> np.ndarray:
    """The (n, ncols) start block: float64 N(0,1) entries, or complex128 with
    real and imaginary parts N(0, 1/2)."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(ncols, dtype=np.uint64)[None, :]
    ctr = np.zeros((n, ncols, 4), dtype=np.uint64)
    ctr[..., 0] = i & _LO
    ctr[..., 1] = j
    ctr[..., 2] = i >> _S32
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u1 = uniform53(w[..., 0], w[..., 1])
    u2 = uniform53(w[..., 2], w[..., 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    if not complex_:
        return rad * np.cos(2.0 * np.pi * u2)
    return np.sqrt(0.5) * rad * np.exp(2j * np.pi * u2)
