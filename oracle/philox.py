"""Philox4x32-10 and Box-Muller Gaussians (oracle side; test infrastructure only).

Philox4x32-10 follows its published definition (Salmon et al., SC'11):
a 128-bit counter (c0,c1,c2,c3) and a 64-bit key (k0,k1); each of the ten
rounds maps
    (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),
                      hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and between rounds the key is bumped
by the Weyl constants (0x9E3779B9, 0xBB67AE85).

Project convention for the method's random draws (the paper only asks for
i.i.d. N(0,1) entries, Alg. 1 and Alg. 4, and notes that the distribution
is not critical):
  key     = (seed mod 2^32, seed div 2^32)
  counter = (c mod 2^32, c div 2^32, stream, 0)
  element g of a stream (for the n x r test matrix, g = j*n + i for entry
  (i, j), i.e. column j is the test vector omega_j) uses counter c = g // 2;
  the four output words give two uniforms
      u1 = ((x0 * 2^32 + x1) >> 11) * 2^-53 + 2^-54,
      u2 = ((x2 * 2^32 + x3) >> 11) * 2^-53 + 2^-54,   both in (0, 1),
  and Box-Muller gives z0 = sqrt(-2 ln u1) cos(2 pi u2) for even g and
  z1 = sqrt(-2 ln u1) sin(2 pi u2) for odd g.
  Streams: 0 = the test matrix Omega, 1 = the start vector of the first
  power iteration of Alg. 5, 2 = that of the second.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)

STREAM_OMEGA = 0
STREAM_POWER1 = 1
STREAM_POWER2 = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments are uint32 arrays (or scalars)
    of a common shape; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.asarray(k0, dtype=np.uint32)
    k1 = np.asarray(k1, dtype=np.uint32)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3 = (x.copy() for x in (c0, c1, c2, c3))
    k0, k1 = k0.copy(), k1.copy()
    for rnd in range(10):
        if rnd > 0:
            # key bump between rounds, modulo 2^32
            k0 = ((k0.astype(np.uint64) + np.uint64(W0)) & _MASK32).astype(np.uint32)
            k1 = ((k1.astype(np.uint64) + np.uint64(W1)) & _MASK32).astype(np.uint32)
        p0 = M0 * c0.astype(np.uint64)
        p1 = M1 * c2.astype(np.uint64)
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & _MASK32).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & _MASK32).astype(np.uint32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.uint32(seed & 0xFFFFFFFF), np.uint32(seed >> 32)


def raw_words(seed: int, stream: int, counters) -> np.ndarray:
    """Philox outputs for counters c (array of ints): shape (len(c), 4) uint32."""
    c = np.asarray(counters, dtype=np.uint64)
    k0, k1 = _key(seed)
    x0, x1, x2, x3 = philox4x32_10((c & _MASK32).astype(np.uint32),
                                   (c >> np.uint64(32)).astype(np.uint32),
                                   np.uint32(stream), np.uint32(0), k0, k1)
    return np.stack([x0, x1, x2, x3], axis=-1)


def _uniform53(hi, lo):
    v = (hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)
    return (v >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) + 2.0 ** -54


def gaussian(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Elements g = start .. start+count-1 of a Gaussian stream (float64)."""
    if count <= 0:
        return np.zeros(0)
    g = np.arange(start, start + count, dtype=np.uint64)
    c = g >> np.uint64(1)
    w = raw_words(seed, stream, c)
    u1 = _uniform53(w[:, 0], w[:, 1])
    u2 = _uniform53(w[:, 2], w[:, 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    odd = (g & np.uint64(1)).astype(bool)
    return np.where(odd, rad * np.sin(ang), rad * np.cos(ang))


def test_matrix(seed: int, n: int, r: int, stream: int = STREAM_OMEGA) -> np.ndarray:
    """The n x r Gaussian test matrix Omega (Alg. 1): entry (i, j) is element j*n+i."""
    flat = gaussian(seed, stream, n * r)
    return flat.reshape(r, n).T.copy()
