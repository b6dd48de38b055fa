"""The subsampled randomized Hadamard test matrix (oracle side; test infrastructure only).

The paper's footnote to the range finder (Sec. 3.1) names structured test matrices, the
subsampled randomized Fourier transform, as a common alternative to Gaussian ones.  For real
symmetric X the real form is used: Omega = D H S restricted to the first n rows, with
  N = 2^m, m = max(1, ceil(log2 n));
  D = diag(d_0 .. d_{N-1}), d_i = +1 or -1 (the low bit of Philox word x0 of counter i, stream 3);
  H the N x N Walsh-Hadamard matrix, H[i][s] = (-1)^popcount(i & s);
  S the N x r selection of columns s_0 .. s_{r-1}, s_j = pi(j) for a random permutation pi of
  [0, N): a four-round Feistel network on w = m + (m mod 2) bits (halves of h = w/2 bits, round t
  mixing the right half R into the left with F_t(R) = low h bits of Philox word x0 of counter
  t 2^h + R, stream 4), applied again while the result is >= N (cycle walking, which keeps it a
  bijection of [0, N)); distinct j give distinct columns.
Readings (listed in the design notes):
  R17  The normalisation sqrt(N / r) / sqrt(N) of the transform is left out: entries are exactly
       +1 or -1.  Only range(X Omega) enters the method, which a scale does not change.
  R18  The random column selection is drawn without replacement through the Feistel permutation
       above, a counter-based construction both sides can evaluate entry by entry.
"""
from __future__ import annotations

import numpy as np

from . import philox

STREAM_SRHT_SIGNS = 3
STREAM_SRHT_PERM = 4


def log2_size(n: int) -> int:
    m = 1
    while (1 << m) < n:
        m += 1
    return m


def signs(seed: int, count: int) -> np.ndarray:
    """d_0 .. d_{count-1} in {+1, -1}."""
    w = philox.raw_words(seed, STREAM_SRHT_SIGNS, np.arange(count, dtype=np.uint64))
    return 1.0 - 2.0 * (w[:, 0] & 1).astype(np.float64)


def feistel(seed: int, x: int, m: int) -> int:
    """One application of the four-round Feistel network on w = m + (m mod 2) bits."""
    w = m + (m & 1)
    h = w // 2
    mask = (1 << h) - 1
    L, R = (x >> h) & mask, x & mask
    for t in range(4):
        f = int(philox.raw_words(seed, STREAM_SRHT_PERM, [t * (1 << h) + R])[0, 0]) & mask
        L, R = R, L ^ f
    return (L << h) | R


def permute(seed: int, j: int, m: int) -> int:
    """pi(j): the Feistel network, re-applied while the value lies outside [0, 2^m)."""
    y = feistel(seed, j, m)
    while y >= (1 << m):
        y = feistel(seed, y, m)
    return y


def columns(seed: int, n: int, r: int) -> np.ndarray:
    m = log2_size(n)
    return np.array([permute(seed, j, m) for j in range(r)], dtype=np.int64)


def hadamard_entry(i, s):
    """(-1)^popcount(i & s), elementwise over integer arrays."""
    v = np.bitwise_and(np.asarray(i, dtype=np.int64), np.asarray(s, dtype=np.int64))
    par = np.zeros(v.shape, dtype=np.int64)
    while np.any(v):
        par ^= v & 1
        v = v >> 1
    return 1.0 - 2.0 * par


def test_matrix(seed: int, n: int, r: int) -> np.ndarray:
    """The n x r structured test matrix Omega[i][j] = d_i (-1)^popcount(i & s_j)."""
    d = signs(seed, n)
    s = columns(seed, n, r)
    i = np.arange(n)[:, None]
    return d[:, None] * hadamard_entry(i, s[None, :])
