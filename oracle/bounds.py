"""Expected-error bounds of Sec. 3 (oracle side; test infrastructure only).

eps1 and eps2 are the two quantities defined before Cor. 1; the
oversampling parameter l of the paper is p here.
"""
from __future__ import annotations

import math

import numpy as np


def eps1(values, k: int, l: int) -> float:
    """sqrt((1 + k/(l-1)) * sum_{j>k} s_j^2) with s sorted decreasingly."""
    s = np.sort(np.abs(np.asarray(values, dtype=np.float64)))[::-1]
    return math.sqrt((1.0 + k / (l - 1.0)) * float(np.sum(s[k:] ** 2)))


def eps2(sigma: float, k: int, l: int, q: int, n: int) -> float:
    """(1 + sqrt(k/(l-1)) + e sqrt(k+l)/l * sqrt(n-k))^(1/(2q+1)) * sigma."""
    base = 1.0 + math.sqrt(k / (l - 1.0)) + math.e * math.sqrt(k + l) / l * math.sqrt(n - k)
    return base ** (1.0 / (2 * q + 1)) * sigma


def cor1_frobenius(eigs, k: int, l: int) -> float:
    """Cor. 1 (q = 0): E||X_+ - Xhat_+||_F <= sqrt(2) eps1(sigma(X), k, l)."""
    return math.sqrt(2.0) * eps1(np.abs(eigs), k, l)


def prop2_frobenius(eigs, alpha: float, k: int, l: int) -> float:
    """Prop. 2 (q = 0): E||X_+ - Xhat_+||_F <= sqrt(2) eps1({lambda_i + alpha}, k, l)."""
    return math.sqrt(2.0) * eps1(np.asarray(eigs) + alpha, k, l)


def _spectral(e2: float, sigma1: float, n: int) -> float:
    a = (1.0 + math.sqrt(n)) * e2
    b = (1.0 + 4.0 / math.pi + (2.0 / math.pi) * math.log(2.0 * sigma1)) * e2 \
        + (1.0 / math.pi) * min(math.exp(-1.0), math.sqrt(2.0 * e2))
    return min(a, b)


def cor1_spectral(eigs, k: int, l: int, q: int) -> float:
    """Cor. 1 spectral-norm bound with eps2(sigma_{k+1}(X), k, l, q)."""
    s = np.sort(np.abs(np.asarray(eigs, dtype=np.float64)))[::-1]
    n = s.size
    return _spectral(eps2(float(s[k]), k, l, q, n), float(s[0]), n)


def prop2_spectral(eigs, alpha: float, k: int, l: int, q: int) -> float:
    """Prop. 2 spectral-norm bound with eps2(lambda_{k+1}(X) + alpha, k, l, q)."""
    lam = np.sort(np.asarray(eigs, dtype=np.float64))[::-1]
    n = lam.size
    s1 = float(np.max(np.abs(lam)))
    return _spectral(eps2(float(lam[k] + alpha), k, l, q, n), s1, n)
