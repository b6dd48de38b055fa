"""Pins for the error-bound calculators (oracle/bounds.py) and the Sec. 4 error metrics
(oracle/rnla.projection_errors).

The bound functions are checked against identities that a misplaced exponent, index or
constant breaks, and against seed-mean errors of the oracle's own projections at q >= 1
(Cor. 1 and Prop. 2 hold in expectation).  projection_errors is checked against closed
forms for a basis made of exact eigenvectors.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import bounds, rnla


def sym_from(lam, seed):
    U = workloads.haar_orthogonal(len(lam), seed)
    return workloads.from_spectrum(U, np.asarray(lam, float)), U


# ---------------------------------------------------------------- eps1 / eps2 (Sec. 3.1)
@pytest.mark.parametrize("q", [1, 2, 3])
@pytest.mark.parametrize("k,l,n", [(2, 2, 10), (20, 6, 300), (200, 20, 20000)])
def test_eps2_power_exponent(q, k, l, n):
    """eps2 takes the (2q+1)-th root of the q = 0 factor: eps2(s, q)^(2q+1) equals
    eps2(s^(2q+1), 0).  An exponent other than 1/(2q+1) breaks this for some q."""
    for s in (0.3, 1.0, 7.5):
        lhs = bounds.eps2(s, k, l, q, n) ** (2 * q + 1)
        rhs = bounds.eps2(s ** (2 * q + 1), k, l, 0, n)
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_eps2_decreases_to_sigma():
    """The power scheme compresses the factor towards 1: eps2 decreases in q and tends to sigma."""
    vals = [bounds.eps2(2.0, 20, 6, q, 300) for q in range(0, 60)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert vals[-1] == pytest.approx(2.0, rel=0.05)
    assert vals[0] > 2.0 * 5


def test_eps1_flat_tail():
    """eps1 over n equal values s: sqrt((1 + k/(l-1)) (n - k)) s (only the n - k values past k count)."""
    n, k, l, s = 50, 7, 4, 0.6
    assert bounds.eps1(np.full(n, s), k, l) == pytest.approx(math.sqrt((1 + k / (l - 1)) * (n - k)) * s, rel=1e-14)
    # values past k only, sorted by magnitude whatever their sign and order
    vals = np.concatenate([np.full(k, 100.0), np.full(n - k, -s)])
    np.random.default_rng(0).shuffle(vals)
    assert bounds.eps1(vals, k, l) == pytest.approx(math.sqrt((1 + k / (l - 1)) * (n - k)) * s, rel=1e-14)


# ---------------------------------------------------------------- Cor. 1 / Prop. 2 at q >= 1
@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("variant", ["plain", "scaled"])
def test_spectral_bounds_with_power_steps(variant, q):
    """Cor. 1 and Prop. 2, spectral form for q in N: the seed mean of ||X_+ - Xhat_+|| (spectral)
    stays below the bound with eps2 at the (2q+1)-th root.  The spectrum has a slowly decaying
    tail so that the q = 0 bound is far above the q >= 1 one."""
    n, k, l = 240, 12, 4
    rng = np.random.default_rng(40 + q)
    lam = np.concatenate([np.linspace(3.0, 1.0, 16), rng.uniform(-0.9, 0.4, n - 16)])
    X, U = sym_from(lam, 41)
    Xp = (U * np.maximum(lam, 0)[None, :]) @ U.T
    alpha = abs(lam.min())
    errs = []
    for s in range(8):
        P = rnla.project(X, k, l, q, variant, seed=s, alpha=alpha).P
        errs.append(np.linalg.norm(Xp - P, 2))
    if variant == "plain":
        b = bounds.cor1_spectral(lam, k, l, q)
        b0 = bounds.cor1_spectral(lam, k, l, 0)
    else:
        b = bounds.prop2_spectral(lam, alpha, k, l, q)
        b0 = bounds.prop2_spectral(lam, alpha, k, l, 0)
    assert np.mean(errs) <= b
    assert b < b0


@pytest.mark.parametrize("q", [0, 1, 2])
def test_range_error_power_scheme_bound(q):
    """The range-finder bound behind eps2: E ||(I - Q Q^T) X|| (spectral) <= eps2(sigma_{k+1}, k, l, q),
    as a mean over seeds; the power steps shrink the observed error as well."""
    n, k, l = 200, 10, 5
    lam = np.concatenate([np.linspace(4.0, 2.0, 10), 0.8 * (-1.0) ** np.arange(n - 10)])
    X, _ = sym_from(lam, 43)
    s_sorted = np.sort(np.abs(lam))[::-1]
    errs = []
    for s in range(8):
        Q = rnla.ran_proj(X, k, l, q, seed=s, keep_P=False).Q
        errs.append(np.linalg.norm(X - Q @ (Q.T @ X), 2))
    assert np.mean(errs) <= bounds.eps2(float(s_sorted[k]), k, l, q, n)
    assert np.mean(errs) >= s_sorted[k + l] * (1 - 1e-12)   # never below the best rank-(k+l) error


# ---------------------------------------------------------------- Sec. 4 error metrics
@pytest.mark.parametrize("take", [[0, 1, 2, 3, 4, 5], [0, 2, 7, 9, 30, 31, 60], list(range(40))])
def test_projection_errors_exact_eigenvectors(take):
    """With Q made of exact eigenvectors u_i (i in S) of X = U diag(lam) U^T:
    ||X - Q Q^T X|| / ||X|| = ||lam_{not S}|| / ||lam||, the plain projection is
    sum_{i in S} max(lam_i, 0) u_i u_i^T, so ||X_+ - P|| / ||X_+|| = ||max(lam_{not S}, 0)|| / ||max(lam, 0)||."""
    n = 64
    lam = np.concatenate([np.linspace(2.0, 0.05, 24), -np.linspace(0.03, 1.5, n - 24)])
    X, U = sym_from(lam, 44)
    S = np.array(take)
    rest = np.setdiff1d(np.arange(n), S)
    Q = U[:, S]
    C = Q.T @ X @ Q
    d, V = np.linalg.eigh(0.5 * (C + C.T))
    W = Q @ V
    P = (W * np.maximum(d, 0.0)[None, :]) @ W.T
    Xp = (U * np.maximum(lam, 0.0)[None, :]) @ U.T
    out = rnla.projection_errors(X, P, Xp, Q)
    assert out["range_err"] == pytest.approx(np.linalg.norm(lam[rest]) / np.linalg.norm(lam), rel=1e-10)
    assert out["e_alg"] == pytest.approx(np.linalg.norm(np.maximum(lam[rest], 0.0))
                                         / np.linalg.norm(np.maximum(lam, 0.0)), rel=1e-10)
    assert set(out) == {"range_err", "e_alg"}
    assert set(rnla.projection_errors(X, P, Xp)) == {"e_alg"}
