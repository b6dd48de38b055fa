"""The randomized PSD projection, step by step, in FP64 (oracle; test infrastructure only).

Follows Jones & Anderson, "Approximate Projection onto the Positive
Semidefinite Cone Using Randomization":
  * Thm 1 (Sec. 3): X_+ = U max(D,0) U^T from the eigendecomposition X = U D U^T.
  * Alg. 1 (Sec. 3.1): range finder, Q = orth((X X^T)^q X Omega).
  * Alg. 2 (Sec. 3.1): plain randomized projection Q V max(D,0) V^T Q^T with
    Q^T X Q = V D V^T.
  * Alg. 3 (Sec. 3.2): scaled projection with B = (X + alpha I)/alpha and
    alpha Q V (max(D,1) - I) V^T Q^T, Q^T B Q = V D V^T.
  * Alg. 4 (Sec. 3.2): power iteration for sigma_1.
  * Alg. 5 (Sec. 3.2): alpha = |sigma_1(X) - sigma_1(X - sigma_1(X) I)|.

Readings taken where the paper is silent or garbled (each is listed in the
design notes of the repository):
  R1  Alg. 1 forms (X X^T)^q X Omega and orthonormalises once.  Here the
      range is built by subspace iteration with an orthonormalisation after
      every product with X (X is symmetric, so X^T = X):
      Q = orth(X Omega); q times: Q = orth(X orth(X Q)).  In exact arithmetic
      the range is the same; ``range_finder_literal`` keeps the printed form
      for comparison at small sizes.
  R2  Omega is n x (k+l) (the printed randn(m, k+l) is for a general m x n X).
  R3  All k+l eigenpairs of the (k+l) x (k+l) compressed matrix are kept; the
      clamp decides which contribute (no truncation to rank k).
  R4  The compressed matrix is symmetrised, C <- (C + C^T)/2, before the
      eigensolve.
  R5  Weights are exactly max(d, 0) (Alg. 2) and alpha (max(d, 1) - 1)
      (Alg. 3); a weight of zero contributes nothing.
  R6  Alg. 4 draws a fresh N(0,1) start vector on each call (Philox streams 1
      and 2); if X v = 0 the estimate is 0.  N >= 1.
  R7  The test matrix entries are the Philox/Box-Muller normals rounded to the
      storage precision of the computation (FP64, or FP32 for the FP32 and
      split-BF16 paths), then promoted back to FP64.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import philox, srht

__all__ = [
    "orth", "range_finder", "range_finder_literal", "ran_proj", "ran_proj_scal",
    "power_iteration", "min_eig", "exact_projection", "projection_errors",
    "ProjResult", "parity_error", "project",
]


@dataclasses.dataclass
class ProjResult:
    """Everything the oracle computes on the way to the projection."""
    Q: np.ndarray            # n x r orthonormal basis of the sketch range
    C: np.ndarray            # r x r compressed matrix (symmetrised)
    evals: np.ndarray        # ascending eigenvalues of C
    V: np.ndarray            # eigenvectors of C (columns)
    weights: np.ndarray      # clamped weights per eigenpair (same order as evals)
    U_keep: np.ndarray       # Q V restricted to positive weights
    w_keep: np.ndarray       # the positive weights
    alpha: float | None      # scaling parameter (scaled variant)
    sigma1: float | None = None
    sigma2: float | None = None
    P: np.ndarray | None = None

    @property
    def r_plus(self) -> int:
        return int(self.w_keep.size)

    def entries(self, rows, cols) -> np.ndarray:
        """P[rows[i], cols[i]] computed one by one from the factors."""
        Uw = self.U_keep * self.w_keep[None, :]
        return np.einsum("ij,ij->i", Uw[np.asarray(rows)], self.U_keep[np.asarray(cols)])


def _f64(X) -> np.ndarray:
    return np.asarray(X, dtype=np.float64)


def orth(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) by Householder economy QR (LAPACK
    dgeqrf/dorgqr): the 'orth' / economy-QR step of Alg. 1."""
    q, _ = np.linalg.qr(Y, mode="reduced")
    return q


def range_finder(X: np.ndarray, Omega: np.ndarray, q: int) -> np.ndarray:
    """Alg. 1 with reading R1: Q = orth(X Omega), then q times Q = orth(X orth(X Q))."""
    Q = orth(X @ Omega)
    for _ in range(q):
        Q = orth(X.T @ Q)
        Q = orth(X @ Q)
    return Q


def range_finder_literal(X: np.ndarray, Omega: np.ndarray, q: int) -> np.ndarray:
    """Alg. 1 exactly as printed: one QR of (X X^T)^q X Omega (diagnostic only)."""
    W = X @ Omega
    for _ in range(q):
        W = X @ (X.T @ W)
    return orth(W)


def _omega(seed: int, n: int, r: int, omega_dtype, sketch: str = "gaussian") -> np.ndarray:
    if sketch == "srht":
        return srht.test_matrix(seed, n, r)          # entries +-1, exact in every precision
    om = philox.test_matrix(seed, n, r)
    return om.astype(omega_dtype).astype(np.float64)


def _finish(Q, C, alpha, scaled, keep_P):
    C = 0.5 * (C + C.T)                                  # R4
    evals, V = np.linalg.eigh(C)                         # Alg. 2/3: eig(Q^T X Q) / eig(Q^T B Q)
    if scaled:
        weights = alpha * (np.maximum(evals, 1.0) - 1.0)  # Alg. 3: alpha (max(D,1) - I)
    else:
        weights = np.maximum(evals, 0.0)                  # Alg. 2: D_+
    keep = weights > 0.0
    U = Q @ V
    res = ProjResult(Q=Q, C=C, evals=evals, V=V, weights=weights,
                     U_keep=U[:, keep], w_keep=weights[keep], alpha=alpha)
    if keep_P:
        # Alg. 2/3 last line: Q V D V^T Q^T with the clamped diagonal.
        res.P = (U * weights[None, :]) @ U.T
    return res


def ran_proj(X, k: int, p: int, q: int, seed: int = 0, omega_dtype=np.float64,
             Omega: np.ndarray | None = None, keep_P: bool = True, sketch: str = "gaussian") -> ProjResult:
    """Alg. 2 (plain randomized PSD projection), oversampling l = p."""
    X = _f64(X)
    n = X.shape[0]
    r = k + p
    if not (1 <= r <= n):
        raise ValueError("need 1 <= k+p <= n")
    if Omega is None:
        Omega = _omega(seed, n, r, omega_dtype, sketch)
    Q = range_finder(X, Omega, q)                        # Alg. 2 line 1
    C = Q.T @ (X @ Q)                                    # Q^T X Q
    return _finish(Q, C, None, False, keep_P)


def ran_proj_scal(X, k: int, p: int, q: int, alpha: float, seed: int = 0,
                  omega_dtype=np.float64, Omega: np.ndarray | None = None,
                  keep_P: bool = True, sketch: str = "gaussian") -> ProjResult:
    """Alg. 3 (scaled randomized PSD projection) for a given alpha > 0."""
    X = _f64(X)
    n = X.shape[0]
    r = k + p
    if not (alpha > 0.0 and np.isfinite(alpha)):
        raise ValueError("alpha must be positive and finite")
    if not (1 <= r <= n):
        raise ValueError("need 1 <= k+p <= n")
    B = X / alpha                                        # Alg. 3 line 1: B = (X + alpha I)/alpha
    B[np.diag_indices(n)] = (np.diag(X) + alpha) / alpha
    if Omega is None:
        Omega = _omega(seed, n, r, omega_dtype, sketch)
    Q = range_finder(B, Omega, q)                        # line 2
    C = Q.T @ (B @ Q)                                    # line 3: Q^T B Q
    return _finish(Q, C, float(alpha), True, keep_P)     # line 4


def power_iteration(X, N: int, v0: np.ndarray) -> float:
    """Alg. 4: N normalised products with X from v0, then sigma_1 = ||X v||."""
    X = _f64(X)
    if N < 1:
        raise ValueError("N >= 1")
    v = np.array(v0, dtype=np.float64)
    for _ in range(N):
        y = X @ v
        nrm = np.linalg.norm(y)
        if nrm == 0.0:
            return 0.0                                   # R6
        v = y / nrm
    return float(np.linalg.norm(X @ v))


def min_eig(X, N: int, seed: int = 0):
    """Alg. 5: returns (alpha, sigma1, sigma2) with alpha = |sigma1 - sigma2|."""
    X = _f64(X)
    n = X.shape[0]
    s1 = power_iteration(X, N, philox.gaussian(seed, philox.STREAM_POWER1, n))
    Y = X.copy()
    Y[np.diag_indices(n)] -= s1                           # Y = X - sigma1 I
    s2 = power_iteration(Y, N, philox.gaussian(seed, philox.STREAM_POWER2, n))
    return abs(s1 - s2), s1, s2


def project(X, k: int, p: int, q: int, variant: str = "plain", seed: int = 0,
            alpha: float | None = None, alpha_iters: int = 10,
            omega_dtype=np.float64, keep_P: bool = True, sketch: str = "gaussian") -> ProjResult:
    """One call of the method as the library exposes it: plain (Alg. 2) or
    scaled (Alg. 3 with alpha given, or estimated by Alg. 5 with N = alpha_iters);
    sketch "gaussian" (Alg. 1's randn) or "srht" (the structured test matrix)."""
    if variant == "plain":
        return ran_proj(X, k, p, q, seed, omega_dtype, keep_P=keep_P, sketch=sketch)
    s1 = s2 = None
    if alpha is None or alpha <= 0.0:
        alpha, s1, s2 = min_eig(X, alpha_iters, seed)
    res = ran_proj_scal(X, k, p, q, alpha, seed, omega_dtype, keep_P=keep_P, sketch=sketch)
    res.sigma1, res.sigma2 = s1, s2
    return res


def exact_projection(X) -> np.ndarray:
    """Thm 1: X_+ = U max(D, 0) U^T from a full symmetric eigendecomposition."""
    X = _f64(X)
    d, U = np.linalg.eigh(0.5 * (X + X.T))
    return (U * np.maximum(d, 0.0)[None, :]) @ U.T


def parity_error(P, P_ref, A_fro: float) -> float:
    """||P - P_ref||_F / max(||P_ref||_F, 1e-2 ||A||_F) (floor for P_ref = 0)."""
    P = _f64(P)
    P_ref = _f64(P_ref)
    return float(np.linalg.norm(P - P_ref) / max(np.linalg.norm(P_ref), 1e-2 * A_fro))


def projection_errors(X, P, X_plus, Q=None) -> dict:
    """The Sec. 4 metrics: ||X_+ - P||/||X_+|| and, given Q, ||X - Q Q^T X||/||X||
    (Frobenius, written ||.||_2 in the paper)."""
    X = _f64(X)
    out = {"e_alg": float(np.linalg.norm(X_plus - P) / np.linalg.norm(X_plus))}
    if Q is not None:
        out["range_err"] = float(np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X))
    return out
