"""Seeded synthetic inputs shaped like the paper's workloads.

This module only manufactures test matrices; it contains no step of the
projection method (no sketch, no orthonormalisation of a sketch, no
compression, eigensolve, clamp or rebuild).  Both the FP64 oracle and the
GPU library consume what it produces, so neither side can drift from the
other's inputs.

Every matrix is A = U diag(lam) U^T (optionally plus a symmetric Gaussian
perturbation), with U Haar-orthogonal: the Q factor of a seeded N(0,1)
matrix with the sign fix U = Q diag(sign(diag R)) (Mezzadri, "How to
generate random matrices from the classical compact groups", 2007).  The
closed-form PSD projection U diag(max(lam,0)) U^T of Thm 1 is then known
without a full eigendecomposition.

The spectra follow the synthetic stand-ins for the paper's workloads: the
paper projects large sparse matrices from the SuiteSparse collection
(Sec. 4, Example 2, Table 1) that are not available here, so seeded dense
matrices with spectra of the same character (mostly negative, a decaying
positive head, n up to about 20K) stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "haar_orthogonal", "from_spectrum",
    "spectrum_small", "spectrum_medium", "spectrum_large", "spectrum_batched",
    "cor2_spectrum", "make_matrix", "batched_problem_sizes", "serving_requests", "sdls_problem",
    "sparse_symmetric",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and parameters of one benchmark workload."""
    name: str
    n: int
    k: int
    p: int
    q: int
    precision: str          # "fp64" | "fp32" | "bf16x3"
    variants: tuple         # ("plain",) or ("plain", "scaled")
    gen_seed: int
    description: str


WORKLOADS = {
    "small_fp64": Workload(
        "small_fp64", 512, 40, 10, 0, "fp64", ("plain",), 1001,
        "n=512 FP64, 32 positive eigenvalues geometric 1..1e-3, 480 uniform "
        "in [-0.1,0]; k=40, p=10, q=0; plain"),
    "medium_fp32": Workload(
        "medium_fp32", 4096, 100, 10, 1, "fp32", ("plain", "scaled"), 0,
        "n=4096 FP32, 200 positive eigenvalues 1/i, 3896 uniform in "
        "[-0.5,0], symmetric Gaussian noise 1e-3/sqrt(n); k=100, p=10, "
        "q in {0,1}; plain and scaled; seeds 0..7"),
    "large_20k": Workload(
        "large_20k", 20000, 200, 20, 1, "bf16x3", ("plain", "scaled"), 3001,
        "n=20000, A stored FP32 (1.6 GB); 5% positive eigenvalues decaying "
        "exponentially 10..1e-4, the rest uniform in [-1,0]; k=200, p=20, "
        "q=1; plain and scaled"),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthogonal(n: int, seed: int, device: str = "cpu"):
    """Haar-distributed orthogonal n x n matrix (Mezzadri 2007).

    On device="cpu" returns a float64 numpy array.  Any other device
    returns a float64 torch tensor built there (used for the n = 20000
    workload, where a host QR would take minutes).
    """
    if device == "cpu":
        g = _rng(seed).standard_normal((n, n))
        q, r = np.linalg.qr(g)
        s = np.sign(np.diag(r))
        s[s == 0] = 1.0
        return q * s[None, :]
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn((n, n), dtype=torch.float64, device=device, generator=gen)
    q, r = torch.linalg.qr(g)
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def from_spectrum(U, lam):
    """A = U diag(lam) U^T, symmetrised so that A == A^T bit for bit."""
    if isinstance(U, np.ndarray):
        a = (U * np.asarray(lam)[None, :]) @ U.T
        return 0.5 * (a + a.T)
    import torch
    lam_t = torch.as_tensor(lam, dtype=U.dtype, device=U.device)
    a = (U * lam_t[None, :]) @ U.T
    return 0.5 * (a + a.T)


def spectrum_small(n: int = 512, n_pos: int = 32, seed: int = 1001) -> np.ndarray:
    """n_pos eigenvalues geometric from 1 to 1e-3, the rest uniform in [-0.1, 0]."""
    pos = 10.0 ** (-3.0 * np.arange(n_pos) / max(n_pos - 1, 1))
    neg = -0.1 * _rng(seed + 17).random(n - n_pos)
    return np.concatenate([pos, neg])


def spectrum_medium(n: int = 4096, n_pos: int = 200, seed: int = 0) -> np.ndarray:
    """n_pos eigenvalues 1/i (power law), the rest uniform in [-0.5, 0]."""
    pos = 1.0 / np.arange(1, n_pos + 1, dtype=np.float64)
    neg = -0.5 * _rng(seed + 29).random(n - n_pos)
    return np.concatenate([pos, neg])


def spectrum_large(n: int = 20000, frac_pos: float = 0.05, seed: int = 3001) -> np.ndarray:
    """frac_pos*n eigenvalues decaying exponentially from 10 to 1e-4, the rest uniform in [-1, 0]."""
    n_pos = max(1, int(round(frac_pos * n)))
    pos = 10.0 * 10.0 ** (-5.0 * np.arange(n_pos) / max(n_pos - 1, 1))
    neg = -_rng(seed + 31).random(n - n_pos)
    return np.concatenate([pos, neg])


def spectrum_batched(n: int, frac_pos: float, seed: int) -> np.ndarray:
    """Per-matrix spectrum of the batched workload: round(frac_pos*n) values
    geometric 1..1e-3, the rest uniform in [-0.1, 0]."""
    n_pos = max(1, int(round(frac_pos * n)))
    pos = 10.0 ** (-3.0 * np.arange(n_pos) / max(n_pos - 1, 1))
    neg = -0.1 * _rng(seed + 41).random(n - n_pos)
    return np.concatenate([pos, neg])


def cor2_spectrum(n: int, beta=(3.0, 1.0, 6.0, 2.0)) -> np.ndarray:
    """Eigenvalues of the matrix class of Cor. 2: blocks of n/4 equal values
    -beta1, -beta2, beta3, beta4 (the second and fourth block lengths read as
    n/4; the printed subscript is garbled)."""
    assert n % 4 == 0
    b1, b2, b3, b4 = beta
    m = n // 4
    return np.concatenate([np.full(m, -b1), np.full(m, -b2), np.full(m, b3), np.full(m, b4)])


def symmetric_noise(n: int, scale: float, seed: int) -> np.ndarray:
    g = _rng(seed + 53).standard_normal((n, n))
    return (g + g.T) * (scale / math.sqrt(2.0))


def make_matrix(kind: str, n: int, seed: int, storage: str = "fp64", device: str = "cpu", **kw):
    """Build one synthetic workload matrix.

    kind: "small" | "medium" | "large" | "batched" | "cor2" | "spectrum"
    (for "spectrum" pass lam=...).  Returns (A, lam, U) where A is in the
    storage precision (numpy on cpu, torch on other devices) and lam/U
    are the float64 spectrum and eigenvectors of the noiseless part.
    """
    if kind == "small":
        lam = spectrum_small(n, kw.get("n_pos", min(32, n)), seed)
    elif kind == "medium":
        lam = spectrum_medium(n, kw.get("n_pos", min(200, n)), seed)
    elif kind == "large":
        lam = spectrum_large(n, kw.get("frac_pos", 0.05), seed)
    elif kind == "batched":
        lam = spectrum_batched(n, kw["frac_pos"], seed)
    elif kind == "cor2":
        lam = cor2_spectrum(n, kw.get("beta", (3.0, 1.0, 6.0, 2.0)))
    elif kind == "spectrum":
        lam = np.asarray(kw["lam"], dtype=np.float64)
    else:
        raise ValueError(kind)
    U = haar_orthogonal(n, seed, device)
    A = from_spectrum(U, lam)
    noise = kw.get("noise", 0.0)
    if noise:
        E = symmetric_noise(n, noise, seed)
        if device == "cpu":
            A = A + E
        else:
            import torch
            A = A + torch.as_tensor(E, device=A.device)
    if device == "cpu":
        A = A.astype(np.float32 if storage in ("fp32", "bf16x3") else np.float64)
    else:
        import torch
        A = A.to(torch.float32 if storage in ("fp32", "bf16x3") else torch.float64)
    return A, lam, U


def batched_problem_sizes(count: int = 256, seed: int = 4000, nmin: int = 64, nmax: int = 4096,
                          kmax: int = 128, p: int = 10):
    """(n, k, p, frac_pos) for the batched uneven workload: n log-uniform in
    [nmin, nmax], k = min(n // 8, kmax), positive fraction uniform in [0.02, 0.3]."""
    g = _rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        k = max(1, min(n // 8, kmax))
        f = float(g.uniform(0.02, 0.3))
        out.append((n, k, p, f))
    return out


def serving_requests(count: int, qps: float, seed: int, nmin: int = 256, nmax: int = 16384,
                     ks=(20, 50, 100, 200), p: int = 10, q: int = 1):
    """Poisson arrival stream: list of (t_arrival_s, n, k, p, q, variant)."""
    g = _rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(g.exponential(1.0 / qps))
        n = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        k = int(g.choice(ks))
        k = min(k, max(1, n - p))
        variant = "scaled" if g.random() < 0.5 else "plain"
        out.append((t, n, k, p, q, variant))
    return out


def sdls_problem(n: int, m: int, seed: int, dtype=np.float64):
    """Synthetic SDLS instance after the recipe of the supplementary SDP section's first example:
    A_i = (G_i + G_i^T) / (2 ||G_i||_F) with G_i N(0,1) n x n; a PSD X0 = H H^T / n (H N(0,1))
    and b_i = Tr(A_i X0), so the problem is feasible; C = (K + K^T) / (2 sqrt(n)) with K N(0,1);
    y0 ~ N(0,1) (the random initialisation of the dual iterate).  Returns (C, A (m x n x n), b,
    y0), C and A in `dtype`, b and y0 computed in float64 from the stored A."""
    g = _rng(seed)
    A = np.empty((m, n, n), dtype=dtype)
    for i in range(m):
        G = g.standard_normal((n, n))
        A[i] = ((G + G.T) / (2.0 * np.linalg.norm(G))).astype(dtype)
    H = g.standard_normal((n, n))
    X0 = H @ H.T / n
    K = g.standard_normal((n, n))
    C = ((K + K.T) / (2.0 * math.sqrt(n))).astype(dtype)
    b = np.array([float(np.sum(A[i].astype(np.float64) * X0)) for i in range(m)])
    y0 = g.standard_normal(m)
    return C, A, b, y0


def sparse_symmetric(n: int, per_row: int, seed: int, dtype=np.float64):
    """Sparse symmetric stand-in for the paper's sparse benchmark matrices (Sec. 4, Table 1,
    which are not available here): off-diagonal pattern of about per_row random entries per row
    (N(0,1) / sqrt(per_row), symmetrised), diagonal with 5% of its entries decaying from 10 to
    1e-4 and the rest uniform in [-1, 0], the spectral character of the large dense stand-in.
    Returns (row_ptr int32 (n+1), col_idx int32, vals (dtype)) in CSR form with both triangles
    stored, columns sorted within each row, and the same matrix dense in float64 (from the
    stored values)."""
    import scipy.sparse as sp
    g = _rng(seed)
    half = max(1, per_row // 2)
    rows = np.repeat(np.arange(n), half)
    cols = g.integers(0, n, size=n * half)
    vals = g.standard_normal(n * half) / math.sqrt(per_row)
    S = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    n_pos = max(1, int(round(0.05 * n)))
    d = np.concatenate([10.0 * 10.0 ** (-5.0 * np.arange(n_pos) / max(n_pos - 1, 1)), -g.random(n - n_pos)])
    d = d[g.permutation(n)]
    A = ((S + S.T) * 0.5 + sp.diags(d)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    vals = A.data.astype(dtype)
    dense = sp.csr_matrix((vals.astype(np.float64), A.indices, A.indptr), shape=(n, n)).toarray()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), vals, dense
