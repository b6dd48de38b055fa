"""Pins for the FP64 oracle of the randomized PSD projection.

Each check ties the oracle to something other than itself: a value or claim
printed in the paper (tests/golden/worked_examples.json), a closed form, a
theorem of the paper, an independent library routine for a special case, or
brute force at tiny sizes.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import bounds, philox, rnla

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def sym_from(lam, seed):
    U = workloads.haar_orthogonal(len(lam), seed)
    return workloads.from_spectrum(U, np.asarray(lam, float)), U


def closed_form_plus(U, lam):
    return (U * np.maximum(lam, 0.0)[None, :]) @ U.T


# ---------------------------------------------------------------- Thm 1
def test_exact_projection_closed_form():
    lam = workloads.spectrum_small(96, 12, 5)
    A, U = sym_from(lam, 5)
    assert np.allclose(rnla.exact_projection(A), closed_form_plus(U, lam), atol=1e-13, rtol=0)


def test_exact_projection_distance_is_negative_part():
    """Thm 1: ||A - A_+||_F = ||lambda_-||_2 and A_+ is the nearest PSD matrix."""
    lam = workloads.spectrum_medium(80, 10, 2)
    A, _ = sym_from(lam, 2)
    Ap = rnla.exact_projection(A)
    assert abs(np.linalg.norm(A - Ap) - np.linalg.norm(np.minimum(lam, 0))) < 1e-12
    rng = np.random.default_rng(0)
    for _ in range(20):               # any other PSD matrix is farther away
        G = rng.standard_normal((80, 6))
        Y = Ap + 0.01 * G @ G.T
        assert np.linalg.norm(A - Y) >= np.linalg.norm(A - Ap)


def test_polar_form():
    """Eq. (polar form, Prop. 1 proof): X_+ = (X + (X^T X)^{1/2}) / 2 via scipy's sqrtm."""
    rng = np.random.default_rng(1)
    lam = np.concatenate([rng.uniform(0.5, 2, 20), -rng.uniform(0.5, 2, 20)])
    A, _ = sym_from(lam, 3)
    polar = 0.5 * (A + np.real(sla.sqrtm(A.T @ A)))
    assert np.allclose(rnla.exact_projection(A), polar, atol=1e-10)


def test_fig2_norm_comparison():
    """Fig. 2: the Frobenius norm is non-expansive for every d; the spectral norm is not."""
    g = GOLD["fig2"]
    A = np.array(g["A"])
    Ap = rnla.exact_projection(A)
    spectral_ok = []
    for d in np.linspace(*g["d_range"], 2001):
        B = np.array([[0.0, g["B_offdiag"]], [g["B_offdiag"], d]])
        Bp = rnla.exact_projection(B)
        assert np.linalg.norm(Ap - Bp) <= np.linalg.norm(A - B) + 1e-9
        spectral_ok.append(np.linalg.norm(Ap - Bp, 2) <= np.linalg.norm(A - B, 2) + 1e-9)
    assert all(spectral_ok) == g["spectral_nonexpansive_for_all_d"]


# ---------------------------------------------------------------- Counterexample 1
def test_cex1_values():
    g = GOLD["cex1"]
    X = np.diag(g["X_diag"])
    assert np.allclose(rnla.exact_projection(X), np.diag(g["X_plus_diag"]), atol=1e-15)
    assert np.allclose(rnla.exact_projection(np.diag(g["best_rank1_diag"])),
                       np.diag(g["best_rank1_projection_diag"]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cex1_plain_vs_scaled(seed):
    """Cex. 1 with k=1, l=0: the plain sketch locks onto the -3 direction (projection 0);
    the scaled sketch with alpha = 3 locks onto the +1 direction (projection X_+)."""
    g = GOLD["cex1"]
    X = np.diag(g["X_diag"])
    Xp = np.diag(g["X_plus_diag"])
    plain = rnla.ran_proj(X, 1, 0, 5, seed)
    assert np.array_equal(plain.P, np.zeros((3, 3)))
    scal = rnla.ran_proj_scal(X, 1, 0, 5, g["alpha"], seed)
    assert np.linalg.norm(scal.P - Xp) < 1e-5


# ---------------------------------------------------------------- Alg. 1 range
@pytest.mark.parametrize("q", [0, 1, 2])
def test_range_finder_matches_printed_form(q):
    """Reading R1 (orthonormalise after every product) spans the same range as the
    printed Alg. 1, orth((X X^T)^q X Omega), and as an SVD-based orth of it."""
    lam = np.concatenate([np.linspace(2.0, 1.0, 10), np.linspace(0.3, -0.3, 70)])
    X, _ = sym_from(lam, 11)
    Om = philox.test_matrix(4, 80, 10)
    Q = rnla.range_finder(X, Om, q)
    Ql = rnla.range_finder_literal(X, Om, q)
    W = np.linalg.matrix_power(X, 2 * q + 1) @ Om
    Qs = sla.orth(W)
    assert np.allclose(Q.T @ Q, np.eye(10), atol=1e-13)
    assert np.linalg.norm(Q @ Q.T - Ql @ Ql.T) < 1e-9
    assert np.linalg.norm(Q @ Q.T - Qs @ Qs.T) < 1e-9


def test_only_the_range_matters():
    """Lemma 'interchange' (appendix): the output depends on range(Q) only, so any
    invertible recombination of the test vectors gives the same projection."""
    lam = workloads.spectrum_small(100, 12, 3)
    X, _ = sym_from(lam, 3)
    Om = philox.test_matrix(0, 100, 20)
    G = np.random.default_rng(5).standard_normal((20, 20)) + 3 * np.eye(20)
    a = rnla.ran_proj(X, 15, 5, 1, Omega=Om)
    b = rnla.ran_proj(X, 15, 5, 1, Omega=Om @ G)
    assert np.linalg.norm(a.P - b.P) < 1e-11 * np.linalg.norm(a.P)


# ---------------------------------------------------------------- Alg. 2 / Alg. 3 identities
@pytest.mark.parametrize("q", [0, 1])
def test_plain_equals_projection_of_compressed(q):
    """Alg. 2 output = (Q Q^T X Q Q^T)_+ (interchange lemma), checked with a full n x n eig."""
    lam = workloads.spectrum_medium(90, 15, 4)
    X, _ = sym_from(lam, 4)
    res = rnla.ran_proj(X, 12, 6, q, seed=2)
    Q = res.Q
    Xhat = Q @ Q.T @ X @ Q @ Q.T
    d, U = np.linalg.eigh(Xhat)
    ref = (U * np.maximum(d, 0)) @ U.T
    assert np.linalg.norm(res.P - ref) < 1e-12 * max(1.0, np.linalg.norm(ref))


@pytest.mark.parametrize("alpha", [0.5, 1.7])
def test_scaled_equals_lemma3(alpha):
    """Lemma 3: Alg. 3 output = alpha (Q Q^T B Q Q^T - I)_+ with B = (X + alpha I)/alpha."""
    lam = workloads.spectrum_small(70, 20, 6)
    X, _ = sym_from(lam, 6)
    res = rnla.ran_proj_scal(X, 10, 5, 1, alpha, seed=3)
    Q = res.Q
    B = (X + alpha * np.eye(70)) / alpha
    M = Q @ Q.T @ B @ Q @ Q.T - np.eye(70)
    d, U = np.linalg.eigh(M)
    ref = alpha * (U * np.maximum(d, 0)) @ U.T
    assert np.linalg.norm(res.P - ref) < 1e-12 * max(1.0, np.linalg.norm(ref))


def test_lemma2_spectrum_of_B():
    """Lemma 2: with alpha = |lambda_min|, B = (X + alpha I)/alpha is PSD with eigenvalues (lambda+alpha)/alpha."""
    lam = workloads.spectrum_small(50, 8, 7)
    X, _ = sym_from(lam, 7)
    alpha = abs(lam.min())
    B = (X + alpha * np.eye(50)) / alpha
    assert np.allclose(np.sort(np.linalg.eigvalsh(B)), np.sort((lam + alpha) / alpha), atol=1e-12)


# ---------------------------------------------------------------- exact recovery
@pytest.mark.parametrize("q", [0, 1, 2])
def test_plain_exact_recovery_low_rank(q):
    """rank(X) <= k+l: the sketch captures range(X) and Alg. 2 returns X_+ exactly."""
    rng = np.random.default_rng(q)
    lam = np.zeros(120)
    lam[:15] = rng.uniform(0.1, 3.0, 15)
    lam[15:30] = -rng.uniform(0.1, 3.0, 15)
    X, U = sym_from(lam, 20 + q)
    res = rnla.ran_proj(X, 30, 5, q, seed=q)
    Xp = closed_form_plus(U, lam)
    assert np.linalg.norm(res.P - Xp) < 1e-12 * np.linalg.norm(Xp)


def test_scaled_exact_recovery():
    """Remark after Prop. 2: lambda_i + alpha = 0 beyond the sketch width gives zero error."""
    rng = np.random.default_rng(3)
    alpha = 2.0
    lam = np.full(120, -alpha)
    lam[:25] = rng.uniform(-1.5, 3.0, 25)
    X, U = sym_from(lam, 33)
    res = rnla.ran_proj_scal(X, 25, 5, 1, alpha, seed=1)
    Xp = closed_form_plus(U, lam)
    assert np.linalg.norm(res.P - Xp) < 1e-12 * np.linalg.norm(Xp)


def test_full_width_is_exact():
    """k + l = n: Q is square orthogonal and both variants return X_+."""
    lam = workloads.spectrum_small(40, 7, 8)
    X, U = sym_from(lam, 8)
    Xp = closed_form_plus(U, lam)
    assert np.linalg.norm(rnla.ran_proj(X, 30, 10, 0).P - Xp) < 1e-12 * np.linalg.norm(Xp)
    assert np.linalg.norm(rnla.ran_proj_scal(X, 30, 10, 0, 0.3).P - Xp) < 1e-12 * np.linalg.norm(Xp)


# ---------------------------------------------------------------- properties of the output
def test_output_symmetric_psd_idempotent():
    lam = workloads.spectrum_small(150, 20, 9)
    X, U = sym_from(lam, 9)
    P = rnla.ran_proj(X, 20, 10, 1, seed=4).P
    assert np.linalg.norm(P - P.T) < 1e-14 * np.linalg.norm(P)
    assert np.linalg.eigvalsh(P).min() > -1e-13 * np.linalg.norm(P)
    # rank(P) <= k+l, so projecting P again with the same width returns P
    P2 = rnla.ran_proj(P, 20, 10, 1, seed=5).P
    assert np.linalg.norm(P2 - P) < 1e-11 * np.linalg.norm(P)


@pytest.mark.parametrize("variant", ["plain", "scaled"])
def test_negative_definite_projects_to_zero(variant):
    """X negative definite: X_+ = 0, and every Ritz value is negative, so the clamps of Alg. 2
    (max(d, 0)) and Alg. 3 (max(d, 1) - 1 with d = lambda/alpha + 1 < 1) keep nothing."""
    lam = -np.linspace(0.1, 1.0, 120)
    X, _ = sym_from(lam, 31)
    res = rnla.project(X, 15, 10, 1, variant, seed=6)
    assert res.r_plus == 0
    assert not res.P.any()
    assert np.all(res.evals < (1.0 if variant == "scaled" else 0.0))


def test_obtuse_angle_inequality():
    """Projection onto the convex PSD cone: ||X_+ - P||^2 <= ||X - P||^2 - ||X - X_+||^2 for PSD P."""
    lam = workloads.spectrum_medium(120, 20, 10)
    X, U = sym_from(lam, 10)
    Xp = closed_form_plus(U, lam)
    for variant in ("plain", "scaled"):
        P = rnla.project(X, 15, 5, 1, variant, seed=6, alpha=abs(lam.min())).P
        lhs = np.linalg.norm(Xp - P) ** 2
        rhs = np.linalg.norm(X - P) ** 2 - np.linalg.norm(X - Xp) ** 2
        assert lhs <= rhs + 1e-10


# ---------------------------------------------------------------- Alg. 4 / Alg. 5
@pytest.mark.parametrize("lam,expect", [
    ([5.0, 4.0, 1.0, -0.5, -3.0], 3.0),      # sigma_1 is the largest eigenvalue (case 2 of the lemma)
    ([1.0, 0.5, -2.0, -4.0], 4.0),            # sigma_1 is |lambda_min| (case 1)
    (GOLD["cex1"]["X_diag"], GOLD["cex1"]["alpha"]),
])
def test_min_eig_lemma(lam, expect):
    """Lemma (appendix): |lambda_min| = |sigma_1(X - sigma_1 I) - sigma_1(X)|; Alg. 5 converges to it."""
    lam = np.asarray(lam, float)
    X, _ = sym_from(lam, 12)
    alpha, s1, s2 = rnla.min_eig(X, 400, seed=1)
    assert abs(s1 - np.abs(lam).max()) < 1e-10
    assert abs(alpha - expect) < 1e-8


def test_power_iteration_rate():
    """Alg. 4 on a matrix with |lambda_2/lambda_1| = 1/2: error decays like 4^-N."""
    lam = np.array([4.0, -2.0, 1.0, 0.5, 0.1])
    X, _ = sym_from(lam, 13)
    v0 = philox.gaussian(0, 1, 5)
    errs = [abs(rnla.power_iteration(X, N, v0) - 4.0) for N in (5, 10, 20)]
    assert errs[2] < 1e-9 and errs[1] < errs[0]


def test_cor2_alpha_and_bounds():
    """Cor. 2: alpha = beta1 for its matrix class, and the scaled Frobenius bound is smaller at k = n/2,
    with both eps1 values equal to the closed forms written in its proof."""
    g = GOLD["cor2"]
    b1, b2, b3, b4 = g["beta"]
    n, l = 200, g["l"]
    lam = workloads.cor2_spectrum(n, g["beta"])
    X, _ = sym_from(lam, 14)
    alpha, _, _ = rnla.min_eig(X, 60, seed=2)
    assert abs(alpha - g["alpha"]) < 1e-8
    assert (b1 - b2) ** 2 < b2 ** 2 + b4 ** 2
    e_scaled = bounds.eps1(lam + g["alpha"], n // 2, l)
    e_plain = bounds.eps1(np.abs(lam), n // 2, l)
    fac = math.sqrt(1 + n / (2 * (l - 1)))
    assert abs(e_scaled - fac * math.sqrt(n / 4 * (b1 - b2) ** 2)) < 1e-9
    assert abs(e_plain - fac * math.sqrt(n / 4 * (b2 ** 2 + b4 ** 2))) < 1e-9
    assert e_scaled < e_plain


def test_example1_scaled_wins_for_large_k():
    """Example 1 / Fig. 4: on the Cor. 2 class the scaled projection is the more accurate one once k > n/4."""
    g = GOLD["cor2"]
    n = 200
    lam = workloads.cor2_spectrum(n, g["beta"])
    X, U = sym_from(lam, 15)
    Xp = closed_form_plus(U, lam)
    k = 3 * n // 8
    e_plain, e_scal = [], []
    for s in range(3):
        e_plain.append(np.linalg.norm(rnla.project(X, k, g["l"], g["q"], "plain", seed=s).P - Xp))
        e_scal.append(np.linalg.norm(rnla.project(X, k, g["l"], g["q"], "scaled", seed=s,
                                                  alpha_iters=10).P - Xp))
    assert np.mean(e_scal) < np.mean(e_plain)


@pytest.mark.parametrize("variant", ["plain", "scaled"])
def test_expected_error_bounds(variant):
    """Cor. 1 / Prop. 2 (q = 0): the seed-averaged Frobenius and spectral errors respect the bounds."""
    n, k, l = 300, 20, 6
    lam = workloads.spectrum_medium(n, 40, 16)
    X, U = sym_from(lam, 16)
    Xp = closed_form_plus(U, lam)
    alpha = abs(lam.min())
    fro, spec = [], []
    for s in range(8):
        P = rnla.project(X, k, l, 0, variant, seed=s, alpha=alpha).P
        fro.append(np.linalg.norm(Xp - P))
        spec.append(np.linalg.norm(Xp - P, 2))
    if variant == "plain":
        bf, bs = bounds.cor1_frobenius(lam, k, l), bounds.cor1_spectral(lam, k, l, 0)
    else:
        bf, bs = bounds.prop2_frobenius(lam, alpha, k, l), bounds.prop2_spectral(lam, alpha, k, l, 0)
    assert np.mean(fro) <= bf
    assert np.mean(spec) <= bs


def test_lemma1_bounds():
    """Lemma 1: ||X - QQ^T X QQ^T|| <= 2 eps_1 (spectral) and <= sqrt(2) eps_2 (Frobenius)."""
    lam = workloads.spectrum_medium(100, 10, 17)
    X, _ = sym_from(lam, 17)
    Q = rnla.ran_proj(X, 10, 5, 0, seed=1).Q
    R = X - Q @ Q.T @ X
    Xh = Q @ Q.T @ X @ Q @ Q.T
    assert np.linalg.norm(X - Xh, 2) <= 2 * np.linalg.norm(R, 2) + 1e-12
    assert np.linalg.norm(X - Xh) <= math.sqrt(2) * np.linalg.norm(R) + 1e-12


def test_parity_metric_floor():
    P_ref = np.zeros((4, 4))
    A = np.eye(4)
    assert rnla.parity_error(np.full((4, 4), 1e-3), P_ref, np.linalg.norm(A)) == pytest.approx(
        np.linalg.norm(np.full((4, 4), 1e-3)) / (1e-2 * 2.0))


def test_entries_match_full_rebuild():
    lam = workloads.spectrum_small(64, 8, 18)
    X, _ = sym_from(lam, 18)
    res = rnla.ran_proj(X, 10, 4, 0)
    rows = np.array([0, 5, 63, 17])
    cols = np.array([3, 5, 0, 40])
    assert np.allclose(res.entries(rows, cols), res.P[rows, cols], atol=1e-15)
