"""Pins for the structured (subsampled randomized Hadamard) test matrix of the oracle."""
import numpy as np
import pytest

import workloads
from oracle import rnla, srht


@pytest.mark.parametrize("m", range(1, 11))
def test_column_permutation_is_a_bijection(m):
    """pi is a permutation of [0, 2^m) for even and odd m (odd m walks the cycle of a Feistel
    network on m + 1 bits), so distinct j select distinct columns."""
    N = 1 << m
    perm = [srht.permute(11, j, m) for j in range(N)]
    assert sorted(perm) == list(range(N))


def test_hadamard_against_sylvester_construction():
    """(-1)^popcount(i & s) equals the Sylvester construction H_{2N} = [[H, H], [H, -H]]."""
    H = np.array([[1.0]])
    for _ in range(5):
        H = np.block([[H, H], [H, -H]])
    i, s = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    assert np.array_equal(srht.hadamard_entry(i, s), H)


@pytest.mark.parametrize("n,r", [(64, 20), (256, 100), (2, 2)])
def test_power_of_two_order_gives_orthogonal_columns(n, r):
    """n = N: the columns are distinct columns of D H, so Omega^T Omega = n I exactly."""
    Om = srht.test_matrix(5, n, r)
    assert np.array_equal(Om.T @ Om, n * np.eye(r))
    assert set(np.unique(Om)) <= {-1.0, 1.0}


def test_signs_are_balanced():
    d = srht.signs(9, 200000)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 0.01


def test_selected_columns_spread_over_the_transform():
    """The selected columns of a 2^14-point transform fall evenly into 16 bins (chi-square)."""
    s = srht.columns(21, 16384, 2000)
    counts = np.bincount(s // 1024, minlength=16)
    chi2 = np.sum((counts - 125.0) ** 2 / 125.0)
    assert len(set(s.tolist())) == 2000
    assert chi2 < 40.0          # 15 degrees of freedom: P(chi2 > 40) < 1e-3


def test_exact_recovery_with_structured_sketch():
    """rank(A) <= k + p: the structured sketch spans range(A) and the projection is A_+."""
    n = 300
    lam = np.zeros(n)
    lam[:10] = np.linspace(1.0, 2.0, 10)
    lam[10:20] = -np.linspace(0.5, 1.5, 10)
    U = workloads.haar_orthogonal(n, 4)
    A = workloads.from_spectrum(U, lam)
    res = rnla.project(A, 20, 6, 0, "plain", seed=2, sketch="srht")
    Ap = (U * np.maximum(lam, 0)) @ U.T
    assert np.linalg.norm(res.P - Ap) < 1e-12 * np.linalg.norm(Ap)
    assert not np.allclose(res.Q, rnla.project(A, 20, 6, 0, "plain", seed=2).Q)   # a different sketch


def test_structured_sketch_error_is_comparable_to_gaussian():
    """On a decaying spectrum the two sketches give errors of the same order (the footnote's
    'perform exceptionally well in practice')."""
    n = 512
    lam = workloads.spectrum_small(n, 32, 3)
    U = workloads.haar_orthogonal(n, 3)
    A = workloads.from_spectrum(U, lam)
    Ap = (U * np.maximum(lam, 0)) @ U.T
    e = {sk: np.linalg.norm(rnla.project(A, 40, 10, 1, "plain", seed=1, sketch=sk).P - Ap) / np.linalg.norm(Ap)
         for sk in ("gaussian", "srht")}
    assert e["srht"] < 3 * e["gaussian"] + 1e-3 and e["gaussian"] < 3 * e["srht"] + 1e-3
