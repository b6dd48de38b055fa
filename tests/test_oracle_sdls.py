"""Pins for the SDLS dual gradient descent oracle (Alg. 6): each check ties it to the
mathematics of the supplementary SDP section rather than to itself."""
import numpy as np
import pytest

import workloads
from oracle import rnla, sdls


def small_problem(n=12, m=3, seed=5):
    return workloads.sdls_problem(n, m, seed)


def test_gradient_is_minus_constraint_residual():
    """The dual function theta(y) = L(X*(y); y) has gradient -(Tr(A_i X*(y)) - b_i)_i (Danskin,
    with X*(y) the exact projection of C/rho + sum y_i A_i): central differences agree."""
    C, A, b, y0 = small_problem()
    rho = 0.7
    y = 0.5 * y0
    g = sdls.constraint_residual(A, b, rnla.exact_projection(sdls.form_x(C, A, y, rho)))
    h = 1e-6
    fd = np.array([(sdls.dual_value(C, A, b, y + h * e, rho) - sdls.dual_value(C, A, b, y - h * e, rho)) / (2 * h)
                   for e in np.eye(len(y))])
    assert np.allclose(fd, -g, rtol=1e-5, atol=1e-7)


def test_dual_function_is_concave():
    C, A, b, y0 = small_problem(seed=6)
    rng = np.random.default_rng(1)
    for _ in range(10):
        u, v = rng.standard_normal(3), rng.standard_normal(3)
        mid = sdls.dual_value(C, A, b, 0.5 * (u + v), 1.0)
        assert mid >= 0.5 * (sdls.dual_value(C, A, b, u, 1.0) + sdls.dual_value(C, A, b, v, 1.0)) - 1e-12


def test_exact_gd_reaches_feasibility():
    """scal = -1 on a feasible instance: the constraint error falls to round-off (Example 3 reports
    2.8e-15 for the deterministic descent)."""
    C, A, b, y0 = small_problem(n=20, m=2, seed=7)
    res = sdls.dual_gd(C, A, b, rho=1.0, k=0, p=0, q=0, N=0, scal=-1, eps=1e-12, beta=0.5, M=5000, y0=y0)
    assert res.history[-1] < 1e-10
    assert res.iters < 5000
    # the primal iterate is PSD and the last step's projection of C/rho + sum y A
    assert np.linalg.eigvalsh(res.X_plus).min() > -1e-12


def test_single_constraint_against_scalar_root():
    """m = 1 with A_1 = I/sqrt(n): X*(y) = (C/rho + y I/sqrt(n))_+, so the optimal y is the root of
    the increasing scalar function t -> Tr((C/rho + t I/sqrt(n))_+)/sqrt(n) - b_1, found here by
    bisection on the eigenvalues of C alone."""
    n, rho = 15, 2.0
    C, _, _, _ = workloads.sdls_problem(n, 1, 8)
    A = (np.eye(n) / np.sqrt(n))[None]
    b = np.array([2.5])
    lam = np.linalg.eigvalsh(C / rho)

    def f(t):
        return np.sum(np.maximum(lam + t / np.sqrt(n), 0.0)) / np.sqrt(n) - b[0]

    lo, hi = -100.0, 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    res = sdls.dual_gd(C, A, b, rho=rho, k=0, p=0, q=0, N=0, scal=-1, eps=1e-13, beta=1.0, M=20000, y0=np.zeros(1))
    # g(y) = Tr(A_1 X*(y)) - b_1 increases with y and the update moves y against g: y -> the root
    assert abs(res.y[0] - lo) < 1e-8


def test_randomized_gd_follows_the_projection_it_is_given():
    """With the projection replaced by the exact one through the test hook, scal = 0 and scal = -1
    give the same iterates; and one step of scal = 0 matches Alg. 2 at seed + 0."""
    C, A, b, y0 = small_problem(n=30, m=2, seed=9)
    r_exact = sdls.dual_gd(C, A, b, 1.0, 0, 0, 0, 0, -1, 1e-12, 0.5, 6, y0)
    r_hook = sdls.dual_gd(C, A, b, 1.0, 5, 5, 1, 10, 0, 1e-12, 0.5, 6, y0,
                          project=lambda X, i: rnla.exact_projection(X))
    assert np.allclose(r_exact.y, r_hook.y, atol=1e-14)
    one = sdls.dual_gd(C, A, b, 1.0, 8, 4, 1, 10, 0, 1e-12, 0.5, 1, y0, seed=3)
    P = rnla.ran_proj(sdls.form_x(C, A, y0, 1.0), 8, 4, 1, seed=3).P
    assert np.allclose(one.y, y0 - 0.5 * sdls.constraint_residual(A, b, P), atol=1e-13)


def test_loop_runs_at_most_m_iterations_and_at_least_one():
    C, A, b, y0 = small_problem(n=10, m=1, seed=10)
    r = sdls.dual_gd(C, A, b, 1.0, 0, 0, 0, 0, -1, 1e30, 0.5, 7, y0)   # eps huge: one iteration
    assert r.iters == 1
    r = sdls.dual_gd(C, A, b, 1.0, 0, 0, 0, 0, -1, 0.0, 0.5, 7, y0)    # eps 0: all M
    assert r.iters == 7


@pytest.mark.parametrize("scal", [0, 1])
def test_randomized_gd_converges_to_a_neighbourhood(scal):
    """Example 3's qualitative claim: the randomized descent settles near the exact one, closer as
    k grows (n = 60, m = 2, q = 6, l = 10)."""
    C, A, b, y0 = small_problem(n=60, m=2, seed=11)
    exact = sdls.dual_gd(C, A, b, 1.0, 0, 0, 0, 0, -1, 1e-12, 0.5, 300, y0)
    errs = []
    for k in (20, 45):
        r = sdls.dual_gd(C, A, b, 1.0, k, 10, 6, 10, scal, 1e-12, 0.5, 100, y0, seed=1)
        errs.append(np.linalg.norm(r.y - exact.y))
    assert errs[1] < errs[0] and errs[1] < 0.1 * np.linalg.norm(exact.y)
