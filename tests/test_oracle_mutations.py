"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake -- a dropped term or factor, a wrong sign, a wrong
index or exponent, a wrong operand -- in a fresh copy of one oracle module, points the pin
tests at the copy, and requires that at least one pin fails.  The committed oracle itself
is never modified: the copies live in a temporary directory and are imported under a
package name of their own.

Mistakes that no CPU pin can see are left out on purpose and named here: the rounding of
the test matrix to the storage precision (reading R7) and the cos/sin assignment of the
Box-Muller pair change no statistical or algebraic property the CPU pins test; the GPU
parity tests, which compare against an independent implementation, cover them.  A mistake
that only loosens a bound (a larger constant in the spectral bounds of Cor. 1 / Prop. 2)
cannot fail an expected-error inequality either; the exponent and index of eps1/eps2 are
pinned by identities instead.
"""
import importlib.util
import os
import shutil
import sys
import tempfile

import pytest

import test_oracle_bounds as TB
import test_oracle_method as TM
import test_oracle_philox as TP
import test_oracle_sdls as TS
import test_oracle_srht as TR

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def _load_mutant(fname, old, new, tag):
    """Copy oracle/ to a temporary package with one textual change in `fname`; import it."""
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    pkg = f"oracle_mut_{tag}"
    dst = os.path.join(d, pkg)
    shutil.copytree(ORACLE, dst, ignore=shutil.ignore_patterns("__pycache__"))
    path = os.path.join(dst, fname)
    src = open(path).read()
    assert src.count(old) == 1, f"mutation anchor not unique in {fname}: {old!r}"
    open(path, "w").write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(pkg, os.path.join(dst, "__init__.py"),
                                                  submodule_search_locations=[dst])
    mod = importlib.util.module_from_spec(spec)
    sys.modules[pkg] = mod
    spec.loader.exec_module(mod)
    return mod, d


# pins, by name: each a call of a committed pin test with fixed parameters
PINS = {
    "cex1_plain_vs_scaled": lambda: TM.test_cex1_plain_vs_scaled(0),
    "cex1_values": lambda: TM.test_cex1_values(),
    "exact_closed_form": lambda: TM.test_exact_projection_closed_form(),
    "exact_distance": lambda: TM.test_exact_projection_distance_is_negative_part(),
    "range_printed_q1": lambda: TM.test_range_finder_matches_printed_form(1),
    "range_printed_q2": lambda: TM.test_range_finder_matches_printed_form(2),
    "plain_compressed_q1": lambda: TM.test_plain_equals_projection_of_compressed(1),
    "lemma3": lambda: TM.test_scaled_equals_lemma3(1.7),
    "plain_recovery_q1": lambda: TM.test_plain_exact_recovery_low_rank(1),
    "scaled_recovery": lambda: TM.test_scaled_exact_recovery(),
    "full_width": lambda: TM.test_full_width_is_exact(),
    "neg_def_plain": lambda: TM.test_negative_definite_projects_to_zero("plain"),
    "neg_def_scaled": lambda: TM.test_negative_definite_projects_to_zero("scaled"),
    "min_eig_case1": lambda: TM.test_min_eig_lemma([1.0, 0.5, -2.0, -4.0], 4.0),
    "min_eig_case2": lambda: TM.test_min_eig_lemma([5.0, 4.0, 1.0, -0.5, -3.0], 3.0),
    "power_rate": lambda: TM.test_power_iteration_rate(),
    "cor2": lambda: TM.test_cor2_alpha_and_bounds(),
    "parity_floor": lambda: TM.test_parity_metric_floor(),
    "eps2_exponent": lambda: TB.test_eps2_power_exponent(1, 20, 6, 300),
    "eps1_flat": lambda: TB.test_eps1_flat_tail(),
    "proj_errors": lambda: TB.test_projection_errors_exact_eigenvectors([0, 2, 7, 9, 30, 31, 60]),
    "philox_kat0": lambda: TP.test_philox_known_answers(*TP.KAT[0]),
    "philox_kat2": lambda: TP.test_philox_known_answers(*TP.KAT[2]),
    "gauss_stats": lambda: TP.test_gaussian_statistics(),
    "srht_bijection_odd": lambda: TR.test_column_permutation_is_a_bijection(5),
    "srht_bijection_even": lambda: TR.test_column_permutation_is_a_bijection(6),
    "srht_sylvester": lambda: TR.test_hadamard_against_sylvester_construction(),
    "srht_orthogonal": lambda: TR.test_power_of_two_order_gives_orthogonal_columns(64, 20),
    "srht_signs": lambda: TR.test_signs_are_balanced(),
    "srht_recovery": lambda: TR.test_exact_recovery_with_structured_sketch(),
    "sdls_gradient": lambda: TS.test_gradient_is_minus_constraint_residual(),
    "sdls_feasible": lambda: TS.test_exact_gd_reaches_feasibility(),
    "sdls_scalar_root": lambda: TS.test_single_constraint_against_scalar_root(),
    "sdls_hook": lambda: TS.test_randomized_gd_follows_the_projection_it_is_given(),
    "sdls_loop": lambda: TS.test_loop_runs_at_most_m_iterations_and_at_least_one(),
}

# (id, oracle file, text, replacement, pins expected to notice)
MUTANTS = [
    ("plain_no_clamp", "rnla.py", "weights = np.maximum(evals, 0.0)", "weights = evals.copy()",
     ["cex1_plain_vs_scaled", "plain_compressed_q1", "neg_def_plain"]),
    ("plain_clamp_sign", "rnla.py", "weights = np.maximum(evals, 0.0)", "weights = np.maximum(-evals, 0.0)",
     ["cex1_plain_vs_scaled", "plain_compressed_q1", "plain_recovery_q1", "neg_def_plain"]),
    ("scaled_drops_alpha", "rnla.py", "alpha * (np.maximum(evals, 1.0) - 1.0)", "(np.maximum(evals, 1.0) - 1.0)",
     ["lemma3", "scaled_recovery", "full_width"]),
    ("scaled_threshold_zero", "rnla.py", "alpha * (np.maximum(evals, 1.0) - 1.0)", "alpha * np.maximum(evals, 0.0)",
     ["lemma3", "scaled_recovery", "full_width", "neg_def_scaled"]),
    ("B_shift_sign", "rnla.py", "(np.diag(X) + alpha) / alpha", "(np.diag(X) - alpha) / alpha",
     ["lemma3", "cex1_plain_vs_scaled", "scaled_recovery"]),
    ("B_not_scaled", "rnla.py", "B = X / alpha  ", "B = X.copy()  ",
     ["lemma3", "scaled_recovery"]),
    ("power_loop_short", "rnla.py", "    for _ in range(q):\n        Q = orth(X.T @ Q)",
     "    for _ in range(max(q - 1, 0)):\n        Q = orth(X.T @ Q)", ["range_printed_q1", "range_printed_q2"]),
    ("power_missing_orth", "rnla.py", "        Q = orth(X @ Q)\n    return Q", "        Q = X @ Q\n    return Q",
     ["range_printed_q1"]),
    ("compress_wrong_operand", "rnla.py", "C = Q.T @ (X @ Q)  ", "C = Q.T @ (X @ (X @ Q))  ",
     ["plain_compressed_q1", "plain_recovery_q1", "full_width"]),
    ("symmetrise_sign", "rnla.py", "C = 0.5 * (C + C.T)", "C = 0.5 * (C - C.T)",
     ["plain_compressed_q1", "plain_recovery_q1"]),
    ("rebuild_sqrt_weights", "rnla.py", "res.P = (U * weights[None, :]) @ U.T",
     "res.P = (U * np.sqrt(weights)[None, :]) @ U.T", ["plain_recovery_q1", "lemma3", "full_width"]),
    ("power_unnormalised", "rnla.py", "        v = y / nrm\n", "        v = y\n",
     ["min_eig_case1", "min_eig_case2", "power_rate"]),
    ("shift_sign", "rnla.py", "Y[np.diag_indices(n)] -= s1", "Y[np.diag_indices(n)] += s1",
     ["min_eig_case1", "min_eig_case2", "cor2"]),
    ("alpha_combination", "rnla.py", "return abs(s1 - s2), s1, s2", "return abs(s2), s1, s2",
     ["min_eig_case1", "min_eig_case2", "cor2"]),
    ("exact_abs", "rnla.py", "(U * np.maximum(d, 0.0)[None, :]) @ U.T", "(U * np.abs(d)[None, :]) @ U.T",
     ["exact_closed_form", "exact_distance", "cex1_values"]),
    ("parity_floor", "rnla.py", "1e-2 * A_fro", "1e-3 * A_fro", ["parity_floor"]),
    ("e_alg_denominator", "rnla.py", "np.linalg.norm(X_plus - P) / np.linalg.norm(X_plus)",
     "np.linalg.norm(X_plus - P) / np.linalg.norm(P)", ["proj_errors"]),
    ("range_err_denominator", "rnla.py", "np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X)",
     "np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(Q.T @ X)", ["proj_errors"]),
    ("eps2_exponent", "bounds.py", "1.0 / (2 * q + 1)", "1.0 / (q + 1)", ["eps2_exponent"]),
    ("eps1_index", "bounds.py", "s[k:] ** 2", "s[k + 1:] ** 2", ["eps1_flat", "cor2"]),
    ("eps1_factor", "bounds.py", "1.0 + k / (l - 1.0)", "1.0 + k / l", ["eps1_flat", "cor2"]),
    ("philox_multiplier", "philox.py", "M0 = np.uint64(0xD2511F53)", "M0 = np.uint64(0xD2511F57)", ["philox_kat0", "philox_kat2"]),
    ("philox_weyl", "philox.py", "W1 = np.uint32(0xBB67AE85)", "W1 = np.uint32(0xBB67AE84)", ["philox_kat0", "philox_kat2"]),
    ("philox_round_swap", "philox.py", "hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0", "hi0 ^ c1 ^ k0, lo1, hi1 ^ c3 ^ k1, lo0",
     ["philox_kat0", "philox_kat2"]),
    ("box_muller_radius", "philox.py", "np.sqrt(-2.0 * np.log(u1))", "np.sqrt(-np.log(u1))", ["gauss_stats"]),
    ("srht_no_cycle_walk", "srht.py", "    while y >= (1 << m):\n        y = feistel(seed, y, m)\n", "",
     ["srht_bijection_odd"]),
    ("srht_parity", "srht.py", "par ^= v & 1", "par += v & 1", ["srht_sylvester", "srht_orthogonal"]),
    ("srht_feistel_round", "srht.py", "L, R = R, L ^ f", "L, R = R, R ^ f", ["srht_bijection_odd", "srht_bijection_even"]),
    ("srht_sign_bit", "srht.py", "(w[:, 0] & 1)", "(w[:, 0] & 0)", ["srht_signs"]),
    ("srht_not_used", "rnla.py", "        return srht.test_matrix(seed, n, r)", "        return philox.test_matrix(seed, n, r)",
     ["srht_recovery"]),
    ("sdls_update_sign", "sdls.py", "y = y - beta * g  ", "y = y + beta * g  ",
     ["sdls_feasible", "sdls_scalar_root", "sdls_hook"]),
    ("sdls_rho_dropped", "sdls.py", "X = np.asarray(C, np.float64) / rho", "X = np.asarray(C, np.float64)",
     ["sdls_gradient", "sdls_scalar_root"]),
    ("sdls_residual_sign", "sdls.py", "for Ai in A]) - np.asarray(b, np.float64)",
     "for Ai in A]) + np.asarray(b, np.float64)", ["sdls_gradient", "sdls_feasible", "sdls_scalar_root"]),
    ("sdls_seed_offset", "sdls.py", "X_plus = rnla.ran_proj(X, k, p, q, seed=seed + i - 1,",
     "X_plus = rnla.ran_proj(X, k, p, q, seed=seed + i,", ["sdls_hook"]),
    ("sdls_extra_iteration", "sdls.py", "while i < M and", "while i <= M and", ["sdls_loop"]),
]


@pytest.mark.parametrize("mid,fname,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(mid, fname, old, new, pins, monkeypatch):
    mod, tmp = _load_mutant(fname, old, new, mid)
    try:
        for test_mod in (TM, TB):
            monkeypatch.setattr(test_mod, "rnla", mod.rnla)
            monkeypatch.setattr(test_mod, "bounds", mod.bounds)
        for test_mod in (TM, TP):
            monkeypatch.setattr(test_mod, "philox", mod.philox)
        monkeypatch.setattr(TS, "rnla", mod.rnla)
        monkeypatch.setattr(TS, "sdls", mod.sdls)
        monkeypatch.setattr(TR, "rnla", mod.rnla)
        monkeypatch.setattr(TR, "srht", mod.srht)
        caught = []
        for name in pins:
            try:
                PINS[name]()
            except Exception:       # an assertion, or the mutant breaking a computation outright
                caught.append(name)
        assert caught, f"planted mistake {mid!r} passed every pin in {pins}"
    finally:
        sys.modules.pop(f"oracle_mut_{mid}", None)
        shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_copy_passes_every_pin(monkeypatch):
    """The harness itself: an unchanged copy of the oracle passes all the pins used above."""
    mod, tmp = _load_mutant("bounds.py", "import math", "import math", "identity")
    try:
        for test_mod in (TM, TB):
            monkeypatch.setattr(test_mod, "rnla", mod.rnla)
            monkeypatch.setattr(test_mod, "bounds", mod.bounds)
        for test_mod in (TM, TP):
            monkeypatch.setattr(test_mod, "philox", mod.philox)
        monkeypatch.setattr(TS, "rnla", mod.rnla)
        monkeypatch.setattr(TS, "sdls", mod.sdls)
        monkeypatch.setattr(TR, "rnla", mod.rnla)
        monkeypatch.setattr(TR, "srht", mod.srht)
        for name, pin in PINS.items():
            pin()
    finally:
        sys.modules.pop("oracle_mut_identity", None)
        shutil.rmtree(tmp, ignore_errors=True)
