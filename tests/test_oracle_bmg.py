"""Pins of the oracle's BMG iteration against the plain definition of the result."""
import numpy as np
import pytest

from oracle import bmg, reference


@pytest.fixture(scope="module")
def c1_levels():
    return bmg.build_levels("sphere", 3)


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
def test_c1_matches_dense_eigensolve(c1_levels, smoother):
    lv = c1_levels[-1]
    ev, U, info = bmg.solve(c1_levels, 9, 0.0, 1e-8, m=12, smoother=smoother)
    assert info["converged"]
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 9, 0.0)
    rel, sine = reference.compare(ev, U, ref_ev, ref_U, lv.M)
    assert rel < 1e-9 and sine < 1e-6
    G = U.T @ (lv.M @ U)
    assert np.abs(G - np.eye(9)).max() < 1e-12
    # sign convention: largest-magnitude entry of each vector is positive
    assert np.all(U[np.argmax(np.abs(U), axis=0), np.arange(9)] > 0)


def test_ritz_values_are_upper_bounds(c1_levels):
    # exact Rayleigh-Ritz with sigma = 0: the j-th Ritz value is >= the j-th eigenvalue
    lv = c1_levels[-1]
    ref_ev, _ = reference.discrete_eigs(lv.A, lv.M, 12, 0.0)
    _, _, info = bmg.solve(c1_levels, 9, 0.0, 1e-8, m=12, history=True)
    for theta, _, _ in info["history"]:
        assert np.all(theta >= ref_ev - 1e-11)


def test_certificates_bound_true_errors(c1_levels):
    lv = c1_levels[-1]
    ev, U, info = bmg.solve(c1_levels, 9, 0.0, 1e-6, m=12)
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 9, 0.0)
    rel, sine = reference.compare(ev, U, ref_ev, ref_U, lv.M)
    # stopping rule guarantees rel <= 0.1 tol (Kato-Temple) and sine <= 1e-7 (Davis-Kahan)
    assert rel <= 0.1 * 1e-6 + 1e-15 and sine <= 2e-7


def test_small_shift_interior_cluster():
    levels = bmg.build_levels("sphere", 4)
    lv = levels[-1]
    # the 5 eigenpairs nearest sigma = 6 are the l = 2 cluster
    ev, U, info = bmg.solve(levels, 5, 6.0, 1e-8, m=12)
    assert info["converged"]
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 5, 6.0)
    rel, sine = reference.compare(ev, U, ref_ev, ref_U, lv.M)
    assert rel < 1e-9 and sine < 1e-6


def test_cut_cluster_containment(c1_levels):
    # k = 6 cuts the l = 2 cluster: the returned 2 vectors lie in the full eigenspace
    lv = c1_levels[-1]
    ev, U, info = bmg.solve(c1_levels, 6, 0.0, 1e-8, m=12)
    full_ev, full_U = reference.discrete_eigs(lv.A, lv.M, 9, 0.0)
    rel, sine = reference.compare(ev, U, full_ev[:6], full_U[:, :6], lv.M, full_ev, full_U)
    assert rel < 1e-9 and sine < 1e-6


def test_default_block_width():
    assert [bmg.default_m(k, s) for k, s in [(9, 0), (25, 0), (16, 100), (64, 0)]] == [12, 32, 24, 80]


def test_coarsest_level_rule():
    levels = bmg.build_levels("sphere", 4)
    assert bmg.coarsest_level(levels, 0.0) == 0
    # n_W(30) = area * 30 / (4 pi) ~ 30 -> needs N_l >= 240 -> level 3 (642 vertices)
    assert bmg.coarsest_level(levels, 30.0) == 3
