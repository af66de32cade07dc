"""Pins of the oracle's level ramp (BFMG, Alg. 4; oracle/bmg.py level_ramp).

The continuum eigenvalues of the Laplace-Beltrami operator on the unit sphere
are l (l + 1) with multiplicity 2 l + 1, so the error of a level's eigenvalue
approximation is known in closed form.  P1 elements converge as O(h^2), i.e.
O(N^-1): the rate r of |lambda - lambda_l| ~ N_l^-r is 1 (the a priori
estimate of Sec. 2.2, Lemma 2.2), which Table 1 (lambda = 2, 6, 12, fixed shift) and
Table 2 (lambda = 20, adaptive shift) report for the one-pass BFMG.  The
ramp's values are further pinned against each level's own discrete
eigenvalues from a dense LAPACK eigensolve: one cycle per level must bring the
approximation to the level's discretisation accuracy.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bmg, reference

# index ranges of the multiplets l = 1, 2, 3 among the 16 smallest eigenvalues
MULTIPLETS = [(2.0, slice(1, 4)), (6.0, slice(4, 9)), (12.0, slice(9, 16))]


@pytest.fixture(scope="module")
def sphere6():
    return bmg.build_levels("sphere", 6)


def _rates(err, n):
    return np.log(err[:-1] / err[1:]) / np.log(n[1:] / n[:-1])


@pytest.mark.parametrize("smoother,nu", [("gs", (2, 2)), ("gs", (1, 0)), ("jacobi", (2, 2))])
def test_one_pass_rates_table1(sphere6, smoother, nu):
    # 16 smallest pairs (0, the l = 1, 2, 3 multiplets), 20 vectors, one cycle
    # per level: the error of each multiplet's mean against l (l + 1) falls by
    # 4x per level (r = 1) from level 3 on
    lv = sphere6
    ev, U, info = bmg.solve(lv, 16, 0.0, 1e-8, m=20, smoother=smoother, nu1=nu[0], nu2=nu[1],
                            ramp_cycles=1, max_cycles=1)
    rows = info["ramp_evals"]
    assert info["ramp_start"] == 1  # 42 vertices >= 2 m
    assert np.all(np.isnan(rows[0])) and np.all(np.isfinite(rows[1:]))
    np.testing.assert_array_equal(rows[-1], ev)
    n = np.array([l.n for l in lv], dtype=np.float64)
    for lam, sl in MULTIPLETS:
        err = np.abs(rows[:, sl].mean(axis=1) - lam)
        r = _rates(err[2:], n[2:])  # levels 2 -> 3 ... 5 -> 6
        assert np.all(r > 0.97) and np.all(r < 1.08), (lam, r)
    assert abs(rows[-1, 0]) < 1e-10  # the constant mode


def test_one_pass_reaches_each_levels_discrete_eigenvalues(sphere6):
    # the value recorded after level l is within a small fraction of that
    # level's discretisation error from the exact discrete eigenvalue of level
    # l: 5 % on level 2 (the first level after the start), 1 % from level 3
    # on, where the prolongated block is already close
    lv = sphere6
    ev, U, info = bmg.solve(lv, 16, 0.0, 1e-8, m=20, smoother="gs", ramp_cycles=1, max_cycles=1)
    rows = info["ramp_evals"]
    for l in range(2, 6):
        # the level's exact discrete eigenvalues: dense on the small levels,
        # ARPACK shift-invert (the same values to 1e-12) on the larger ones
        if lv[l].n <= 3000:
            d = sla.eigh(lv[l].A.toarray(), lv[l].M.toarray(), eigvals_only=True, subset_by_index=[0, 15])
        else:
            d = reference.discrete_eigs(lv[l].A, lv[l].M, 16, 0.0)[0]
        for lam, sl in MULTIPLETS:
            gap = np.abs(rows[l, sl] - d[sl])
            assert np.all(gap <= (0.05 if l == 2 else 0.01) * np.abs(d[sl] - lam)), (l, lam, gap)
    # level 1 (the start level): its exact eigenpairs
    d1 = sla.eigh(lv[1].A.toarray(), lv[1].M.toarray(), eigvals_only=True)
    np.testing.assert_allclose(rows[1], d1[:16], rtol=1e-12, atol=1e-12)


def test_shifted_one_pass_rate_table2(sphere6):
    # the l = 4 multiplet (lambda = 20, 9 pairs) with the interior shift 20:
    # r = 1 with the adaptive shifts; the fixed-shift enriched ramp does not
    # converge to the multiplet (its recorded spread blows up)
    lv = sphere6
    n = np.array([l.n for l in lv], dtype=np.float64)
    ev, U, info = bmg.solve(lv, 9, 20.0, 1e-8, m=16, smoother="gs", ramp_cycles=1, max_cycles=1)
    rows = info["ramp_evals"]
    assert info["scheme"] == "shifted" and info["ramp_start"] == info["l_c"] == 2
    err = np.abs(rows[2:].mean(axis=1) - 20.0)
    r = _rates(err, n[2:])
    assert np.all(r > 0.97) and np.all(r < 1.08), r
    assert np.ptp(rows[-1]) < 1e-3  # the nine values of the multiplet stay together
    ev, U, info = bmg.solve(lv, 9, 20.0, 1e-8, m=16, smoother="gs", ramp_cycles=1, max_cycles=1,
                            scheme="enriched")
    assert np.ptp(info["ramp_evals"][-1]) > 1.0


def test_ramp_then_converge_matches_arpack(sphere6):
    # the ramp as the start of a full solve: the same certified pairs
    lv = sphere6[:6]
    L = lv[-1]
    ref_ev, ref_U = reference.discrete_eigs(L.A, L.M, 20, 0.0)
    ev0, U0, info0 = bmg.solve(lv, 16, 0.0, 1e-8, m=20, smoother="gs")
    ev, U, info = bmg.solve(lv, 16, 0.0, 1e-8, m=20, smoother="gs", ramp_cycles=1)
    assert info["converged"] and info0["converged"]
    rel, sine = reference.compare(ev, U, ref_ev[:16], ref_U[:, :16], L.M, ref_ev, ref_U)
    assert rel < 1e-9 and sine < 1e-6
    # starting from the prolongated level-4 pairs saves cycles on level L
    assert info["cycles"] < info0["cycles"], (info["cycles"], info0["cycles"])


def test_ramp_level_default_and_limits():
    lv = bmg.build_levels("sphere", 3)
    assert bmg.ramp_start_level(lv, 20, 0) == 1   # 42 >= 40
    assert bmg.ramp_start_level(lv, 24, 0) == 2   # 42 < 48 <= 162
    assert bmg.ramp_start_level(lv, 20, 2) == 2   # never below l_c
    assert bmg.ramp_start_level(lv, 400, 0) == 3  # the finest level when none holds 2 m
    # starting on the finest level: its exact pairs, certified at cycle 0
    ev, U, info = bmg.solve(lv, 9, 0.0, 1e-8, m=12, ramp_cycles=1, ramp_level=3)
    assert info["converged"] and info["cycles"] == 0
    d = sla.eigh(lv[3].A.toarray(), lv[3].M.toarray(), eigvals_only=True, subset_by_index=[0, 8])
    np.testing.assert_allclose(ev, d, rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        bmg.solve(lv, 9, 0.0, 1e-8, m=12, ramp_cycles=1, ramp_level=4)
