"""Pins of the oracle's interior-shift scheme (oracle/bmg.py, "shifted").

The converged pairs are pinned against the plain definition of the result
(library eigensolvers: ARPACK shift-invert, dense LAPACK), the coarse solve
against a sparse direct solve, the adaptive-shift offsets against the O(h^2)
convergence of a nodal interpolant's Rayleigh quotient, and the coarse-level
rule against hand-computed values.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import bmg, reference

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _nearest(ev, sigma, k):
    return np.sort(np.argsort(np.abs(ev - sigma), kind="stable")[:k])


@pytest.fixture(scope="module")
def ell5():
    return bmg.build_levels("ellipsoid", 5, axes=(1.0, 1.5, 2.0))


@pytest.mark.parametrize("smoother", ["jacobi", "gs"])
def test_ellipsoid_ref5_sigma40_matches_arpack(ell5, smoother):
    # 16 pairs nearest 40 on the 10242-vertex ellipsoid (about 89 eigenvalues below sigma)
    lv = ell5[-1]
    ev, U, info = bmg.solve(ell5, 16, 40.0, 1e-8, m=24, smoother=smoother)
    assert info["converged"] and info["scheme"] == "shifted" and info["l_c"] == 4
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 24, 40.0)
    idx = _nearest(ref_ev, 40.0, 16)
    rel, sine = reference.compare(ev, U, ref_ev[idx], ref_U[:, idx], lv.M, ref_ev, ref_U)
    assert rel < 1e-9 and sine < 1e-6
    assert np.abs(U.T @ (lv.M @ U) - np.eye(16)).max() < 1e-12
    # the level-l_c shift moved up from sigma: coarse levels misplace these
    # eigenvalues (Remark 4.1), and the offset shrinks towards the finest level
    off = info["offsets"]
    assert off[4] > off[5] == 0.0 and off[4] > 0.5


def test_without_adaptive_shift_the_fixed_shift_cycle_stalls(ell5):
    # the same problem with the fixed-shift enriched scheme does not reach the
    # certificate: the reason the shifted scheme exists
    ev, U, info = bmg.solve(ell5, 16, 40.0, 1e-8, m=24, smoother="jacobi", scheme="enriched",
                            max_cycles=40)
    assert not info["converged"]


@pytest.mark.slow
def test_c3_oracle_matches_stored_arpack_eigenvalues():
    # C3: ellipsoid (1, 1.5, 2) refined 7 times, 16 pairs nearest 100, m = 24
    levels = bmg.build_levels("ellipsoid", 7, axes=(1.0, 1.5, 2.0))
    ev, U, info = bmg.solve(levels, 16, 100.0, 1e-8, m=24, smoother="jacobi")
    assert info["converged"] and info["l_c"] == 5
    gold = np.array([float(x) for x in open(os.path.join(GOLDEN, "c3_ellipsoid_ref7_eigs.txt"))
                     if not x.startswith("#")])
    near = gold[_nearest(gold, 100.0, 16)]
    assert np.max(np.abs(ev - near) / np.maximum(np.abs(near), 1.0)) < 1e-9


def test_exact_coarse_level_is_the_fine_eigensolve():
    # l_c = L (the rule asks for a finer level than exists): the start block
    # is the exact fine eigenpairs, certified at cycle 0
    levels = bmg.build_levels("sphere", 3)
    lv = levels[-1]
    ev, U, info = bmg.solve(levels, 8, 150.0, 1e-8)
    assert info["converged"] and info["cycles"] == 0 and info["l_c"] == 3
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 8, 150.0)
    assert np.max(np.abs(ev - ref_ev) / ref_ev) < 1e-12


@pytest.mark.slow
def test_torus_interior_shift():
    levels = bmg.build_levels("torus", 1)
    lv = levels[-1]
    ev, U, info = bmg.solve(levels, 12, 60.0, 1e-8)
    assert info["converged"]
    ref_ev, ref_U = reference.discrete_eigs(lv.A, lv.M, 20, 60.0)
    idx = _nearest(ref_ev, 60.0, 12)
    rel, sine = reference.compare(ev, U, ref_ev[idx], ref_U[:, idx], lv.M, ref_ev, ref_U)
    assert rel < 1e-9 and sine < 1e-6


def test_spectral_coarse_solve_is_the_inverse():
    # with no mode inside the truncation window the coarse solve is
    # (A - s M)^-1, checked against SuperLU
    levels = bmg.build_levels("sphere", 3)
    sh = bmg.ShiftedBMG(levels, 7.3, 8, 2)
    lc = levels[2]
    assert np.all(sh.g != 0.0)
    f = np.random.default_rng(1).standard_normal((lc.n, 3))
    e = sh.vcycle(2, f)
    x = spla.spsolve((lc.A - 7.3 * lc.M).tocsc(), f)
    assert np.max(np.abs(e - x)) < 1e-10 * np.max(np.abs(x))


def test_spectral_truncation_drops_the_modes_near_the_shift():
    levels = bmg.build_levels("sphere", 2)
    lam = bmg.ShiftedBMG(levels, 1.0, 8, 2).lam
    sigma = lam[10] + 0.02  # within 1e-2 sigma of the 11th level-2 eigenvalue
    sh = bmg.ShiftedBMG(levels, sigma, 8, 2)
    near = np.abs(sh.lam - sigma) < 1e-2 * sigma
    assert near.sum() >= 1 and np.all(sh.g[near] == 0.0) and np.all(sh.g[~near] != 0.0)
    # a right-hand side made of those modes (M times them) gets no correction
    f = levels[2].M @ sh.phi[:, near]
    assert np.max(np.abs(sh.vcycle(2, f))) < 1e-12


def test_injected_rayleigh_offsets_converge_at_h2():
    # the coordinate z on the sphere is an l = 1 harmonic (eigenvalue 2); its
    # nodal values on level l are the first N_l entries of the fine vector, so
    # the offsets RQ_l - RQ_L must fall about 4x per level (O(h^2)); reading
    # the wrong rows or a wrong norm breaks this
    levels = bmg.build_levels("sphere", 5)
    z = levels[-1].xyz[:, 2:3].copy()
    lvL = levels[-1]
    th = np.array([float(z[:, 0] @ (lvL.A @ z[:, 0]) / (z[:, 0] @ (lvL.M @ z[:, 0])))])
    off = bmg.injected_rayleigh_offsets(levels, z, th, 1)
    assert off[0] == 0.0 and off[-1] == 0.0  # below l_c and on L: not computed / zero
    err = off[1:5] + (th[0] - 2.0)  # RQ_l - 2, the error against the continuum
    ratios = err[:-1] / err[1:]
    assert np.all(ratios > 3.5) and np.all(ratios < 4.5), (off, ratios)


@pytest.mark.parametrize("kind,nref,axes,sigma,m,want", [
    ("ellipsoid", 7, (1.0, 1.5, 2.0), 100.0, 24, (5, 24)),   # C3
    ("ellipsoid", 5, (1.0, 1.5, 2.0), 40.0, 24, (4, 24)),
    ("ellipsoid", 5, (1.0, 1.5, 2.0), 50.0, 24, (5, 24)),   # level 4 is too coarse at 50: l_c = L
    ("sphere", 4, (1.0, 1.0, 1.0), 6.0, 8, (1, 8)),
    # a small shift with a wide block: the level must hold 2 m eigenpairs (162 >= 96)
    ("sphere", 3, (1.0, 1.0, 1.0), 12.0, 48, (2, 48)),
    # the stretched torus grid needs a finer coarse level than its vertex count suggests
    ("torus", 2, (1.0, 1.0, 1.0), 138.0, 48, (1, 48)),
])
def test_shifted_coarse_level_rule(kind, nref, axes, sigma, m, want):
    levels = bmg.build_levels(kind, nref, axes=axes)
    area = levels[-1].area
    lc, mm = bmg.shifted_coarse_level(levels, sigma, m, m_given=True)
    assert (lc, mm) == want

    def ok(l):
        return sigma ** 2 * levels[l].hmax ** 2 * area / m <= 60.0 and levels[l].n >= 2 * m
    capped = levels[lc].n <= 12288 and (lc + 1 == len(levels) or levels[lc + 1].n > 12288)
    assert (ok(lc) or capped) and all(not ok(l) for l in range(lc))


def test_longest_edge_halves_per_level():
    # h_max of the sphere hierarchy: the icosahedron edge 4 / sqrt(10 + 2 sqrt(5))
    # on level 0, then about half per refinement (midpoints lifted to the sphere)
    levels = bmg.build_levels("sphere", 4)
    assert abs(levels[0].hmax - 4.0 / math.sqrt(10.0 + 2.0 * math.sqrt(5.0))) < 1e-14
    for a, b in zip(levels[:-1], levels[1:]):
        assert 0.45 < b.hmax / a.hmax < 0.6


def test_shifted_coarse_level_cap_raises_m():
    # torus refined twice (32768 vertices > the 12288 cap) at sigma = 200 with
    # m = 8: the rule wants level 2, the cap gives level 1 (8192 vertices) and
    # a block of 4 ceil(sigma^2 h_max^2 |Gamma| / 60 / 4) vectors there
    levels = bmg.build_levels("torus", 2)
    want = 4 * math.ceil(200.0 ** 2 * levels[1].hmax ** 2 * levels[-1].area / 60.0 / 4)
    lc, m = bmg.shifted_coarse_level(levels, 200.0, 8, m_given=False)
    assert lc == 1 and m == want and 8 < m <= 96
    assert bmg.shifted_coarse_level(levels, 200.0, 8, m_given=True) == (1, 8)
