"""Pins of the oracle's P1 assembly and transfers (paper Sec. 2.1-2.2, Sec. 3)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.special import ellipeinc, ellipkinc

from oracle import fem, mesh, transfer


def test_equilateral_triangle_closed_form():
    s = 1.7
    xyz = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]])
    A, M = fem.assemble(xyz, np.array([[0, 1, 2]]))
    area = math.sqrt(3) / 4 * s * s
    # cotangent formula: A_ij = -cot(60 deg)/2, A_ii = cot(60 deg)
    cot = 1 / math.sqrt(3)
    Aex = np.full((3, 3), -cot / 2) + np.eye(3) * (1.5 * cot)
    Mex = area / 12 * (np.ones((3, 3)) + np.eye(3))
    assert np.allclose(A.toarray(), Aex, atol=1e-15)
    assert np.allclose(M.toarray(), Mex, atol=1e-15)


def test_right_triangle_closed_form():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0]], dtype=float)
    A, _ = fem.assemble(xyz, np.array([[0, 2, 1]]))  # either orientation
    # angle at vertex 0 is 90 deg -> A_12 = 0; angle at 1: tan = 2 -> cot = 1/2
    # A_02 = -cot(angle at 1)/2 = -1/4; angle at 2: cot = 2 -> A_01 = -1
    Ad = A.toarray()
    assert abs(Ad[1, 2]) < 1e-15
    assert abs(Ad[0, 2] + 0.25) < 1e-15 and abs(Ad[0, 1] + 1.0) < 1e-15


@pytest.mark.parametrize("kind", ["sphere", "ellipsoid", "torus"])
def test_assembly_invariants(kind):
    # dense eigenvalue checks below: the torus's unrefined 64 x 32 grid (2048
    # vertices) is already larger than the refined icosphere (642)
    lv = mesh.hierarchy(kind, 0 if kind == "torus" else 3, axes=(1.0, 1.5, 2.0))[-1]
    A, M = fem.assemble(lv.xyz, lv.tri)
    assert abs(A - A.T).max() < 1e-14 and abs(M - M.T).max() < 1e-16
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-13
    area = fem.triangle_areas(lv.xyz, lv.tri).sum()
    assert abs(M.sum() - area) < 1e-12 * area
    w = np.linalg.eigvalsh(M.toarray())
    assert w.min() > 0
    # A positive semidefinite with a one-dimensional kernel (closed connected surface)
    wa = np.linalg.eigvalsh(A.toarray())
    assert wa[0] > -1e-12 and wa[1] > 1e-6
    # lumped-mass bound 1/4 D <= M <= D (elementwise P1 identity used by the certificates)
    D = fem.lumped_mass(M)
    s = 1 / np.sqrt(D)
    ws = np.linalg.eigvalsh((M.toarray() * s[:, None]) * s[None, :])
    assert ws.min() >= 0.25 - 1e-12 and ws.max() <= 1 + 1e-12


def test_icosahedron_area_closed_form_and_h2_convergence():
    s2 = 16 / (10 + 2 * math.sqrt(5))
    levels = mesh.hierarchy("sphere", 5)
    areas = [fem.triangle_areas(l.xyz, l.tri).sum() for l in levels]
    assert abs(areas[0] - 20 * math.sqrt(3) / 4 * s2) < 1e-13
    err = [4 * math.pi - a for a in areas]
    ratios = [err[i] / err[i + 1] for i in range(len(err) - 1)]
    assert all(e > 0 for e in err)
    assert all(3.5 < r < 4.5 for r in ratios[1:])  # O(h^2)


def test_ellipsoid_area_legendre():
    a, b, c = 2.0, 1.5, 1.0
    phi = math.acos(c / a)
    k2 = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    S = 2 * math.pi * c * c + 2 * math.pi * a * b / math.sin(phi) * (
        ellipeinc(phi, k2) * math.sin(phi) ** 2 + ellipkinc(phi, k2) * math.cos(phi) ** 2)
    levels = mesh.hierarchy("ellipsoid", 5, axes=(1.0, 1.5, 2.0))
    err = [S - fem.triangle_areas(l.xyz, l.tri).sum() for l in levels]
    assert abs(err[-1]) < 2e-3 * S
    assert 3.5 < err[-2] / err[-1] < 4.5


def test_torus_area():
    S = 4 * math.pi ** 2 * 1.0 * 0.4
    levels = mesh.hierarchy("torus", 2)
    err = [S - fem.triangle_areas(l.xyz, l.tri).sum() for l in levels]
    assert abs(err[-1]) < 1e-3 * S and 3.5 < err[0] / err[1] < 4.5


@pytest.mark.parametrize("kind", ["sphere", "torus"])
def test_nested_flat_galerkin_identity(kind):
    # without projection the meshes are nested and P is the exact inclusion
    levels = mesh.hierarchy(kind, 2 if kind == "sphere" else 1, flat=True)
    for lc, lf in zip(levels[:-1], levels[1:]):
        Ac, Mc = fem.assemble(lc.xyz, lc.tri)
        Af, Mf = fem.assemble(lf.xyz, lf.tri)
        P = transfer.prolongation(len(lc.xyz), lf.parents)
        assert abs(P.T @ Af @ P - Ac).max() < 1e-13
        assert abs(P.T @ Mf @ P - Mc).max() < 1e-15


def test_prolongation_rows():
    levels = mesh.hierarchy("sphere", 2)
    P = transfer.prolongation(len(levels[1].xyz), levels[2].parents)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0)
    nc = P.shape[1]
    assert abs(P[:nc] - sp.eye(nc)).max() == 0
    assert np.all(np.diff(P.indptr)[nc:] == 2)
