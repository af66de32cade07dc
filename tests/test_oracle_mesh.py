"""Pins of the oracle's meshes and refinement (paper Sec. 3, Fig. 2; Sec. 5)."""
import os

import numpy as np
import pytest

from oracle import mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _edge_use(tri):
    d = {}
    for a, b, c in tri:
        for u, v in ((a, b), (b, c), (c, a)):
            d[(int(u), int(v))] = d.get((int(u), int(v)), 0) + 1
    return d


@pytest.mark.parametrize("l", range(5))
def test_icosphere_counts(l):
    lv = mesh.hierarchy("sphere", l)[-1]
    n, f = len(lv.xyz), len(lv.tri)
    e = len(mesh.edges(lv.tri))
    assert n == 10 * 4 ** l + 2 and f == 20 * 4 ** l and e == 30 * 4 ** l
    assert n - e + f == 2  # Euler characteristic of the sphere


def test_genus0_refinement_rule_matches_paper_dofs():
    # V' = 4V - 6 holds for our refinement, and reproduces the paper's 54 -> 3330
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_dof_counts.txt")) if l[0] != "#"]
    (r0, d0), (r1, d1) = [(int(a), int(b)) for a, b in rows]
    v = d0
    for _ in range(r1 - r0):
        v = 4 * v - 6
    assert v == d1
    lv = mesh.hierarchy("sphere", 4)
    for a, b in zip(lv[:-1], lv[1:]):
        assert len(b.xyz) == 4 * len(a.xyz) - 6


@pytest.mark.parametrize("kind", ["sphere", "ellipsoid", "torus"])
def test_closed_oriented_manifold(kind):
    levels = mesh.hierarchy(kind, 2, axes=(1.0, 1.5, 2.0))
    for lv in levels:
        use = _edge_use(lv.tri)
        # each directed edge once and its reverse once: closed and consistently oriented
        assert all(c == 1 for c in use.values())
        assert all((v, u) in use for (u, v) in use)
        n, f, e = len(lv.xyz), len(lv.tri), len(mesh.edges(lv.tri))
        assert n - e + f == (0 if kind == "torus" else 2)


def test_vertices_on_surface_and_midpoint_parents():
    a = np.array([1.0, 1.5, 2.0])
    for lv in mesh.hierarchy("ellipsoid", 3, axes=tuple(a)):
        q = np.sum((lv.xyz / a) ** 2, axis=1)
        assert np.allclose(q, 1.0, atol=1e-14)
    levels = mesh.hierarchy("sphere", 3)
    for lc, lf in zip(levels[:-1], levels[1:]):
        nc = len(lc.xyz)
        mid = lc.xyz[lf.parents[:, 0]] + lc.xyz[lf.parents[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        assert np.allclose(lf.xyz[nc:], mid, atol=1e-15)
        assert np.array_equal(lf.xyz[:nc], lc.xyz)
        assert np.all(lf.parents[:, 0] < lf.parents[:, 1])


def test_torus_counts_and_surface():
    R, r = 1.0, 0.4
    levels = mesh.hierarchy("torus", 2)
    for t, lv in enumerate(levels):
        assert len(lv.xyz) == 2048 * 4 ** t
        rho = np.hypot(lv.xyz[:, 0], lv.xyz[:, 1])
        assert np.allclose((rho - R) ** 2 + lv.xyz[:, 2] ** 2, r * r, atol=1e-14)


def test_outward_orientation_sphere():
    lv = mesh.hierarchy("sphere", 2)[-1]
    x = lv.xyz[lv.tri]
    n = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    assert np.all(np.einsum("tk,tk->t", n, x.sum(axis=1)) > 0)


def test_icosahedron_order():
    xyz, tri = mesh.icosahedron()
    assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0)
    assert np.all(tri[:, 0] == tri.min(axis=1))
    assert np.array_equal(tri, tri[np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0]))])
