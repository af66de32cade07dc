"""Pins of the oracle's a posteriori estimator (Sec. 5, eq. est-res; oracle/estimator.py).

- Element residual: its sum over triangles, divided by h_T^2 lambda^2, is the
  mass-matrix norm u^T M u of the P1 function (assembly of oracle/fem.py).
- Gradients: for u = a . x at the vertices, the per-triangle gradient is the
  projection of a onto the triangle's plane.
- Jumps: on the icosahedron refined without projecting the midpoints (flat
  faces), a linear function jumps only across the 30 original edges; the
  total is the closed form sum_E (a . (mu_1 + mu_2))^2 L_E^2 / 2^l from the
  icosahedron's own face geometry.
- Lift matrix A_h of the sphere: int over T of A_h g . g equals the Dirichlet
  energy of the radially lifted P1 function on the spherical triangle,
  computed by brute force (a fine subdivision mapped onto the sphere).
- Rates on the sphere's discrete eigenfunctions: eta = O(h) (halves per
  level), the geometric term O(h^4) of |grad u|^2, and the effectivity
  eta / |u - u_h|_{H1} against the exact eigenfunction a . x / |x| constant
  across levels.
"""
import numpy as np
import pytest

from oracle import bmg, estimator, fem, mesh, reference


@pytest.fixture(scope="module")
def sphere5():
    return bmg.build_levels("sphere", 5)


def test_residual_term_is_the_mass_norm(sphere5):
    L = sphere5[3]
    u = np.random.default_rng(0).standard_normal(L.n)
    parts, eta = estimator.estimate(L.xyz, L.tri, u, 3.0)
    X = L.xyz[L.tri]
    hT = np.max([np.linalg.norm(X[:, (i + 2) % 3] - X[:, (i + 1) % 3], axis=1) for i in range(3)], axis=0)
    A, M = fem.assemble(L.xyz, L.tri)
    assert abs(np.sum(parts[0][:, 0] / (hT ** 2 * 9.0)) - u @ (M @ u)) < 1e-12 * (u @ (M @ u))
    assert np.all(parts[2] == 0.0)  # no geometric term unless asked for the sphere


def test_gradients_of_linear_functions(sphere5):
    L = sphere5[2]
    a = np.array([0.3, -1.2, 0.7])
    X, n, area, grads = estimator._geometry(L.xyz, L.tri)
    g = np.einsum("fid,fi->fd", grads, (L.xyz @ a)[L.tri])
    Pa = a[None, :] - (n @ a)[:, None] * n
    assert np.max(np.abs(g - Pa)) < 1e-12
    assert np.allclose(area, fem.triangle_areas(L.xyz, L.tri))


@pytest.mark.parametrize("nref", [1, 2])
def test_jumps_of_a_linear_function_on_flat_faces(nref):
    levels = mesh.hierarchy("sphere", nref, flat=True)
    xyz, tri = levels[-1].xyz, levels[-1].tri
    a = np.array([0.4, 0.9, -0.5])
    parts, _ = estimator.estimate(xyz, tri, xyz @ a, 0.0)
    # closed form from the icosahedron's faces: every original edge E of
    # length L_E between faces F1, F2 contributes (a . (mu_1 + mu_2))^2 L_E^2 / 2^l
    x0, t0 = levels[0].xyz, levels[0].tri
    faces = {}
    for f, t in enumerate(t0):
        for i in range(3):
            e = tuple(sorted((int(t[(i + 1) % 3]), int(t[(i + 2) % 3]))))
            faces.setdefault(e, []).append((f, int(t[i])))
    want = 0.0
    for (p, q), fl in faces.items():
        assert len(fl) == 2
        tau = (x0[q] - x0[p]) / np.linalg.norm(x0[q] - x0[p])
        s = 0.0
        for f, opp in fl:
            v = 0.5 * (x0[p] + x0[q]) - x0[opp]
            v -= (v @ tau) * tau
            s += a @ (v / np.linalg.norm(v))
        want += s * s * np.sum((x0[q] - x0[p]) ** 2) / 2 ** nref
    assert abs(parts[1].sum() - want) < 1e-12 * want
    assert parts[0].sum() == 0.0


def test_sphere_lift_matrix_against_the_lifted_energy():
    # a triangle of the 42-vertex level (chordal, inside the sphere) and three
    # P1 functions on it: int_T A_h g . g (fine quadrature of the oracle's A_h)
    # against the energy of the lifted function on the spherical triangle
    lv = bmg.build_levels("sphere", 1)[-1]
    T = lv.xyz[lv.tri[7]]
    n = np.cross(T[1] - T[0], T[2] - T[0])
    area = 0.5 * np.linalg.norm(n)
    n /= np.linalg.norm(n)
    N = 96
    # barycentric grid of the triangle: points and sub-triangles
    pts, idx = [], {}
    for i in range(N + 1):
        for j in range(N + 1 - i):
            idx[(i, j)] = len(pts)
            pts.append(T[0] + (T[1] - T[0]) * i / N + (T[2] - T[0]) * j / N)
    pts = np.array(pts)
    subs = []
    for i in range(N):
        for j in range(N - i):
            subs.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
            if i + j < N - 1:
                subs.append((idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
    subs = np.array(subs)
    lifted = pts / np.linalg.norm(pts, axis=1)[:, None]
    cen = pts[subs].mean(axis=1)
    Ah = estimator.sphere_lift_matrix(cen, np.repeat(n[None], len(subs), axis=0))
    for vals in ([1.0, 0.0, 0.0], [0.0, 1.0, -2.0], [0.3, 0.5, 0.9]):
        # the P1 function on T: its gradient g and values at the grid points
        M3 = np.c_[T, np.ones(3)]  # rows (x, y, z, 1) of the vertices
        coef = np.linalg.lstsq(M3, np.asarray(vals), rcond=None)[0]
        g = coef[:3] - (coef[:3] @ n) * n
        u = pts @ coef[:3] + coef[3]
        # energy on the sphere: P1 on each lifted sub-triangle
        P = lifted[subs]
        e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
        cr = np.cross(e1, e2)
        a2 = np.linalg.norm(cr, axis=1)
        nn = cr / a2[:, None]
        du1, du2 = u[subs[:, 1]] - u[subs[:, 0]], u[subs[:, 2]] - u[subs[:, 0]]
        grad = (du1[:, None] * np.cross(e2, nn) - du2[:, None] * np.cross(e1, nn)) / a2[:, None]
        brute = np.sum(0.5 * a2 * np.einsum("fd,fd->f", grad, grad))
        quad = area / len(subs) * np.einsum("d,fde,e->", g, Ah, g)
        assert abs(brute - quad) < 2e-4 * brute, (vals, brute, quad)


def test_rates_and_effectivity_on_the_sphere():
    lv = bmg.build_levels("sphere", 6)
    prev, eff = None, []
    for l in range(3, 7):
        L = lv[l]
        ev, U = reference.discrete_eigs(L.A, L.M, 4, 0.0)
        u = U[:, 1]
        parts, eta = estimator.estimate(L.xyz, L.tri, u, ev[1], sphere=True)
        g2 = u @ (L.A @ u)
        assert parts[2].sum() / g2 < 3e-5 * 16.0 ** (2 - l)  # O(h^4)
        if prev is not None:
            assert 1.95 < prev / eta[0] < 2.05
        prev = eta[0]
        # H1 error on Gamma_h of the exact eigenfunction a . x / |x| nearest u
        B = L.xyz
        a = np.linalg.solve(B.T @ (L.M @ B), B.T @ (L.M @ u))
        X, n, area, grads = estimator._geometry(L.xyz, L.tri)
        gh = np.einsum("fid,fi->fd", grads, u[L.tri])
        err2 = 0.0
        for i in range(3):
            xq = 0.5 * (X[:, (i + 1) % 3] + X[:, (i + 2) % 3])
            r = np.linalg.norm(xq, axis=1)
            ge = a[None, :] / r[:, None] - (xq @ a)[:, None] * xq / r[:, None] ** 3
            ge -= np.einsum("fd,fd->f", ge, n)[:, None] * n
            err2 += np.sum(area / 3 * np.einsum("fd,fd->f", ge - gh, ge - gh))
        eff.append(eta[0] / np.sqrt(err2))
    assert max(eff) / min(eff) < 1.01 and 1.0 < min(eff) < 20.0, eff
