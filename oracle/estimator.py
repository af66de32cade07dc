"""A posteriori error estimator eta_T of an eigenpair (Sec. 5, eq. est-res).

TEST INFRASTRUCTURE (see the package docstring).

For a P1 eigenpair (u_h, lambda_h) on the flat-triangle surface Gamma_h, per
triangle T:

  eta_T^2 = h_T^2 lambda_h^2 |u_h|^2_{L2(T)}                           (element residual)
          + 1/2 sum_{e in dT} h_e |[grad u_h . mu_e]|^2_{L2(e)}             (conormal jumps)
          + |B_h grad u_h|^2_{L2(T)}                                        (geometry)

and eta(u_h) = (sum_T eta_T^2)^(1/2).  Readings (the paper defers the
notation to its references):

- h_T is the longest edge of T, h_e the length of e.  Inside a flat triangle
  the P1 function is harmonic, so the element residual is lambda_h u_h;
  |u_h|^2_{L2(T)} = |T|/12 (sum u_i^2 + (sum u_i)^2) exactly.
- The jump across an edge e shared by T and T' is the sum of the two outward
  conormal derivatives, grad u_T . mu_{T,e} + grad u_T' . mu_{T',e}, with
  mu_{T,e} the unit vector in the plane of T normal to e pointing away from T
  (on a surface the two conormals are not opposite).  It is constant on e, so
  |.|^2_{L2(e)} = |e| jump^2; the 1/2 shares each edge between its two
  triangles.
- B_h is the geometric error of the Dirichlet form: with A_h the matrix for
  which int_Gamma grad_Gamma u . grad_Gamma v = int_Gamma_h A_h grad u^-l .
  grad v^-l, B_h = A_h - P_h (P_h the projection onto the plane of T).  For
  the unit sphere, whose lift is the radial projection x -> x / |x|, the area
  element is (nu . n_T) / |x|^2 and the lifted gradient is
  |x| (w - ((nu . w) / c) n_T), c = nu . n_T, which gives
    A_h = c P_h + (1 / c) t t^T,   t = P_h nu,   nu = x / |x|,
  so B_h g = (c - 1) g + ((t . g) / c) t for g in the plane of T.  The L2(T)
  norm uses the edge-midpoint rule (exact for quadratics).  B_h is computed
  for the sphere only; other surfaces get no geometric term (parity of that
  term unpinned beyond the sphere).
"""
import numpy as np


def _edges_of(tri):
    """For edge i of triangle t (opposite its vertex i) the neighbour triangle
    sharing it and that edge's index there."""
    F = len(tri)
    owner = {}
    nbr = np.full((F, 3), -1, dtype=np.int64)
    nbr_edge = np.full((F, 3), -1, dtype=np.int64)
    for t in range(F):
        for i in range(3):
            a, b = int(tri[t, (i + 1) % 3]), int(tri[t, (i + 2) % 3])
            key = (min(a, b), max(a, b))
            if key in owner:
                s, j = owner[key]
                nbr[t, i], nbr_edge[t, i] = s, j
                nbr[s, j], nbr_edge[s, j] = t, i
            else:
                owner[key] = (t, i)
    return nbr, nbr_edge


def _geometry(xyz, tri):
    x0, x1, x2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(x1 - x0, x2 - x0)
    area2 = np.linalg.norm(cr, axis=1)  # 2 |T|
    n = cr / area2[:, None]
    cen = (x0 + x1 + x2) / 3.0
    n = n * np.sign(np.einsum("ij,ij->i", n, cen))[:, None]  # outward for the closed surfaces here
    X = np.stack([x0, x1, x2], axis=1)  # [F][3 vertices][3]
    # gradient of the barycentric function of vertex i: the edge opposite i,
    # rotated in the plane, over 2 |T|
    grads = np.empty_like(X)
    for i in range(3):
        e = X[:, (i + 2) % 3] - X[:, (i + 1) % 3]
        g = np.cross(n, e) / area2[:, None]
        # orient towards vertex i (grad lambda_i points from the edge to i)
        s = np.sign(np.einsum("ij,ij->i", g, X[:, i] - X[:, (i + 1) % 3]))
        grads[:, i] = g * s[:, None]
    return X, n, area2 / 2.0, grads


def sphere_lift_matrix(x, n):
    """A_h at points x [q][3] of triangles with unit normals n [q][3] for the
    radial lift onto the unit sphere: c P_h + t t^T / c ([q][3][3])."""
    nu = x / np.linalg.norm(x, axis=1)[:, None]
    c = np.einsum("ij,ij->i", nu, n)
    t = nu - c[:, None] * n
    Ph = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
    return c[:, None, None] * Ph + t[:, :, None] * t[:, None, :] / c[:, None, None]


def estimate(xyz, tri, U, lam, sphere=False):
    """Per-triangle terms of eta_T^2 for the eigenpairs (lam[j], U[:, j]).

    Returns parts [3][F][k] (residual, jump, geometry) and eta [k]."""
    U = np.asarray(U, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    F, k = len(tri), U.shape[1]
    X, n, area, grads = _geometry(xyz, tri)
    nbr, nbr_edge = _edges_of(tri)
    uv = U[tri]  # [F][3][k]
    g = np.einsum("fid,fik->fkd", grads, uv)  # [F][k][3] gradient per triangle and pair
    edge_len = np.stack([np.linalg.norm(X[:, (i + 2) % 3] - X[:, (i + 1) % 3], axis=1) for i in range(3)], axis=1)
    hT = edge_len.max(axis=1)
    # element residual
    l2 = area[:, None] / 12.0 * (np.sum(uv * uv, axis=1) + np.sum(uv, axis=1) ** 2)
    res = hT[:, None] ** 2 * lam[None, :] ** 2 * l2
    # outward conormal of each edge: in the plane of T, normal to the edge,
    # away from the opposite vertex
    mu = np.empty((F, 3, 3))
    for i in range(3):
        a, b, c = X[:, (i + 1) % 3], X[:, (i + 2) % 3], X[:, i]
        tau = (b - a) / edge_len[:, i:i + 1]
        v = 0.5 * (a + b) - c
        v = v - np.einsum("ij,ij->i", v, tau)[:, None] * tau
        mu[:, i] = v / np.linalg.norm(v, axis=1)[:, None]
    jump = np.zeros((F, k))
    for i in range(3):
        s, j = nbr[:, i], nbr_edge[:, i]
        own = np.einsum("fkd,fd->fk", g, mu[:, i])
        other = np.einsum("fkd,fd->fk", g[s], mu[s, j])
        jump += 0.5 * edge_len[:, i:i + 1] * edge_len[:, i:i + 1] * (own + other) ** 2
    geo = np.zeros((F, k))
    if sphere:
        Ph = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
        for i in range(3):  # edge-midpoint rule, weight |T| / 3 each
            xq = 0.5 * (X[:, (i + 1) % 3] + X[:, (i + 2) % 3])
            B = sphere_lift_matrix(xq, n) - Ph
            Bg = np.einsum("fde,fke->fkd", B, g)
            geo += area[:, None] / 3.0 * np.sum(Bg * Bg, axis=2)
    parts = np.stack([res, jump, geo])
    eta = np.sqrt(parts.sum(axis=(0, 1)))
    return parts, eta

