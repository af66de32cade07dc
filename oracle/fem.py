"""P1 surface finite elements on a flat-triangle surface Gamma_h.

Sec. 2.1 (eq. bl-dis) defines a_h(u,v) = int grad u . grad v and
b_h(u,v) = int u v on the piecewise planar surface; Sec. 2.2 (eq. sp-fe,
eq. pb-eig-fea) restricts them to continuous piecewise-linear functions.  On a
flat triangle T with vertices x0, x1, x2 and e_i the edge vector opposite
vertex i (e_0 = x2 - x1, e_1 = x0 - x2, e_2 = x1 - x0), the P1 gradients are
rotated edges divided by 2|T|, hence

    A_ij += (e_i . e_j) / (4 |T|)          (i != j)
    M_ij += |T| / 12  (i != j),   M_ii += |T| / 6.

The diagonal of A is set to minus the sum of the off-diagonals of its row, which
equals (e_i . e_i)/(4|T|) summed over triangles because e_0 + e_1 + e_2 = 0.
"""
import numpy as np
import scipy.sparse as sp


def triangle_areas(xyz, tri):
    x0, x1, x2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(x1 - x0, x2 - x0), axis=1)


def assemble(xyz, tri):
    """Return (A, M) as scipy CSR matrices in FP64."""
    n = len(xyz)
    x = [xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]]
    e = [x[2] - x[1], x[0] - x[2], x[1] - x[0]]
    area = triangle_areas(xyz, tri)
    rows, cols, av, mv = [], [], [], []
    for i in range(3):
        for j in range(3):
            rows.append(tri[:, i])
            cols.append(tri[:, j])
            if i == j:
                av.append(np.zeros_like(area))
                mv.append(area / 6.0)
            else:
                av.append(np.einsum("tk,tk->t", e[i], e[j]) / (4.0 * area))
                mv.append(area / 12.0)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    A = sp.coo_matrix((np.concatenate(av), (rows, cols)), shape=(n, n)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    M.sum_duplicates()
    # diagonal = - sum of off-diagonal entries of the row (zero row sums)
    A = A.tolil()
    A.setdiag(0.0)
    A = A.tocsr()
    off = np.asarray(A.sum(axis=1)).ravel()
    A = A + sp.diags(-off)
    A = A.tocsr()
    A.sort_indices()
    M.sort_indices()
    return A, M


def lumped_mass(M):
    """Row sums of the consistent mass matrix (the lumped diagonal D)."""
    return np.asarray(M.sum(axis=1)).ravel()
