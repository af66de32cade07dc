"""Geometric prolongation and restriction between consecutive levels.

Sec. 3, eq. (proj-1): the prolongated function keeps the coarse nodal values at
the old vertices and takes the mean of the two parent values at each new
(projected midpoint) vertex.  Its matrix P_h (N_h x N_H) therefore has a unit
row e_i for i < N_H and the row (e_a + e_b)/2 for the vertex created on edge
(a, b).  The restriction is its transpose, P_H = P_h^T (end of Sec. 3).
"""
import numpy as np
import scipy.sparse as sp


def prolongation(n_coarse, parents):
    """P (N_fine x N_coarse) as CSR from the parent table of the new vertices."""
    n_new = len(parents)
    n_fine = n_coarse + n_new
    rows = np.concatenate([np.arange(n_coarse), n_coarse + np.arange(n_new), n_coarse + np.arange(n_new)])
    cols = np.concatenate([np.arange(n_coarse), parents[:, 0], parents[:, 1]])
    vals = np.concatenate([np.ones(n_coarse), np.full(n_new, 0.5), np.full(n_new, 0.5)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_fine, n_coarse))
