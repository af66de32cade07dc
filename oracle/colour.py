"""Greedy vertex colourings for the multicolour Gauss-Seidel and Kaczmarz smoothers.

The paper smooths with (symmetric) Gauss-Seidel (Sec. 5.3, method 4; Remark 4.2)
and does not say how the sweep is ordered.  The reading used here: vertices are
visited in increasing index and each takes the smallest colour not used by a
lower-index neighbour in the matrix graph.  A Gauss-Seidel sweep then updates
the colours one after another; rows of one colour are not coupled, so their
order inside a colour does not change the result.
"""
import numpy as np


def greedy_colouring(A):
    """Colour array (int64) for the graph of the sparse matrix A (the smoothers
    pass the mass matrix, whose pattern is the mesh graph)."""
    A = A.tocsr()
    n = A.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
        used = {int(col[j]) for j in nb if j < i}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def distance2_colouring(A):
    """Colour array (int64) in which no two vertices within two edges of the
    graph of A share a colour: vertices in increasing index, each taking the
    smallest colour not used by a lower-index vertex at distance 1 or 2.

    The Kaczmarz relaxation of Sec. 5.3 projects the iterate onto one row's
    hyperplane at a time, which changes every entry in that row's pattern.
    Two rows can be projected at once when their patterns are disjoint, i.e.
    when the vertices are more than two edges apart; a colour of this
    colouring is such a set (the same reading of the unstated sweep order as
    for Gauss-Seidel above).
    """
    P = A.tocsr().copy()
    P.data[:] = 1.0
    P2 = (P @ P).tocsr()  # pattern of vertices within two edges
    n = A.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nb = P2.indices[P2.indptr[i]:P2.indptr[i + 1]]
        used = {int(col[j]) for j in nb if j < i}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col
