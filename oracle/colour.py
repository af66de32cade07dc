"""Greedy vertex colouring for the multicolour Gauss-Seidel smoother.

The paper smooths with (symmetric) Gauss-Seidel (Sec. 5.3, method 4; Remark 4.2)
and does not say how the sweep is ordered.  The reading used here: vertices are
visited in increasing index and each takes the smallest colour not used by a
lower-index neighbour in the matrix graph.  A Gauss-Seidel sweep then updates
the colours one after another; rows of one colour are not coupled, so their
order inside a colour does not change the result.
"""
import numpy as np


def greedy_colouring(A):
    """Colour array (int64) for the graph of the sparse matrix A."""
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
