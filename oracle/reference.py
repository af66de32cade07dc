"""The plain definition of the result, computed by library eigensolvers.

The result of the method is the set of discrete eigenpairs of eq. (pb-eig-fea)
in matrix form, A_L u = lambda M_L u (Sec. 2.2), nearest the shift sigma, with
b_h-orthonormal eigenvectors (Sec. 2.1).  Small problems use a dense
generalized symmetric eigensolve (LAPACK through scipy.linalg.eigh); larger ones
use ARPACK shift-invert (scipy.sparse.linalg.eigsh) around sigma, or around -1
when sigma = 0 because A_L is singular.

Also here: the eigenpair comparison used by the parity tests (relative
eigenvalue error with denominator max(|lambda|, 1); largest principal angle per
cluster in the M inner product).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def discrete_eigs(A, M, k, sigma=0.0, dense_max=3000, extra=8):
    """k eigenpairs of (A, M) nearest sigma, ascending; M-orthonormal vectors."""
    n = A.shape[0]
    if n <= dense_max:
        w, V = sla.eigh(A.toarray(), M.toarray())
    else:
        shift = -1.0 if sigma == 0 else sigma
        w, V = spla.eigsh(A.tocsc(), k=min(k + extra, n - 2), M=M.tocsc(), sigma=shift,
                          which="LM", tol=1e-14)
        # re-M-normalise (ARPACK returns M-orthonormal vectors up to its tolerance)
        V = V / np.sqrt(np.einsum("ij,ij->j", V, M @ V))[None, :]
    idx = np.lexsort((np.arange(len(w)), w, np.abs(w - sigma)))[:k]
    idx = idx[np.argsort(w[idx], kind="stable")]
    return w[idx], V[:, idx]


def cluster_groups(evals, rel=1e-2):
    """Groups of indices of ascending eigenvalues whose relative gap is < rel."""
    groups = [[0]]
    for j in range(1, len(evals)):
        scale = max(abs(evals[j]), abs(evals[j - 1]), 1.0)
        if evals[j] - evals[j - 1] < rel * scale:
            groups[-1].append(j)
        else:
            groups.append([j])
    return groups


def subspace_sine(Q_ref, U, M):
    """sin of the largest angle between span(U) and span(Q_ref), M inner product.

    Both blocks are M-orthonormal.  When U has fewer columns than Q_ref this is
    the one-sided containment measure ||(I - Q Q^T M) U||_M.
    """
    X = U - Q_ref @ (Q_ref.T @ (M @ U))
    G = X.T @ (M @ X)
    return float(np.sqrt(max(np.linalg.eigvalsh(0.5 * (G + G.T)).max(), 0.0)))


def compare(evals, U, ref_evals, ref_U, M, ref_group_evals=None, ref_group_U=None):
    """Return (max relative eigenvalue error, max per-cluster subspace sine).

    Clusters are formed on the reference eigenvalues.  When a reference with
    more pairs is given (ref_group_*), clusters cut by the k boundary are
    tested for containment in the reference's full cluster.
    """
    rel = np.abs(np.asarray(evals) - np.asarray(ref_evals)) / np.maximum(np.abs(ref_evals), 1.0)
    worst = 0.0
    for g in cluster_groups(np.asarray(ref_evals)):
        Qg = ref_U[:, g]
        if ref_group_evals is not None:
            lo, hi = ref_evals[g[0]], ref_evals[g[-1]]
            span = 1e-2 * max(abs(hi), 1.0)
            full = [j for j in range(len(ref_group_evals))
                    if lo - span <= ref_group_evals[j] <= hi + span]
            Qg = ref_group_U[:, full]
        worst = max(worst, subspace_sine(Qg, U[:, g], M))
    return float(rel.max()), worst
