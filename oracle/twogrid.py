"""Two-grid eigensolver with a spectral shift (Alg. 1), applied in a cascade.

TEST INFRASTRUCTURE (see the package docstring).

Alg. 1: solve the coarse eigenproblem (A_H - mu M_H) u_H = lambda_H M_H u_H
directly, then on the refined, projected mesh approximate the source problem
of eq. (pb-f-s),
    (A_h - (mu + lambda_H) M_h) u^h = M_h P_h u_H,
whose solution is one step of inverse iteration about the coarse eigenvalue;
its Rayleigh quotient is the two-grid eigenvalue.  Remark 3.1 repeats the step
between neighbouring levels, each level's pair acting as the coarse pair of the
next.  The fixed shift mu cancels: the fine problem uses mu + lambda_H, the
unshifted coarse eigenvalue, and the coarse eigenvectors do not depend on it.

The source problem is approximated either by a sparse direct solve (method 1
of the Sec. 5.3 comparison) or, as the remark after Alg. 1 allows and method 2
does, by nu Kaczmarz sweeps (Sec. 5.3; multicolour, alternating directions,
starting forward) from the prolongated approximation of the previous level.
Each level's vectors are M-normalised before they are passed on.

With a coarse mesh too coarse for the wavelength of an eigenfunction, the
coarse eigenvalue lies nearer another fine eigenvalue and the inverse
iteration converges there: the loss of spectra of Sec. 5.1.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .bmg import Smoother


def two_grid(levels, level_H, idx, top=None, source="direct", nu=5):
    """Cascade of Alg. 1 from level_H up to top (default: the finest level)
    for the coarse pairs idx (indices into the ascending spectrum of
    (A_H, M_H)).  Returns (rows, U): rows[l] holds the eigenvalue
    approximations on level l (level_H: the coarse eigenvalues), U the
    M-orthonormal-per-column vectors on level top."""
    top = len(levels) - 1 if top is None else top
    LH = levels[level_H]
    lam, phi = sla.eigh(LH.A.toarray(), LH.M.toarray())
    idx = np.asarray(idx)
    U = phi[:, idx]
    theta = lam[idx].copy()
    rows = {level_H: theta.copy()}
    for k in range(level_H + 1, top + 1):
        L = levels[k]
        Up = L.P @ U
        F = L.M @ Up
        X = np.empty_like(Up)
        for c in range(U.shape[1]):
            if source == "direct":
                X[:, c] = spla.spsolve((L.A - theta[c] * L.M).tocsc(), F[:, c])
            else:
                sm = Smoother(L, theta[c], "kaczmarz", 1.0)
                x = Up[:, c:c + 1].copy()
                for s in range(nu):
                    x = sm.sweep(x, F[:, c:c + 1], forward=(s % 2 == 0))
                X[:, c] = x[:, 0]
        qa = np.einsum("ij,ij->j", X, L.A @ X)
        qm = np.einsum("ij,ij->j", X, L.M @ X)
        theta = qa / qm
        U = X / np.sqrt(qm)[None, :]
        rows[k] = theta.copy()
    return rows, U
