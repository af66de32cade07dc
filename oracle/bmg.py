"""Plain FP64 bootstrap multigrid (BMG) eigensolver for A u = lambda M u.

TEST INFRASTRUCTURE: the reference the HIP path is compared with.  Slow on
purpose: SciPy sparse products and dense LAPACK calls, no blocking or fusion.

What is computed (paper Sec. 4, Alg. 2 and Alg. 3, with Remark 3.2):

 1. Coarse eigensolve on level 0 (Alg. 2 step 1): all eigenpairs of
    (A_0, M_0).  The n_c coarse eigenvectors nearest the shift sigma are
    prolongated to the finest level L: W_c = P_{0->L} Phi_c.  Together with
    the block of test vectors they span the enriched space V_H + X_h
    (Alg. 2 step 4), evaluated exactly on the finest level (Galerkin reading
    of the enriched pencil, which makes the Ritz step an exact Rayleigh-Ritz
    on span[W_c, U]).
 2. Test vectors: an N_L x m Gaussian block (see rng.py), followed by a first
    Rayleigh-Ritz step.
 3. Each cycle relaxes the fine source problem of eq. (pb-f-aux-mat) starting
    from the current approximation (Remark 3.2: a smoother started from the
    previous approximation replaces the solve).  In defect form this is the
    correction U' = U - B_sigma (A U - M U Theta), where B_sigma is one
    V(nu1, nu2) cycle for the rediscretised operators A_l - sigma M_l on
    levels L down to l_c, with P^T as restriction and P as prolongation
    (Sec. 3), smoothing by multicolour symmetric Gauss-Seidel (Sec. 5.3,
    method 4; Remark 4.2), weighted Jacobi (weight 0.85 unless given) or
    multicolour symmetric Kaczmarz (Sec. 5.3, methods 2 and 6; see Smoother).
    All colourings are of the mesh graph (the pattern of M, which S shares).
 4. M-orthonormalisation of Z = [W_c, U'] (Alg. 2 step 3: orthogonalisation
    in the b_h inner product) by SVQB, then the Ritz eigenproblem of the enriched
    pencil (eq. pb-c-aux-mat) shifted by sigma; the m Ritz pairs nearest sigma
    are kept (Alg. 2 step 2 choice of the index set Lambda, Remark 4.1).
 5. Stop when every returned pair carries a residual certificate: with
    rho_i = 2 ||r_i||_{D^-1} (D the lumped mass, 1/4 D <= M <= D elementwise
    for P1 so rho_i >= ||r_i||_{M^-1}) and delta_i the distance from theta_i
    to the nearest Ritz value outside its cluster, require
    rho_i^2 / delta_i <= 0.1 tol max(|theta_i|, 1)   (Kato-Temple)  and
    rho_i / delta_i <= angle_tol                      (Davis-Kahan).

Readings where the paper is silent (the library states the same readings in
its own words): n_c = min(N_0, 32); l_c is the coarsest level with
N_l >= 8 n_W(sigma), n_W(sigma) = |Gamma_h| sigma / (4 pi) (Weyl count); at
l_c = 0 the coarse operator is inverted on its spectrum with the modes within
1e-2 max(1, |sigma|) of sigma dropped, otherwise 8 smoothing sweeps are used;
Ritz values whose relative gap is below 1e-2 form one cluster; the
weighted-Jacobi weight is 0.85 (local Fourier analysis of the P1 stiffness
stencil on a regular triangle lattice: D^-1 A maps the frequencies that the
coarse grid cannot represent into [2/3, 3/2], whose best damping weight is
2 / (2/3 + 3/2) = 12/13; 0.85 keeps a margin for irregular meshes).

Interior shifts (sigma > 0; scheme "shifted").  The fixed-shift cycle above
stalls when sigma lies inside the spectrum: coarse levels misplace the
eigenvalues near sigma by O(sigma^2 h_l^2) (the a priori estimate of Sec. 2.2, Lemma 2.2),
so the coarse correction acts like shift-and-invert about a wrong shift, and
prolongated coarse eigenvectors kept in the Ritz space add Ritz values with
large residuals right next to sigma.  The shifted scheme follows the paper's
own route to interior eigenvalues instead (Sec. 5.2; Remark 4.1; Alg. 3
step 4; Alg. 4 step 1):

 1. Coarse eigensolve (Alg. 2 step 1, Alg. 4 step 1) of every pair of the
    level l_c, the coarsest level with sigma^2 h_max^2 |Gamma_h| / m <= 60
    (h_max its longest edge) and N_l >= 2 m: the coarse level must place the
    eigenvalues near sigma, O(sigma^2 h^2) off (the a priori estimate of
    Sec. 2.2, Lemma 2.2), within a fixed multiple of the window of about 2 pi m / |Gamma|
    that m vectors span around sigma; the constant 60 is a measured reading
    (the ellipsoid (1, 1.5, 2) at sigma = 40..100 and the 64 x 32 torus grid
    at sigma = 84..138 converge in 18-41 cycles at values 39-80, weighted
    Jacobi on the torus grid slows to 127-155 cycles at 79, and the cycle
    stalls from 156).  At
    most the finest level with N_l <= 12288 vertices is used; when that cap
    binds below level L and m was not given, m is raised to meet the rule
    there (a multiple of 4, at most 96).  When l_c = L the coarse eigensolve
    is the fine one and the start already returns the exact pairs.
 2. Start (Alg. 2 steps 2-4): the m level-l_c eigenvectors nearest the level's
    shift, prolongated to level L, relaxed once on the source problem of
    eq. (pb-f-aux-mat) with their coarse eigenvalues as Theta, then a
    Rayleigh-Ritz step in their span (no fixed coarse vectors).
 3. Adaptive shifts (Remark 4.1, Sec. 5.2: the coarse shift moves by the mean
    of Rayleigh quotients, compensating the drift of the discrete spectra
    between levels): on each level l_c <= l < L the correction operator is
    A_l - sigma_l M_l with sigma_l = sigma + Delta_l, Delta_l the mean over the
    block of (Rayleigh quotient on level l of the vector's values at the
    level-l vertices) - (its Ritz value).  Vertices of level l are the first
    N_l vertices of every finer level, so this is nodal injection.  The
    offsets are estimated after the first start, which is then repeated once
    with the coarse pairs nearest sigma + Delta_{l_c} (coarse eigenvalues
    shifted back by Delta_{l_c} as Theta); afterwards they are recomputed from
    the current block before every correction.
 4. Cycles: the V(nu1, nu2) correction of step 3 above with the per-level
    shifts, the truncated spectral inverse of A_{l_c} - sigma_{l_c} M_{l_c}
    as the coarse solve, and the Rayleigh-Ritz step in the span of the block
    alone; stopping rule and output as in step 5 above.

Level ramp (BFMG, Alg. 4; both schemes, ramp_cycles > 0).  Instead of the
seeded block (or the shifted start), the solve begins on a level l0 >= l_c
(default: the coarsest such level with N_l >= 2 m) with the m eigenpairs of
(A_l0, M_l0) nearest sigma (Alg. 4 step 1, a direct eigensolve), then for
every level l0 < l < L: the block prolongated from level l - 1, a
Rayleigh-Ritz step on level l, and ramp_cycles cycles of the scheme's own
cycle on the hierarchy cut at level l (Alg. 4 step 2: the V-cycle between the
coarse end and level l; the enriched scheme takes W_c = P_{0->l} Phi_c, the
shifted one its adaptive shifts relative to level l).  After each level the k
Ritz values nearest sigma are recorded (Alg. 4 step 3, the eigenvalue
approximation of that level).  On level L the block is prolongated, one
Rayleigh-Ritz step follows and the solve continues as usual.  With
max_cycles = ramp_cycles every level gets the same number of cycles: the
one-pass run behind the rates of Table 1.
"""
import math

import numpy as np
import scipy.linalg as sla

from . import fem, mesh, transfer, colour, rng


class LevelOps:
    """Matrices and transfer data of one level of the hierarchy."""

    def __init__(self, lv, P=None):
        self.xyz = lv.xyz
        self.tri = lv.tri
        self.parents = lv.parents
        self.A, self.M = fem.assemble(lv.xyz, lv.tri)
        self.D = fem.lumped_mass(self.M)
        self.P = P  # prolongation from the previous level to this one
        # colourings of the mesh graph: the pattern of M holds every edge, and
        # S = A - sigma M couples every edge for sigma != 0 (A alone can have
        # exact zeros, on edges opposite two right angles of the torus grid)
        self.colours = colour.greedy_colouring(self.M)
        self.n = self.A.shape[0]
        self.area = float(fem.triangle_areas(lv.xyz, lv.tri).sum())
        e = np.concatenate([lv.xyz[lv.tri[:, a]] - lv.xyz[lv.tri[:, b]]
                            for a, b in ((0, 1), (1, 2), (2, 0))])
        self.hmax = float(np.sqrt((e * e).sum(axis=1)).max())  # longest edge
        self._colours2 = None

    @property
    def colours2(self):
        """Distance-2 colouring (Kaczmarz smoother), computed on first use."""
        if self._colours2 is None:
            self._colours2 = colour.distance2_colouring(self.M)
        return self._colours2


def build_levels(kind, n_refine, axes=(1.0, 1.0, 1.0)):
    """Hierarchy with matrices on every level (Sec. 3 refinement; Sec. 2 assembly)."""
    lvls = mesh.hierarchy(kind, n_refine, axes=axes)
    out = []
    for l, lv in enumerate(lvls):
        P = None if l == 0 else transfer.prolongation(len(lvls[l - 1].xyz), lv.parents)
        out.append(LevelOps(lv, P))
    return out


def nearest_indices(values, target, count):
    """Indices of the `count` values nearest target; ties by value, then index."""
    v = np.asarray(values)
    order = np.lexsort((np.arange(len(v)), v, np.abs(v - target)))
    return order[:count]


def coarsest_level(levels, sigma):
    """l_c: the coarsest level with N_l >= 8 n_W(sigma) (Weyl count)."""
    n_w = levels[-1].area * max(sigma, 0.0) / (4.0 * math.pi)
    for l, lv in enumerate(levels):
        if lv.n >= 8.0 * n_w:
            return l
    return len(levels) - 1


class Smoother:
    """Gauss-Seidel (multicolour, symmetric), weighted Jacobi or Kaczmarz
    (multicolour, symmetric; Sec. 5.3) on A_l - sigma M_l.

    Kaczmarz projects the iterate onto the hyperplane of one equation at a
    time: x <- x + ((f_i - s_i^T x) / |s_i|^2) s_i with s_i row i of S (weight
    1).  The rows of one colour of the distance-2 colouring have disjoint
    patterns, so projecting them one after another equals projecting them at
    once, which is what a colour step here does."""

    def __init__(self, lv, sigma, kind, omega):
        self.kind = kind
        self.omega = omega
        colours = lv.colours2 if kind == "kaczmarz" else lv.colours
        nc = int(colours.max()) + 1
        self.rows = [np.flatnonzero(colours == c) for c in range(nc)]
        self.set_shift(lv, sigma)

    def set_shift(self, lv, sigma):
        """S = A_l - sigma M_l and what the sweeps derive from it."""
        self.S = (lv.A - sigma * lv.M).tocsr()
        self.d = self.S.diagonal()
        if self.kind == "kaczmarz":
            self.q = np.asarray(self.S.multiply(self.S).sum(axis=1)).ravel()  # |s_i|^2
            self.Sc = [self.S[r] for r in self.rows]  # the rows of each colour

    def sweep(self, x, f, forward=True):
        if self.kind == "jacobi":
            return x + self.omega * (f - self.S @ x) / self.d[:, None]
        order = range(len(self.rows)) if forward else range(len(self.rows) - 1, -1, -1)
        x = x.copy()
        for c in order:
            r = self.rows[c]
            if self.kind == "kaczmarz":
                Sr = self.Sc[c]
                t = (f[r] - Sr @ x) / self.q[r][:, None]
                x += Sr.T @ t
            else:
                x[r] += (f[r] - self.S[r] @ x) / self.d[r][:, None]
        return x


class BMG:
    """The BMG cycle on a fixed hierarchy and shift (see module docstring)."""

    def __init__(self, levels, sigma, m, nu1=2, nu2=2, smoother="gs", omega=0.85,
                 n_c=None, l_c=None):
        self.levels = levels
        self.sigma = float(sigma)
        self.m = m
        self.nu1, self.nu2 = nu1, nu2
        L = len(levels) - 1
        self.L = L
        self.l_c = coarsest_level(levels, sigma) if l_c is None else l_c
        self.smoothers = [Smoother(lv, sigma, smoother, omega) for lv in levels]
        # Alg. 2 step 1: coarse eigensolve on level 0
        lv0 = levels[0]
        lam0, phi0 = sla.eigh(lv0.A.toarray(), lv0.M.toarray())
        self.lam0, self.phi0 = lam0, phi0
        self.n_c = min(lv0.n, 32) if n_c is None else n_c
        idx = nearest_indices(lam0, self.sigma, self.n_c)
        W = phi0[:, np.sort(idx)]
        for l in range(1, L + 1):
            W = levels[l].P @ W
        self.W = W
        # truncated spectral inverse of A_0 - sigma M_0 (used when l_c == 0)
        x = lam0 - self.sigma
        g = np.where(np.abs(x) >= 1e-2 * max(1.0, abs(self.sigma)), 1.0 / np.where(x == 0, 1, x), 0.0)
        self.coarse_inv = (phi0 * g[None, :]) @ phi0.T

    # ---- correction: one V(nu1, nu2) cycle for (A_l - sigma M_l) e = f ----
    def vcycle(self, l, f):
        sm = self.smoothers[l]
        if l == self.l_c:
            if l == 0:
                return self.coarse_inv @ f
            e = np.zeros_like(f)
            for s in range(8):
                e = sm.sweep(e, f, forward=(s % 2 == 0))
            return e
        e = np.zeros_like(f)
        for _ in range(self.nu1):
            e = sm.sweep(e, f, forward=True)
        r = f - sm.S @ e
        P = self.levels[l].P
        ec = self.vcycle(l - 1, P.T @ r)
        e = e + P @ ec
        for _ in range(self.nu2):
            e = sm.sweep(e, f, forward=False)
        return e

    # ---- enriched Rayleigh-Ritz ----
    def rayleigh_ritz(self, U):
        lv = self.levels[self.L]
        Z = np.hstack([self.W, U])
        GA = Z.T @ (lv.A @ Z)
        GM = Z.T @ (lv.M @ Z)
        GA = 0.5 * (GA + GA.T)
        GM = 0.5 * (GM + GM.T)
        # SVQB (Stathopoulos & Wu 2002): scale to unit diagonal, eigendecompose,
        # drop directions with eigenvalue below 1e-12 of the largest.
        s = 1.0 / np.sqrt(np.diag(GM))
        d, V = np.linalg.eigh(GM * s[:, None] * s[None, :])
        keep = d > 1e-12 * d.max()
        T = (s[:, None] * V[:, keep]) / np.sqrt(d[keep])[None, :]
        C = T.T @ (GA - self.sigma * GM) @ T
        C = 0.5 * (C + C.T)
        mu, Q = np.linalg.eigh(C)
        if len(mu) < self.m:
            raise RuntimeError("enriched space lost rank below m")
        sel = nearest_indices(mu, 0.0, self.m)
        sel = sel[np.argsort(mu[sel], kind="stable")]
        Y = T @ Q[:, sel]
        return Z @ Y, mu[sel] + self.sigma

    def residual(self, U, theta):
        lv = self.levels[self.L]
        return lv.A @ U - (lv.M @ U) * theta[None, :]

    def certificates(self, R, theta, ret):
        """(rho, delta) for the returned Ritz pairs `ret` (indices into theta)."""
        D = self.levels[self.L].D
        rho = 2.0 * np.sqrt(np.sum(R * R / D[:, None], axis=0))
        cl = cluster_ids(theta)
        delta = np.empty(len(theta))
        for i in range(len(theta)):
            out = theta[cl != cl[i]]
            delta[i] = np.min(np.abs(out - theta[i])) if len(out) else 1e-2 * max(abs(theta[i]), 1.0)
        return rho[ret], delta[ret]


def cluster_ids(theta):
    """Cluster label of each (ascending) Ritz value: relative gap < 1e-2 joins."""
    ids = np.zeros(len(theta), dtype=np.int64)
    for j in range(1, len(theta)):
        gap = theta[j] - theta[j - 1]
        scale = max(abs(theta[j]), abs(theta[j - 1]), 1.0)
        ids[j] = ids[j - 1] + (0 if gap < 1e-2 * scale else 1)
    return ids


def normalise_signs(U):
    """Make the largest-magnitude entry of each column positive (first on ties)."""
    U = U.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def default_m(k, sigma):
    """Block width: 4 ceil(1.25 k / 4) for sigma = 0, 4 ceil(1.5 k / 4) otherwise."""
    f = 1.25 if sigma == 0 else 1.5
    return 4 * int(math.ceil(f * k / 4.0))


def ramp_start_level(levels, m, l_c):
    """Default first level of a ramp: the coarsest l >= l_c with N_l >= 2 m."""
    for l in range(l_c, len(levels)):
        if levels[l].n >= 2 * m:
            return l
    return len(levels) - 1


def level_ramp(levels, k, sigma, m, l0, ramp_cycles, cycle_on):
    """The level ramp of the module docstring up to level L - 1.

    cycle_on(l) gives the scheme's cycle object on the hierarchy cut at
    level l; it must offer rayleigh_ritz(U), vcycle(l, f) and adapt(U, theta)
    (the shifts before a correction; nothing for the enriched scheme).
    Returns (U on level L - 1 or l0, row of recorded values per level).
    """
    L = len(levels) - 1
    rows = np.full((L + 1, k), np.nan)
    lv0 = levels[l0]
    lam, phi = sla.eigh(lv0.A.toarray(), lv0.M.toarray())
    U = phi[:, np.sort(nearest_indices(lam, sigma, m))]
    for lev in range(l0, L):
        lv = levels[lev]
        if lev > l0:
            U = lv.P @ U
        cyc = cycle_on(lev)
        U, theta = cyc.rayleigh_ritz(U)
        for _ in range(ramp_cycles if lev > l0 else 0):
            cyc.adapt(U, theta)
            R = lv.A @ U - (lv.M @ U) * theta[None, :]
            U, theta = cyc.rayleigh_ritz(U + cyc.vcycle(lev, -R))
        rows[lev] = theta[np.sort(nearest_indices(theta, sigma, k))]
    if l0 < L:
        U = levels[L].P @ U
    return U, rows


def solve(levels, k, sigma=0.0, tol=1e-8, m=None, nu1=2, nu2=2, smoother="gs",
          omega=0.85, max_cycles=200, seed=0, angle_tol=1e-7, U0=None,
          n_c=None, l_c=None, history=False, scheme="auto", ramp_cycles=0, ramp_level=None):
    """The k eigenpairs of (A_L, M_L) nearest sigma by BMG.

    scheme: "enriched" (fixed shift, coarse vectors in every Ritz step),
    "shifted" (the interior-shift scheme of the module docstring) or "auto"
    (shifted when sigma > 0).  ramp_cycles > 0: start with the level ramp
    (BFMG) from ramp_level (None: the default of ramp_start_level).
    Returns (evals ascending, M-orthonormal evecs N_L x k, info dict); with a
    ramp, info["ramp_evals"] holds the recorded values per level (row L: the
    returned ones) and info["ramp_start"] the first level.
    """
    if scheme == "auto":
        scheme = "shifted" if sigma > 0 else "enriched"
    if scheme == "shifted":
        return solve_shifted(levels, k, sigma, tol, m, nu1, nu2, smoother, omega, max_cycles,
                             angle_tol, l_c, history, ramp_cycles, ramp_level)
    m = default_m(k, sigma) if m is None else m
    bmg = BMG(levels, sigma, m, nu1, nu2, smoother, omega, n_c, l_c)
    lv = levels[-1]
    rows = None
    if ramp_cycles > 0:
        l0 = ramp_start_level(levels, m, bmg.l_c) if ramp_level is None else ramp_level
        if not bmg.l_c <= l0 < len(levels):
            raise ValueError("ramp level outside [l_c, L]")

        def cycle_on(lev):
            c = BMG(levels[:lev + 1], sigma, m, nu1, nu2, smoother, omega, bmg.n_c, bmg.l_c)
            c.adapt = lambda U, theta: None
            return c
        U, rows = level_ramp(levels, k, sigma, m, l0, ramp_cycles, cycle_on)
    else:
        U = rng.gaussian_block(lv.n, m, seed) if U0 is None else np.array(U0, dtype=np.float64)
    U, theta = bmg.rayleigh_ritz(U)
    hist = []
    cycles = 0
    converged = False
    while True:
        R = bmg.residual(U, theta)
        ret = nearest_indices(theta, sigma, k)
        rho, delta = bmg.certificates(R, theta, ret)
        th = theta[ret]
        ok_kt = np.all(rho ** 2 / delta <= 0.1 * tol * np.maximum(np.abs(th), 1.0))
        ok_dk = np.max(rho / delta) <= angle_tol
        if history:
            hist.append((theta.copy(), rho.copy(), delta.copy()))
        if ok_kt and ok_dk:
            converged = True
            break
        if cycles >= max_cycles:
            break
        E = bmg.vcycle(bmg.L, -R)
        U, theta = bmg.rayleigh_ritz(U + E)
        cycles += 1
    ret = np.sort(nearest_indices(theta, sigma, k))
    order = ret[np.argsort(theta[ret], kind="stable")]
    evals = theta[order]
    evecs = normalise_signs(U[:, order])
    info = dict(cycles=cycles, converged=converged, rho=rho, delta=delta, m=m,
                l_c=bmg.l_c, n_c=bmg.n_c, history=hist)
    if rows is not None:
        rows[-1] = evals
        info.update(ramp_evals=rows, ramp_start=l0)
    return evals, evecs, info


# ---------------------------------------------------------------- interior --

MAX_COARSE_EIG_VERTICES = 12288


SHIFT_RESOLUTION = 60.0


def shifted_coarse_level(levels, sigma, m, m_given=True):
    """(l_c, m) for the shifted scheme: the coarsest l with
    sigma^2 h_max,l^2 |Gamma_h| / m <= 60 and N_l >= 2 m, capped at the finest
    level with N_l <= 12288; when the cap binds below the finest level and m
    was not given, m is raised to meet the rule there (multiple of 4, at most
    96 and at most N_cap / 2).  At l_c = L the coarse solve is exact."""
    area = levels[-1].area
    cap = 0
    for l, lv in enumerate(levels):
        if lv.n <= MAX_COARSE_EIG_VERTICES:
            cap = l
    for l, lv in enumerate(levels):
        if sigma * sigma * lv.hmax ** 2 * area / m <= SHIFT_RESOLUTION and lv.n >= 2 * m:
            if l <= cap:
                return l, m
            break
    if not m_given and cap < len(levels) - 1:
        want = 4 * int(math.ceil(sigma * sigma * levels[cap].hmax ** 2 * area / SHIFT_RESOLUTION / 4.0))
        m = min(96, max(m, want), levels[cap].n // 2 // 4 * 4)
    return cap, m


def injected_rayleigh_offsets(levels, U, theta, l_c):
    """Delta_l = mean_i (RQ_l(U_i restricted to the level-l vertices) - theta_i)."""
    L = len(levels) - 1
    off = np.zeros(L + 1)
    for l in range(l_c, L):
        lv = levels[l]
        X = U[:lv.n]
        rq = np.einsum("ij,ij->j", X, lv.A @ X) / np.einsum("ij,ij->j", X, lv.M @ X)
        off[l] = float(np.mean(rq - theta))
    return off


class ShiftedBMG:
    """The interior-shift cycle (module docstring, steps 1-4)."""

    def __init__(self, levels, sigma, m, l_c, nu1=2, nu2=2, smoother="gs", omega=0.85):
        self.levels = levels
        self.sigma = float(sigma)
        self.m = m
        self.l_c = l_c
        self.nu1, self.nu2 = nu1, nu2
        self.kind = smoother
        self.omega = omega
        self.L = len(levels) - 1
        lc = levels[l_c]
        # coarse eigensolve of level l_c (Alg. 2 step 1, Alg. 4 step 1)
        self.lam, self.phi = sla.eigh(lc.A.toarray(), lc.M.toarray())
        self.smoothers = {}
        self.set_offsets(np.zeros(self.L + 1))

    def set_offsets(self, off):
        """Per-level shifts sigma_l = sigma + off[l] (Remark 4.1)."""
        self.off = np.array(off, dtype=np.float64)
        for l in range(self.l_c + 1, self.L + 1):
            lv, sig = self.levels[l], self.sigma + self.off[l]
            if l not in self.smoothers:
                self.smoothers[l] = Smoother(lv, sig, self.kind, self.omega)
            else:
                self.smoothers[l].set_shift(lv, sig)
        x = self.lam - (self.sigma + self.off[self.l_c])
        keep = np.abs(x) >= 1e-2 * max(1.0, abs(self.sigma))
        self.g = np.where(keep, 1.0 / np.where(keep, x, 1.0), 0.0)

    def vcycle(self, l, f):
        if l == self.l_c:
            return self.phi @ (self.g[:, None] * (self.phi.T @ f))
        sm = self.smoothers[l]
        e = np.zeros_like(f)
        for _ in range(self.nu1):
            e = sm.sweep(e, f, forward=True)
        r = f - sm.S @ e
        P = self.levels[l].P
        e = e + P @ self.vcycle(l - 1, P.T @ r)
        for _ in range(self.nu2):
            e = sm.sweep(e, f, forward=False)
        return e

    def rayleigh_ritz(self, U):
        """Exact Rayleigh-Ritz in span(U); the m pairs nearest sigma."""
        lv = self.levels[self.L]
        GA = U.T @ (lv.A @ U)
        GM = U.T @ (lv.M @ U)
        GA = 0.5 * (GA + GA.T)
        GM = 0.5 * (GM + GM.T)
        s = 1.0 / np.sqrt(np.diag(GM))
        d, V = np.linalg.eigh(GM * s[:, None] * s[None, :])
        keep = d > 1e-12 * d.max()
        T = (s[:, None] * V[:, keep]) / np.sqrt(d[keep])[None, :]
        C = T.T @ (GA - self.sigma * GM) @ T
        mu, Q = np.linalg.eigh(0.5 * (C + C.T))
        if len(mu) < self.m:
            raise RuntimeError("block lost rank below m")
        sel = nearest_indices(mu, 0.0, self.m)
        sel = sel[np.argsort(mu[sel], kind="stable")]
        return U @ (T @ Q[:, sel]), mu[sel] + self.sigma

    def start(self):
        """Prolongated coarse pairs nearest the level-l_c shift, one source
        relaxation (eq. pb-f-aux-mat) and a Ritz step (Alg. 2 steps 2-4)."""
        lv = self.levels[self.L]
        sel = np.sort(nearest_indices(self.lam, self.sigma + self.off[self.l_c], self.m))
        U = self.phi[:, sel]
        for l in range(self.l_c + 1, self.L + 1):
            U = self.levels[l].P @ U
        theta0 = self.lam[sel] - self.off[self.l_c]
        if self.l_c < self.L:
            R = lv.A @ U - (lv.M @ U) * theta0[None, :]
            U = U + self.vcycle(self.L, -R)
        return self.rayleigh_ritz(U)


def solve_shifted(levels, k, sigma, tol=1e-8, m=None, nu1=2, nu2=2, smoother="gs", omega=0.85,
                  max_cycles=200, angle_tol=1e-7, l_c=None, history=False, ramp_cycles=0,
                  ramp_level=None):
    """The k eigenpairs nearest an interior shift sigma (module docstring, steps 1-4)."""
    m_given = m is not None
    m = default_m(k, sigma) if m is None else m
    if l_c is None:
        l_c, m = shifted_coarse_level(levels, sigma, m, m_given)
    bmg = ShiftedBMG(levels, sigma, m, l_c, nu1, nu2, smoother, omega)
    lv = levels[-1]
    rows = None
    if ramp_cycles > 0:
        l0 = ramp_start_level(levels, m, l_c) if ramp_level is None else ramp_level
        if not l_c <= l0 < len(levels):
            raise ValueError("ramp level outside [l_c, L]")

        def cycle_on(lev):
            c = ShiftedBMG(levels[:lev + 1], sigma, m, l_c, nu1, nu2, smoother, omega)
            c.adapt = lambda U, theta: c.set_offsets(
                injected_rayleigh_offsets(levels[:lev + 1], U, theta, l_c))
            return c
        U, rows = level_ramp(levels, k, sigma, m, l0, ramp_cycles, cycle_on)
        U, theta = bmg.rayleigh_ritz(U)
    else:
        U, theta = bmg.start()
        if l_c < bmg.L:
            bmg.set_offsets(injected_rayleigh_offsets(levels, U, theta, l_c))
            U, theta = bmg.start()
    cert = BMG.certificates
    hist = []
    cycles = 0
    converged = False
    while True:
        R = lv.A @ U - (lv.M @ U) * theta[None, :]
        ret = nearest_indices(theta, sigma, k)
        rho, delta = cert(bmg, R, theta, ret)
        th = theta[ret]
        ok_kt = np.all(rho ** 2 / delta <= 0.1 * tol * np.maximum(np.abs(th), 1.0))
        ok_dk = np.max(rho / delta) <= angle_tol
        if history:
            hist.append((theta.copy(), rho.copy(), delta.copy()))
        if ok_kt and ok_dk:
            converged = True
            break
        if cycles >= max_cycles:
            break
        if l_c < bmg.L:
            bmg.set_offsets(injected_rayleigh_offsets(levels, U, theta, l_c))
        U, theta = bmg.rayleigh_ritz(U + bmg.vcycle(bmg.L, -R))
        cycles += 1
    ret = np.sort(nearest_indices(theta, sigma, k))
    order = ret[np.argsort(theta[ret], kind="stable")]
    evals = theta[order]
    evecs = normalise_signs(U[:, order])
    info = dict(cycles=cycles, converged=converged, rho=rho, delta=delta, m=m, l_c=l_c, n_c=0,
                offsets=bmg.off.copy(), history=hist, scheme="shifted")
    if rows is not None:
        rows[-1] = evals
        info.update(ramp_evals=rows, ramp_start=l0)
    return evals, evecs, info
