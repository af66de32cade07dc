"""Parity of the interior-shift scheme (HIP path through the C ABI) with the oracle.

Kernels: the coarse spectral solve and the adaptive-shift offsets, element by
element against oracle/bmg.py.  Solves: C3 (ellipsoid (1, 1.5, 2) refined 7
times, the 16 eigenpairs nearest sigma = 100, 24 vectors) in both precisions
against ARPACK shift-invert on the oracle's pencil and the stored oracle
eigenvalues; the 5-refinement ellipsoid at sigma = 40 against the oracle's own
shifted BMG (pairs, cycle counts, final adaptive shift); a coarse level equal
to the finest (exact start).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


def _nearest(ev, sigma, k):
    return np.sort(np.argsort(np.abs(ev - sigma), kind="stable")[:k])


def _check_pairs(ev, U, M, ref_ev, ref_U, sigma, k, rel_tol=1e-8, sine_tol=1e-6):
    from oracle import reference
    idx = _nearest(ref_ev, sigma, k)
    rel, sine = reference.compare(ev, U, ref_ev[idx], ref_U[:, idx], M, ref_ev, ref_U)
    assert rel < rel_tol, rel
    assert sine < sine_tol, sine
    assert np.max(np.abs(U.T @ (M @ U) - np.eye(k))) < 1e-10
    i = np.argmax(np.abs(U), axis=0)
    assert np.all(U[i, np.arange(k)] > 0)
    assert np.all(np.diff(ev) >= 0)
    return rel, sine


@pytest.fixture(scope="module")
def ell(lib):
    from oracle import bmg as ob
    lv = ob.build_levels("ellipsoid", 5, axes=(1.0, 1.5, 2.0))
    return lib.Hierarchy("ellipsoid", 5, axes=(1.0, 1.5, 2.0)), lv


# ----------------------------------------------------------------- kernels --

@pytest.mark.parametrize("level", [3, 4])
@pytest.mark.parametrize("m", [4, 24, 96])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_coarse_solve_kernel(lib, ell, level, m, dtype):
    import torch
    from oracle import bmg as ob
    h, lv = ell
    n = lv[level].n
    sh = ob.ShiftedBMG(lv[: level + 1], 100.0, m, level)  # l_c = level = its finest
    f = np.random.default_rng(level * 100 + m).standard_normal((n, m))
    ref = sh.vcycle(level, f)
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    x = torch.tensor(f, dtype=tdt, device="cuda")
    y = torch.empty_like(x)
    h.apply("coarse_solve", x=x, y=y, level=level, sigma=100.0)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    # FP64: two eigensolvers (LAPACK, rocSOLVER) give the same operator to
    # ~1e-12 of its norm; FP32: n-term sums of rounded products
    assert err < (1e-9 if dtype == "fp64" else 1e-4), err


def test_coarse_solve_kernel_drops_modes_at_the_shift(lib, ell):
    import torch
    from oracle import bmg as ob
    h, lv = ell
    sh0 = ob.ShiftedBMG(lv[:4], 1.0, 8, 3)
    sigma = float(sh0.lam[40] + 0.001)
    sh = ob.ShiftedBMG(lv[:4], sigma, 8, 3)
    f = lv[3].M @ sh.phi[:, 36:44]  # includes the mode within the truncation window
    x = torch.tensor(f, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    h.apply("coarse_solve", x=x, y=y, level=3, sigma=sigma)
    torch.cuda.synchronize()
    ref = sh.vcycle(3, f)
    got = y.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))
    assert np.max(np.abs(got[:, 4])) < 1e-9  # column 4 is mode 40: dropped


@pytest.mark.parametrize("lo", [0, 2, 4])
def test_shift_offsets_kernel(lib, ell, lo):
    import torch
    from oracle import bmg as ob
    h, lv = ell
    L = len(lv) - 1
    m = 24
    U = np.random.default_rng(lo).standard_normal((lv[L].n, m))
    theta = np.linspace(40.0, 60.0, m)
    ref = ob.injected_rayleigh_offsets(lv, U, theta, lo) + 50.0
    y = torch.full((L + 1,), -1.0, dtype=torch.float64, device="cuda")
    h.apply("shift_offsets", x=torch.tensor(U, device="cuda"), f=torch.tensor(theta, device="cuda"), y=y,
            level=L, m=m, l_c=lo, sigma=50.0)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    assert np.all(got[:lo] == -1.0)  # not written
    assert np.max(np.abs(got[lo:] - ref[lo:]) / np.abs(ref[lo:])) < 1e-12


# ------------------------------------------------------------------ solves --

@pytest.fixture(scope="module")
def c3(lib):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("ellipsoid", 7, axes=(1.0, 1.5, 2.0))
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 40, 100.0)
    gold = np.array([float(x) for x in open(os.path.join(GOLDEN, "c3_ellipsoid_ref7_eigs.txt"))
                     if not x.startswith("#")])
    return lib.Hierarchy("ellipsoid", 7, axes=(1.0, 1.5, 2.0)), lv, ref_ev, ref_U, gold


@pytest.mark.parametrize("precision,smoother", [("mixed", "jacobi"), ("fp64", "gs"), ("fp64", "jacobi")])
def test_c3_parity(lib, c3, precision, smoother):
    h, lv, ref_ev, ref_U, gold = c3
    ev, U, st = h.solve(16, 100.0, 1e-8, m=24, precision=precision, smoother=smoother)
    assert st["converged"] == 1 and st["scheme"] == 2 and st["l_c"] == 5 and st["n_c"] == 0
    _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 100.0, 16)
    near = gold[_nearest(gold, 100.0, 16)]
    per_pair = np.abs(ev - near) / np.abs(near)
    assert np.max(per_pair) < 1e-8, per_pair
    # the oracle (weighted Jacobi, FP64) converged in 26 cycles; its GS run in 21
    assert st["cycles"] <= 32, st["cycles"]
    # the level-5 shift sits above sigma by the level's eigenvalue offset
    assert 101.5 < st["lc_shift"] < 103.5, st["lc_shift"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ellipsoid_sigma40_against_oracle_bmg(lib, ell, precision):
    from oracle import bmg as ob
    h, lv = ell
    oev, oU, info = ob.solve(lv, 16, 40.0, 1e-8, m=24, smoother="jacobi", omega=0.85)
    assert info["converged"]
    ev, U, st = h.solve(16, 40.0, 1e-8, m=24, precision=precision, smoother="jacobi")
    assert st["converged"] == 1 and st["l_c"] == info["l_c"] == 4
    from oracle import reference
    rel, sine = reference.compare(ev, U, oev, oU, lv[-1].M)
    assert rel < 1e-8 and sine < 1e-6
    assert abs(st["cycles"] - info["cycles"]) <= (0 if precision == "fp64" else 3), (st["cycles"], info["cycles"])
    # the adaptive shift of level l_c in the last cycle: the same block gives the same shift
    assert abs(st["lc_shift"] - (40.0 + info["offsets"][4])) < (1e-8 if precision == "fp64" else 1e-5)


def test_coarse_level_equal_to_finest_is_exact(lib):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("torus", 1)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 40, 100.0)
    with lib.Hierarchy("torus", 1) as h:
        ev, U, st = h.solve(16, 100.0, 1e-8, precision="mixed", smoother="jacobi")
        assert st["converged"] == 1 and st["cycles"] == 0 and st["l_c"] == 1
        _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 100.0, 16, rel_tol=1e-12, sine_tol=1e-9)


def test_small_shift_wide_block_uses_a_level_with_2m_pairs(lib):
    # sigma = 12 with k = 30 (m = 48): the Weyl rule alone would pick the
    # 12-vertex level, which holds fewer eigenpairs than the start block needs
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 3)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 60, 12.0)
    with lib.Hierarchy("sphere", 3) as h:
        ev, U, st = h.solve(30, 12.0, 1e-8, precision="mixed", smoother="jacobi")
        assert st["converged"] == 1 and st["m"] == 48 and st["l_c"] == 2
        _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 12.0, 30)
        with pytest.raises(lib.BMGError) as e:  # an explicit level with fewer than m vertices
            h.solve(30, 12.0, 1e-8, l_c=0)
        assert e.value.status == lib.EINVAL


@pytest.mark.parametrize("scheme", ["shifted", "enriched"])
def test_small_shift_both_schemes(lib, scheme):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 4)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 16, 6.0)
    with lib.Hierarchy("sphere", 4) as h:
        ev, U, st = h.solve(5, 6.0, 1e-8, m=12, precision="mixed", smoother="jacobi", scheme=scheme)
        assert st["converged"] == 1 and st["scheme"] == (2 if scheme == "shifted" else 1)
        _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 6.0, 5)
        oev, oU, info = ob.solve(lv, 5, 6.0, 1e-8, m=12, smoother="jacobi", scheme=scheme)
        assert info["converged"] and abs(info["cycles"] - st["cycles"]) <= 2


def test_rank_loss_reports_noconv_without_output(lib):
    # a zero initial block leaves the Ritz step without m independent
    # directions: ENOCONV with the reason, evals untouched, no evecs written
    with lib.Hierarchy("sphere", 3) as h:
        blk = np.zeros((h.N, 16))
        evals = None
        with pytest.raises(lib.BMGError) as ei:
            h.solve(9, 0.0, 1e-8, m=16, initial_block=blk, n_c=12, scheme="enriched")
        assert ei.value.status == -4 and "lost rank" in str(ei.value)
        ev, U, st = h.solve(9, 0.0, 1e-8, m=16, initial_block=blk, n_c=12, allow_noconv=True,
                            scheme="enriched")
        assert st["status"] == -4 and np.all(ev == 0.0) and np.all(U == 0.0)
        del evals


# ---------------------------------------------------- default block width --

def test_default_width_covers_a_cut_multiplet(lib):
    # sigma = 101.6 with k = 7: the seven eigenvalues nearest sigma lie in the
    # 21-fold multiplet l = 10 (lambda ~ 110).  The default width (12) ends
    # inside it and the block barely converges; the width taken from the
    # coarse level's spectrum holds the whole multiplet.
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 5)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 40, 101.6)
    with lib.Hierarchy("sphere", 5) as h:
        ev, U, st = h.solve(7, 101.6, 1e-8, precision="mixed", smoother="jacobi")
        assert st["converged"] == 1 and st["m"] >= 24, (st["m"], st["cycles"])
        _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 101.6, 7)
        # an explicit width is kept as given
        ev2, U2, st2 = h.solve(7, 101.6, 1e-8, m=28, precision="mixed", smoother="jacobi")
        assert st2["m"] == 28


def test_default_width_covers_a_split_cluster_at_zero(lib):
    # a nearly round ellipsoid: its l = 4 group (nine eigenvalues, split by
    # under 7%) starts at index 16, so k = 17 cuts it, and the default width
    # (24) ends inside the group as well; the widened block reaches past it
    from oracle import bmg as ob, reference
    axes = (1.961, 1.8452, 1.8167)
    lv = ob.build_levels("ellipsoid", 5, axes=axes)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 40, 0.0)
    with lib.Hierarchy("ellipsoid", 5, axes=axes) as h:
        ev, U, st = h.solve(17, 0.0, 1e-8, precision="mixed", smoother="jacobi")
        assert st["converged"] == 1 and st["m"] >= 28, (st["m"], st["cycles"])
        _check_pairs(ev, U, lv[-1].M, ref_ev, ref_U, 0.0, 17)
