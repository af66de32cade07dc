"""The two-grid cascade (Alg. 1, Remark 3.1) of the HIP path against the oracle's.

bmg_two_grid relaxes each fine source problem by Kaczmarz sweeps with one
shift per followed pair.  On the ellipsoid (1, 1.5, 2), whose spectrum has no
exact multiplicities (so the coarse eigenvectors are unique up to sign), the
per-level values and the final vectors match the oracle's cascade with the
same sweeps.  On the sphere the values approach l (l + 1) level by level.
Argument checks and the cascade of length zero (top = level_H: the coarse
eigenvalues) complete it.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


@pytest.mark.parametrize("nu,idx", [(5, list(range(1, 16))), (2, [0, 7, 30, 31]), (5, [40])])
def test_cascade_matches_oracle_on_the_ellipsoid(lib, nu, idx):
    from oracle import bmg as ob, twogrid
    lv = ob.build_levels("ellipsoid", 5, axes=(1.0, 1.5, 2.0))
    ref_rows, ref_U = twogrid.two_grid(lv, 2, np.array(idx), source="kaczmarz", nu=nu)
    with lib.Hierarchy("ellipsoid", 5, axes=(1.0, 1.5, 2.0)) as h:
        rows, U = h.two_grid(2, idx, nu=nu)
    assert np.all(np.isnan(rows[:2]))
    for l in range(2, 6):
        rel = np.max(np.abs(rows[l] - ref_rows[l]) / np.abs(ref_rows[l]).clip(1.0))
        assert rel < 1e-9, (l, rel)
    L = lv[-1]
    G = U.T @ (L.M @ ref_U)
    assert np.allclose(np.abs(np.diag(G)), 1.0, atol=1e-8)  # the same vectors up to sign
    assert np.allclose(np.einsum("ij,ij->j", U, L.M @ U), 1.0, atol=1e-10)


def test_cascade_on_the_sphere_approaches_the_continuum(lib):
    exact = np.array([2.0] * 3 + [6.0] * 5 + [12.0] * 7)
    with lib.Hierarchy("sphere", 7) as h:
        rows, U = h.two_grid(2, list(range(1, 16)), nu=5, evecs=False)
    assert U is None
    err = np.array([np.max(np.abs(rows[l] - exact)) for l in range(2, 8)])
    assert np.all(np.diff(err) < 0), err
    assert err[-1] < 0.02 * err[0], err


def test_cascade_edge_cases(lib):
    from oracle import bmg as ob
    import scipy.linalg as sla
    lv = ob.build_levels("sphere", 3)
    with lib.Hierarchy("sphere", 3) as h:
        rows, U = h.two_grid(3, [0, 5, 100], top=3)  # no cascade: the level's own pairs
        d = sla.eigh(lv[3].A.toarray(), lv[3].M.toarray(), eigvals_only=True)
        np.testing.assert_allclose(rows[3], d[[0, 5, 100]], rtol=1e-10, atol=1e-12)
        assert np.all(np.isnan(rows[:3]))
        rows, U = h.two_grid(1, [3], top=2, nu=0)  # nu = 0: the prolongated coarse vector's RQ
        u = lv[2].P @ ob.sla.eigh(lv[1].A.toarray(), lv[1].M.toarray())[1][:, 3]
        rq = u @ (lv[2].A @ u) / (u @ (lv[2].M @ u))
        assert abs(rows[2, 0] - rq) < 1e-10 * rq and np.all(np.isnan(rows[3]))
        for bad in (dict(level_H=4, idx=[0]), dict(level_H=1, idx=[42]), dict(level_H=2, idx=[0], top=1),
                    dict(level_H=1, idx=[0], nu=65)):
            with pytest.raises(lib.BMGError) as e:
                h.two_grid(**bad)
            assert e.value.status == lib.EINVAL
