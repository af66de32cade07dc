"""The a posteriori estimator (eq. est-res) of the HIP path against the oracle's.

bmg_estimate on eigenvectors of the library's own solves: the per-pair
totals of the three terms and eta against oracle/estimator.py on the same
vectors (sphere with the geometric term, ellipsoid and the torus grid without
it), the per-triangle sums against the oracle's, eta = O(h) on the sphere,
and the argument checks.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


@pytest.mark.parametrize("kind,nref,kw,k,sigma", [
    ("sphere", 5, {}, 16, 0.0),
    ("ellipsoid", 4, dict(axes=(1.0, 1.5, 2.0)), 9, 0.0),
    ("torus", 1, {}, 12, 0.0),
])
def test_estimator_matches_oracle(lib, kind, nref, kw, k, sigma):
    import torch
    from oracle import estimator
    with lib.Hierarchy(kind, nref, **kw) as h:
        ev, U, st = h.solve(k, sigma, 1e-8, evecs="device")
        eta, parts, e2 = h.estimate(ev, U, per_triangle=True)
        L = h.n_levels - 1
        xyz, tri = h.export(L, "xyz"), h.export(L, "tri")
    Uh = U.double().cpu().numpy()
    ref_parts, ref_eta = estimator.estimate(xyz, tri, Uh, ev, sphere=(kind == "sphere"))
    # the constant mode (lambda ~ 1e-15) has terms at the rounding level:
    # absolute floor 1e-14 of the largest term
    floor = 1e-14 * ref_parts.sum(axis=1).max()
    np.testing.assert_allclose(parts, ref_parts.sum(axis=1), rtol=1e-11, atol=floor)
    np.testing.assert_allclose(eta, ref_eta, rtol=1e-11, atol=np.sqrt(floor))
    np.testing.assert_allclose(e2.cpu().numpy(), ref_parts.sum(axis=(0, 2)), rtol=1e-11, atol=floor)
    if kind != "sphere":
        assert np.all(parts[2] == 0.0)
    else:
        assert np.all(parts[2] > 0.0)


def test_estimator_rate_on_the_sphere(lib):
    prev = None
    for nref in (5, 6, 7):
        with lib.Hierarchy("sphere", nref) as h:
            ev, U, st = h.solve(16, 0.0, 1e-8, evecs="device")
            eta, parts, _ = h.estimate(ev, U)
        if prev is not None:
            ratio = prev / eta[1:]  # pair 0 is the constant mode: eta at the rounding level
            assert np.all(ratio > 1.95) and np.all(ratio < 2.05), ratio
        assert eta[0] < 1e-10
        prev = eta[1:]


def test_estimator_arguments(lib):
    with lib.Hierarchy("sphere", 3) as h:
        ev, U, st = h.solve(4, 0.0, 1e-8, m=8, evecs="device")
        with pytest.raises(lib.BMGError) as e:
            h.estimate(ev, U, level=4)
        assert e.value.status == lib.EINVAL
        with pytest.raises(lib.BMGError) as e:
            h.estimate(np.array([np.nan, 1, 2, 3.0]), U)
        assert e.value.status == lib.EINVAL
