"""The level ramp (BFMG, Alg. 4) of the HIP path against the oracle's.

Per-level eigenvalue approximations (stats["ramp_evals"]) of the library
against oracle/bmg.py level_ramp on the same hierarchy and options (one cycle
per level, the one-pass run of Table 1), both schemes; the one-pass rates
r = 1 for lambda = 2, 6, 12 up to the 655362-vertex sphere (Table 1) and
lambda = 20 with the interior shift (Table 2), against the closed-form
eigenvalues l (l + 1); a ramp followed by the usual certified solve against
the stored oracle eigenvalues; the range checks of ramp_level.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MULTIPLETS = [(2.0, slice(1, 4)), (6.0, slice(4, 9)), (12.0, slice(9, 16))]


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


@pytest.fixture(scope="module")
def sphere6(lib):
    from oracle import bmg as ob
    return lib.Hierarchy("sphere", 6), ob.build_levels("sphere", 6)


def _rates(err, n):
    return np.log(err[:-1] / err[1:]) / np.log(n[1:] / n[:-1])


@pytest.mark.parametrize("precision,smoother,nu", [("fp64", "gs", (2, 2)), ("fp64", "jacobi", (2, 2)),
                                                   ("mixed", "jacobi", (2, 2)), ("fp64", "gs", (1, 0))])
def test_one_pass_rows_match_oracle(lib, sphere6, precision, smoother, nu):
    # m = 16 = 1 + 3 + 5 + 7: the start block is every eigenvector of the
    # level-1 multiplets below a gap (an m that cuts through a degenerate
    # multiplet of the icosahedral mesh leaves the start basis to the
    # eigensolver, and the library's and LAPACK's differ)
    from oracle import bmg as ob
    h, lv = sphere6
    oev, oU, info = ob.solve(lv, 16, 0.0, 1e-8, m=16, smoother=smoother, nu1=nu[0], nu2=nu[1],
                             ramp_cycles=1, max_cycles=1)
    ev, U, st = h.solve(16, 0.0, 1e-8, m=16, smoother=smoother, precision=precision, nu1=nu[0],
                        nu2=nu[1], ramp_cycles=1, max_cycles=1, allow_noconv=True)
    assert st["ramp_start"] == info["ramp_start"] == 1 and st["cycles"] == 1
    got, ref = st["ramp_evals"], info["ramp_evals"]
    assert np.all(np.isnan(got[0])) and np.all(np.isfinite(got[1:]))
    np.testing.assert_array_equal(got[-1], ev)
    # differences from rounding order only (FP64), or from the FP32 correction
    # (mixed), relative to each level's discretisation error |lambda_l - l(l+1)|.
    # The enriched space [W_c, U] is close to dependent on the low levels
    # (both hold the smooth modes), which amplifies rounding: perturbing the
    # oracle's start vectors by 1e-15 moves these values by up to 5e-8 of the
    # discretisation error
    exact = np.array([0.0] + [2.0] * 3 + [6.0] * 5 + [12.0] * 7)
    scale = np.maximum(np.abs(ref[1:] - exact), 1e-6)
    rel = np.abs(got[1:] - ref[1:]) / scale
    assert np.max(rel) < (1e-6 if precision == "fp64" else 1e-4), np.max(rel, axis=1)


def test_one_pass_rates_table1_c4(lib):
    # Table 1 on the 655362-vertex sphere (levels 0..8): one cycle per level,
    # the l = 1, 2, 3 multiplets converge at r = 1 against l (l + 1)
    with lib.Hierarchy("sphere", 8) as h:
        ev, U, st = h.solve(16, 0.0, 1e-8, m=20, smoother="gs", precision="mixed", ramp_cycles=1,
                            max_cycles=1, allow_noconv=True, evecs=None)
        rows = st["ramp_evals"]
        n = np.array([h.info(l)["n_vert"] for l in range(h.n_levels)], dtype=np.float64)
    for lam, sl in MULTIPLETS:
        err = np.abs(rows[:, sl].mean(axis=1) - lam)
        r = _rates(err[2:], n[2:])
        assert np.all(r > 0.97) and np.all(r < 1.08), (lam, r)
        # level 8: the discretisation error of a 655362-vertex sphere
        assert err[-1] < 1e-3 * lam, err[-1]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shifted_one_pass_table2(lib, sphere6, precision):
    from oracle import bmg as ob
    h, lv = sphere6
    oev, oU, info = ob.solve(lv, 9, 20.0, 1e-8, m=16, smoother="gs", ramp_cycles=1, max_cycles=1)
    ev, U, st = h.solve(9, 20.0, 1e-8, m=16, smoother="gs", precision=precision, ramp_cycles=1,
                        max_cycles=1, allow_noconv=True)
    assert st["scheme"] == 2 and st["ramp_start"] == st["l_c"] == info["l_c"] == 2
    got, ref = st["ramp_evals"][2:], info["ramp_evals"][2:]
    rel = np.abs(got - ref) / np.abs(ref - 20.0)
    assert np.max(rel) < (1e-6 if precision == "fp64" else 1e-4), np.max(rel, axis=1)
    n = np.array([l.n for l in lv[2:]], dtype=np.float64)
    r = _rates(np.abs(got.mean(axis=1) - 20.0), n)
    assert np.all(r > 0.97) and np.all(r < 1.08), r


def test_ramp_then_certified_solve_c2(lib):
    # C2 (40962 vertices, 25 smallest pairs) started by the ramp: the stored
    # oracle eigenvalues, in fewer cycles on level L than from the seeded block
    gold = np.array([float(x) for x in open(os.path.join(GOLDEN, "c2_sphere_ref6_eigs.txt"))
                     if not x.startswith("#")])
    with lib.Hierarchy("sphere", 6) as h:
        ev0, U0, st0 = h.solve(25, 0.0, 1e-8, m=32, precision="mixed", smoother="jacobi")
        ev, U, st = h.solve(25, 0.0, 1e-8, m=32, precision="mixed", smoother="jacobi", ramp_cycles=1)
    assert st["converged"] == 1 and st0["converged"] == 1
    assert np.max(np.abs(ev - gold[:25]) / np.maximum(gold[:25], 1.0)) < 1e-8
    assert st["cycles"] < st0["cycles"], (st["cycles"], st0["cycles"])


def test_ramp_level_range(lib):
    with lib.Hierarchy("sphere", 3) as h:
        ev, U, st = h.solve(9, 0.0, 1e-8, m=12, ramp_cycles=1, ramp_level=3)
        assert st["converged"] == 1 and st["cycles"] == 0 and st["ramp_start"] == 3
        for bad in (dict(ramp_level=4), dict(ramp_cycles=65)):
            kw = dict(ramp_cycles=1)
            kw.update(bad)
            with pytest.raises(lib.BMGError) as e:
                h.solve(9, 0.0, 1e-8, m=12, **kw)
            assert e.value.status == lib.EINVAL
