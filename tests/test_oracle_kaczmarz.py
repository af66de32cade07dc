"""Pins of the oracle's Kaczmarz smoother (Sec. 5.3) and its distance-2 colouring.

- The colouring: no two vertices within two edges share a colour (checked by
  brute force over every path of length 1 and 2), and it is the greedy one
  (every vertex sees each smaller colour among its lower-index distance-2
  neighbours).
- A multicolour sweep equals the textbook Kaczmarz method run one equation at
  a time in the same order (colour by colour, ascending rows inside a colour),
  written here as a plain loop over rows.
- Kaczmarz never increases the Euclidean distance to the solution of a
  consistent system, for any nonsingular S, the indefinite shifted operators
  included (where the Gauss-Seidel sweep of the same system diverges).
- Solves with it reach ARPACK's pairs (fixed and interior shift), and the
  one-pass ramp with it converges at r = 1 on the l = 4 multiplet
  (Table 2's setting, lambda = 20).
"""
import numpy as np
import pytest

from oracle import bmg, colour, reference


def _graph(A):
    A = A.tocsr()
    return [set(A.indices[A.indptr[i]:A.indptr[i + 1]]) - {i} for i in range(A.shape[0])]


@pytest.mark.parametrize("kind,nref", [("sphere", 3), ("torus", 0)])
def test_distance2_colouring_is_proper_and_greedy(kind, nref):
    lv = bmg.build_levels(kind, nref)[-1]
    c = colour.distance2_colouring(lv.M)
    nb = _graph(lv.A - 0.7 * lv.M)  # the pattern of the shifted operator
    for i in range(lv.n):
        d2 = set(nb[i])
        for j in nb[i]:
            d2 |= nb[j]
        d2.discard(i)
        assert all(c[j] != c[i] for j in d2), i
        lower = {int(c[j]) for j in d2 if j < i}
        assert set(range(int(c[i]))) <= lower, i  # greedy: the smallest free colour
    assert c.max() + 1 <= 20


def _sequential_kaczmarz(S, rows_in_order, x, f):
    S = S.tocsr()
    x = x.copy()
    for i in rows_in_order:
        cols = S.indices[S.indptr[i]:S.indptr[i + 1]]
        vals = S.data[S.indptr[i]:S.indptr[i + 1]]
        r = f[i] - vals @ x[cols]
        x[cols] += np.outer(vals, r / (vals @ vals))
    return x


@pytest.mark.parametrize("sigma", [0.0, 20.0])
def test_multicolour_sweep_equals_row_by_row_kaczmarz(sigma):
    lv = bmg.build_levels("sphere", 2)[-1]
    sm = bmg.Smoother(lv, sigma, "kaczmarz", 1.0)
    rng = np.random.default_rng(3)
    x, f = rng.standard_normal((lv.n, 5)), rng.standard_normal((lv.n, 5))
    c = lv.colours2
    up = list(range(int(c.max()) + 1))
    for forward in (True, False):
        # colours up (forward) or down (backward), rows ascending inside a colour
        order = [i for k in (up if forward else up[::-1]) for i in np.flatnonzero(c == k)]
        ref = _sequential_kaczmarz(sm.S, order, x, f)
        got = sm.sweep(x, f, forward=forward)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_kaczmarz_does_not_move_away_from_the_solution_of_an_indefinite_system():
    lv = bmg.build_levels("sphere", 3)[-1]
    sigma = 60.0  # about 60 eigenvalues of the level lie below: S is indefinite
    S = (lv.A - sigma * lv.M).tocsr()
    w = np.linalg.eigvalsh(S.toarray())
    assert w.min() < 0 < w.max()
    rng = np.random.default_rng(1)
    xs = rng.standard_normal((lv.n, 3))
    f = S @ xs
    kz = bmg.Smoother(lv, sigma, "kaczmarz", 1.0)
    x = np.zeros_like(xs)
    err = [np.linalg.norm(x - xs)]
    for k in range(30):
        x = kz.sweep(x, f, forward=k % 2 == 0)
        err.append(np.linalg.norm(x - xs))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(err, err[1:]))
    assert err[-1] < err[0]
    # Gauss-Seidel on the same system grows without bound
    gs = bmg.Smoother(lv, sigma, "gs", 1.0)
    x = np.zeros_like(xs)
    for k in range(30):
        x = gs.sweep(x, f, forward=k % 2 == 0)
    assert np.linalg.norm(x - xs) > 1e3 * err[0]


@pytest.mark.parametrize("kind,nref,sigma,k,m,axes", [
    ("sphere", 4, 0.0, 9, 12, (1.0, 1.0, 1.0)),
    ("ellipsoid", 5, 40.0, 16, 24, (1.0, 1.5, 2.0)),
])
def test_solves_with_kaczmarz_match_arpack(kind, nref, sigma, k, m, axes):
    levels = bmg.build_levels(kind, nref, axes=axes)
    L = levels[-1]
    ev, U, info = bmg.solve(levels, k, sigma, 1e-8, m=m, smoother="kaczmarz", nu1=5, nu2=5)
    assert info["converged"]
    ref_ev, ref_U = reference.discrete_eigs(L.A, L.M, k + 8, sigma)
    idx = np.sort(np.argsort(np.abs(ref_ev - sigma), kind="stable")[:k])
    rel, sine = reference.compare(ev, U, ref_ev[idx], ref_U[:, idx], L.M, ref_ev, ref_U)
    assert rel < 1e-9 and sine < 1e-6


def test_one_pass_rate_with_kaczmarz_table2():
    # lambda = 20 with the interior shift, five Kaczmarz sweeps before and
    # after the coarse correction on every level, one cycle per level
    lv = bmg.build_levels("sphere", 6)
    n = np.array([l.n for l in lv], dtype=np.float64)
    ev, U, info = bmg.solve(lv, 9, 20.0, 1e-8, m=16, smoother="kaczmarz", nu1=5, nu2=5,
                            ramp_cycles=1, max_cycles=1)
    rows = info["ramp_evals"][2:]
    err = np.abs(rows.mean(axis=1) - 20.0)
    r = np.log(err[:-1] / err[1:]) / np.log(n[3:] / n[2:-1])
    assert np.all(r > 0.95) and np.all(r < 1.08), r
