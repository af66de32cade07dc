"""Negative and closed-form pins of the checkers every parity test relies on
(oracle/reference.py: cluster_groups, subspace_sine, compare), of the greedy
colouring the Gauss-Seidel smoother needs (no edge inside a colour), and of
the Gaussian test vectors' distribution (Kolmogorov-Smirnov against the normal
CDF)."""
import math

import numpy as np
import pytest

from oracle import bmg, colour, reference, rng


@pytest.fixture(scope="module")
def sphere3():
    levels = bmg.build_levels("sphere", 3)
    lv = levels[-1]
    ev, U = reference.discrete_eigs(lv.A, lv.M, 16, 0.0)
    return lv, ev, U


def test_cluster_groups_closed_cases():
    assert reference.cluster_groups(np.array([1.0, 1.005, 2.0, 2.001, 3.0])) == [[0, 1], [2, 3], [4]]
    # a gap below 1e-2 max(|lambda_j|, |lambda_j-1|, 1) joins: 1.0 < 1.01 joins,
    # 1.02 > 1.0102 does not
    assert reference.cluster_groups(np.array([100.0, 101.0])) == [[0, 1]]
    assert reference.cluster_groups(np.array([100.0, 101.02])) == [[0], [1]]
    # below 1 the scale is 1: 0 and 0.009 join, 0 and 0.011 do not
    assert reference.cluster_groups(np.array([0.0, 0.009])) == [[0, 1]]
    assert reference.cluster_groups(np.array([0.0, 0.011])) == [[0], [1]]


@pytest.mark.parametrize("angle", [1e-7, 1e-3, 0.3, 1.2])
def test_subspace_sine_reports_a_known_rotation(sphere3, angle):
    lv, ev, U = sphere3
    x1, x2 = U[:, 1:2], U[:, 5:6]  # M-orthonormal, different eigenspaces
    u = math.cos(angle) * x1 + math.sin(angle) * x2
    s = reference.subspace_sine(x1, u, lv.M)
    assert abs(s - math.sin(angle)) < 1e-12 + 1e-9 * math.sin(angle)
    # two-dimensional: rotate one direction of a plane out of it
    Q = U[:, 1:3]
    V = np.hstack([U[:, 1:2], math.cos(angle) * U[:, 2:3] + math.sin(angle) * U[:, 9:10]])
    assert abs(reference.subspace_sine(Q, V, lv.M) - math.sin(angle)) < 1e-12 + 1e-9 * math.sin(angle)


def test_compare_fails_perturbed_pairs(sphere3):
    lv, ev, U = sphere3
    rel, sine = reference.compare(ev[:9], U[:, :9], ev[:9], U[:, :9], lv.M)
    assert rel == 0.0 and sine < 1e-12
    # a perturbed eigenvalue is reported with its relative error
    bad = ev[:9].copy()
    bad[4] *= 1 + 1e-6
    rel, _ = reference.compare(bad, U[:, :9], ev[:9], U[:, :9], lv.M)
    assert abs(rel - 1e-6) < 1e-12
    # a vector rotated out of its cluster is reported by its cluster's sine
    V = U[:, :9].copy()
    V[:, 6] = math.cos(1e-4) * U[:, 6] + math.sin(1e-4) * U[:, 12]
    _, sine = reference.compare(ev[:9], V, ev[:9], U[:, :9], lv.M)
    assert abs(sine - math.sin(1e-4)) < 1e-10
    # a rotation inside the l = 2 cluster (indices 4..8) is not an error
    c, s = math.cos(0.7), math.sin(0.7)
    W = U[:, :9].copy()
    W[:, 4], W[:, 5] = c * U[:, 4] + s * U[:, 5], -s * U[:, 4] + c * U[:, 5]
    _, sine = reference.compare(ev[:9], W, ev[:9], U[:, :9], lv.M)
    assert sine < 1e-12


def test_compare_cut_cluster_uses_the_full_reference_group(sphere3):
    lv, ev, U = sphere3
    # k = 6 cuts the l = 2 cluster; vectors inside the full cluster pass ...
    c, s = math.cos(0.4), math.sin(0.4)
    V = U[:, :6].copy()
    V[:, 5] = c * U[:, 5] + s * U[:, 8]
    _, sine = reference.compare(ev[:6], V, ev[:6], U[:, :6], lv.M, ev, U)
    assert sine < 1e-12
    # ... one that leaves it fails
    V[:, 5] = c * U[:, 5] + s * U[:, 12]
    _, sine = reference.compare(ev[:6], V, ev[:6], U[:, :6], lv.M, ev, U)
    assert abs(sine - s) < 1e-10


@pytest.mark.parametrize("kind,nref", [("sphere", 4), ("ellipsoid", 3), ("torus", 1)])
def test_colouring_is_proper_on_every_level(kind, nref):
    axes = (1.0, 1.5, 2.0) if kind == "ellipsoid" else (1.0, 1.0, 1.0)
    for lv in bmg.build_levels(kind, nref, axes=axes):
        # the smoothers' operator S = A - sigma M couples every mesh edge: its
        # pattern is that of M (A alone has exact zeros on the torus grid)
        col = lv.colours
        assert np.array_equal(col, colour.greedy_colouring(lv.M))
        A = (lv.A - 0.7 * lv.M).tocoo()
        off = A.row != A.col
        assert np.all(col[A.row[off]] != col[A.col[off]])
        # greedy in index order: each vertex has a lower-index neighbour of
        # every smaller colour (otherwise it would have taken that colour)
        Acsr = lv.M.tocsr()
        for i in range(0, lv.n, max(1, lv.n // 200)):
            nb = Acsr.indices[Acsr.indptr[i]:Acsr.indptr[i + 1]]
            lower = set(col[nb[nb < i]])
            assert all(c in lower for c in range(col[i]))


def test_gaussian_block_is_normal_by_kolmogorov_smirnov():
    z = np.sort(rng.gaussian_block(1000, 100, 3).ravel())
    n = z.size
    cdf = 0.5 * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in z]))
    d = max(np.max(np.arange(1, n + 1) / n - cdf), np.max(cdf - np.arange(n) / n))
    assert d < 1.63 / math.sqrt(n)  # 1% critical value
    # tails: P(|z| > 3) = 0.0027
    assert abs(np.mean(np.abs(z) > 3.0) - 0.0027) < 5 * math.sqrt(0.0027 / n)
