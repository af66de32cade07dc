"""Pins of the discrete spectrum (paper Sec. 2.2 Lemma 2.2, Sec. 5 sphere spectrum)."""
import os

import numpy as np
import scipy.linalg as sla

from oracle import fem, mesh, reference, bmg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and l[0] != "#"]


def test_icosahedron_closed_form_eigenvalues():
    xyz, tri = mesh.icosahedron()
    A, M = fem.assemble(xyz, tri)
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    expect = []
    for row in _golden("icosahedron_eigs.txt"):
        expect += [float(row[3])] * int(row[1])
    assert np.allclose(w, sorted(expect), atol=1e-12, rtol=1e-13)


def test_sphere_spectrum_multiplicities_and_h2_rate():
    table = [(int(r[0]), float(r[1]), int(r[2]), int(r[3]), int(r[4])) for r in _golden("sphere_spectrum.txt")]
    levels = bmg.build_levels("sphere", 4)
    errs = []
    for lv in levels[1:]:
        # the lowest 40 values (every cluster the table checks, and the next one)
        w = sla.eigh(lv.A.toarray(), lv.M.toarray(), eigvals_only=True,
                     subset_by_index=[0, min(40, lv.n - 1)])
        errs.append(w[1] - 2.0)
    for l, lam, mult, j0, j1 in table[:5]:
        cl = w[j0:j1 + 1]
        assert len(cl) == mult
        assert np.all(np.abs(cl - lam) <= 0.01 * max(lam, 1) + 1e-12)  # O(h^2) at 2562 vertices
        # clusters are separated from their neighbours
        if j1 + 1 < len(w):
            assert w[j1 + 1] - cl.max() > 0.5 * (table[l + 1][1] - lam)
    # l = 1 and l = 2 stay exactly degenerate under icosahedral symmetry
    assert np.ptp(w[1:4]) < 1e-10 and np.ptp(w[4:9]) < 1e-10
    # eigenvalue error O(h^2): ratio ~4 per refinement (Lemma 2.2, eq. est-ev)
    assert all(e > 0 for e in errs)
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.7 < r < 4.3 for r in ratios[1:]), ratios


def test_reference_dense_vs_shift_invert():
    lv = bmg.build_levels("sphere", 4)[-1]
    wd, Vd = reference.discrete_eigs(lv.A, lv.M, 16, 0.0, dense_max=10 ** 9)
    ws, Vs = reference.discrete_eigs(lv.A, lv.M, 16, 0.0, dense_max=0)
    assert np.allclose(wd, ws, rtol=1e-11, atol=1e-11)
    rel, sine = reference.compare(ws, Vs, wd, Vd, lv.M)
    assert rel < 1e-11 and sine < 1e-6
