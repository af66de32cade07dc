"""Library checks that need no GPU: symbols, host-side hierarchy vs the oracle."""
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "bmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bmg_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (bmg_\w+)", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert set(lib.EXPORTED) <= set(declared)


def _ell_to_csr(cols, vals):
    n, W = cols.shape
    rows = np.repeat(np.arange(n), W)
    return sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(n, n))


@pytest.mark.parametrize("kind,nref,kw", [("sphere", 4, {}), ("ellipsoid", 3, dict(axes=(1.0, 1.5, 2.0))),
                                          ("torus", 1, dict(nu=32, nv=16))])
def test_host_hierarchy_matches_oracle(lib, kind, nref, kw):
    from oracle import mesh, fem, colour
    h = lib.Hierarchy(kind, nref, device=False, **kw)
    if kind == "torus":
        from oracle.mesh import torus_grid, refine, torus_project, Level
        xyz, tri = torus_grid(1.0, 0.4, kw["nu"], kw["nv"])
        levels = [Level(xyz, tri)]
        for _ in range(nref):
            xyz, tri, par = refine(xyz, tri, torus_project(1.0, 0.4))
            levels.append(Level(xyz, tri, par))
    else:
        levels = mesh.hierarchy(kind, nref, axes=kw.get("axes", (1.0, 1.0, 1.0)))
    for l, lv in enumerate(levels):
        assert np.array_equal(h.export(l, "tri"), lv.tri)
        assert np.allclose(h.export(l, "xyz"), lv.xyz, rtol=0, atol=1e-15)
        if l > 0:
            assert np.array_equal(h.export(l, "parents"), lv.parents)
        A, M = fem.assemble(lv.xyz, lv.tri)
        cols = h.export(l, "ell_cols")
        Ah = _ell_to_csr(cols, h.export(l, "ell_a"))
        Mh = _ell_to_csr(cols, h.export(l, "ell_m"))
        assert np.all(cols[:, 0] == np.arange(len(cols)))  # diagonal first
        assert abs(Ah - A).max() <= 1e-13 * abs(A).max()
        assert abs(Mh - M).max() <= 1e-14 * abs(M).max()  # summation order only
        assert np.array_equal(h.export(l, "colours"), colour.greedy_colouring(M))
        assert np.array_equal(h.export(l, "colours2"), colour.distance2_colouring(M))
        assert np.allclose(h.export(l, "lumped"), fem.lumped_mass(M), rtol=1e-14)
        inf = h.info(l)
        # structural nonzeros: diagonal + both directions of every edge
        assert inf["nnz"] == len(lv.xyz) + 2 * len(mesh.edges(lv.tri)) and inf["n_vert"] == len(lv.xyz)
        assert abs(inf["area"] - fem.triangle_areas(lv.xyz, lv.tri).sum()) < 1e-12 * inf["area"]
    h.close()


def test_coarse_eigendecomposition(lib):
    h = lib.Hierarchy("sphere", 0, device=False)
    lam, phi = h.export(0, "coarse_eig")
    s5 = 5 ** 0.5
    expect = [0.0] + [5 - s5] * 3 + [(15 + 3 * s5) / 2] * 5 + [10 + 4 * s5] * 3
    assert np.allclose(lam, expect, atol=1e-12)
    cols = h.export(0, "ell_cols")
    M = _ell_to_csr(cols, h.export(0, "ell_m")).toarray()
    A = _ell_to_csr(cols, h.export(0, "ell_a")).toarray()
    assert np.abs(phi.T @ M @ phi - np.eye(12)).max() < 1e-12
    assert np.abs(phi.T @ A @ phi - np.diag(lam)).max() < 1e-11


def test_custom_mesh_equals_builtin_sphere(lib):
    from oracle import mesh
    xyz, tri = mesh.icosahedron()
    proj = lambda p: p / np.linalg.norm(p)
    hc = lib.Hierarchy("custom", 2, xyz=xyz, tri=tri, project=proj, device=False)
    hs = lib.Hierarchy("sphere", 2, device=False)
    for l in range(3):
        assert np.array_equal(hc.export(l, "tri"), hs.export(l, "tri"))
        assert np.allclose(hc.export(l, "xyz"), hs.export(l, "xyz"), atol=1e-15)


def test_invalid_inputs_rejected(lib):
    from oracle import mesh
    xyz, tri = mesh.icosahedron()
    with pytest.raises(lib.BMGError) as e:
        lib.Hierarchy("custom", 1, xyz=xyz, tri=tri[:-1], device=False)  # open surface
    assert e.value.status == lib.EINVAL
    bad = tri.copy()
    bad[0] = bad[0][::-1]  # one flipped triangle: inconsistent orientation
    with pytest.raises(lib.BMGError):
        lib.Hierarchy("custom", 1, xyz=xyz, tri=bad, device=False)
    with pytest.raises(lib.BMGError):
        lib.Hierarchy("sphere", -1, device=False)
    with pytest.raises(lib.BMGError):
        lib.Hierarchy("ellipsoid", 1, axes=(1.0, -1.0, 1.0), device=False)
    with pytest.raises(lib.BMGError):
        lib.Hierarchy("torus", 1, R=0.3, r=0.4, device=False)
    h = lib.Hierarchy("sphere", 1, device=False)
    with pytest.raises(lib.BMGError):  # host-only hierarchy cannot solve
        h.solve(3)


def test_server_arguments_and_missing_device(lib):
    # argument checks come first; with no GPU visible a valid call reports
    # BMG_EDEVICE instead of queueing work that could never run
    import torch
    with pytest.raises(lib.BMGError) as e:
        lib.Server(0, 4)
    assert e.value.status == lib.EINVAL
    with pytest.raises(lib.BMGError) as e:
        lib.Server(1 << 30, 0)
    assert e.value.status == lib.EINVAL
    if not torch.cuda.is_available():
        with pytest.raises(lib.BMGError) as e:
            lib.Server(1 << 30, 4)
        assert e.value.status == lib.EDEVICE


@pytest.mark.parametrize("kind,nref,kw", [("sphere", 4, {}), ("torus", 2, dict(nu=16, nv=8)),
                                          ("ellipsoid", 3, dict(axes=(1.0, 1.5, 2.0)))])
def test_finest_vertex_formula(lib, kind, nref, kw):
    h = lib.Hierarchy(kind, nref, device=False, **kw)
    assert lib.finest_vertices(kind, nref, **{k: v for k, v in kw.items() if k in ("nu", "nv")}) == h.N


def test_apply_rejects_an_output_of_the_wrong_precision(lib):
    # the library writes y in the operator's precision without knowing its
    # size, so the binding refuses a y of the other precision before any call
    import torch

    class _H:
        n_levels = 3
    x64 = torch.zeros((8, 4), dtype=torch.float64)
    y32 = torch.zeros((8, 4), dtype=torch.float32)
    with pytest.raises(ValueError):
        lib.Hierarchy.apply(_H(), "eigres", x=x64, f=torch.zeros(4, dtype=torch.float64), y=y32)
    with pytest.raises(ValueError):
        lib.Hierarchy.apply(_H(), "eigres", x=x64, f=torch.zeros(4, dtype=torch.float64), y=x64.clone(),
                            dtype=1)
    with pytest.raises(ValueError):
        lib.Hierarchy.apply(_H(), "A", x=y32, y=x64.clone())
