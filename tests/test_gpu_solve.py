"""End-to-end parity of bmg_solve (HIP path through the C ABI) with the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1511_07042_amd as p
    return p


@pytest.fixture(scope="module")
def c1(lib):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 3)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 16, 0.0)
    return lib.Hierarchy("sphere", 3), lv, ref_ev, ref_U


def _check_pairs(ev, U, lv, ref_ev, ref_U, k, rel_tol=1e-8, sine_tol=1e-6):
    from oracle import reference
    M = lv[-1].M
    rel, sine = reference.compare(ev, U, ref_ev[:k], ref_U[:, :k], M, ref_ev, ref_U)
    assert rel < rel_tol, rel
    assert sine < sine_tol, sine
    G = U.T @ (M @ U)
    assert np.max(np.abs(G - np.eye(U.shape[1]))) < 1e-10
    idx = np.argmax(np.abs(U), axis=0)
    assert np.all(U[idx, np.arange(U.shape[1])] > 0)
    assert np.all(np.diff(ev) >= 0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
def test_c1_parity(lib, c1, precision, smoother):
    h, lv, ref_ev, ref_U = c1
    from oracle import bmg as ob
    ev, U, st = h.solve(9, 0.0, 1e-8, m=12, smoother=smoother, precision=precision)
    assert st["converged"] == 1
    _check_pairs(ev, U, lv, ref_ev, ref_U, 9)
    # same algorithm as the oracle: comparable cycle counts
    _, _, info = ob.solve(lv, 9, 0.0, 1e-8, m=12, smoother=smoother)
    assert abs(st["cycles"] - info["cycles"]) <= max(3, info["cycles"] // 5)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_cold_ritz_start_parity(lib, c1, precision, monkeypatch):
    # BMG_NO_WARM: every Ritz step's Jacobi starts from the identity instead of
    # the previous step's basis of the coarse block.  That basis is only a
    # change of basis of the same space, so both paths meet the oracle's pairs
    # and agree with each other up to rounding.
    h, lv, ref_ev, ref_U = c1
    monkeypatch.setenv("BMG_NO_WARM", "1")
    ev0, U0, s0 = h.solve(9, 0.0, 1e-8, m=12, smoother="jacobi", precision=precision)
    monkeypatch.delenv("BMG_NO_WARM")
    ev1, U1, s1 = h.solve(9, 0.0, 1e-8, m=12, smoother="jacobi", precision=precision)
    assert s0["converged"] == 1 and s1["converged"] == 1
    _check_pairs(ev0, U0, lv, ref_ev, ref_U, 9)
    assert abs(s0["cycles"] - s1["cycles"]) <= 1
    assert np.max(np.abs(ev0 - ev1) / np.maximum(np.abs(ev1), 1.0)) < 1e-9


def test_seeded_block_equals_initial_block(lib, c1):
    h, lv, ref_ev, ref_U = c1
    from oracle import rng
    U0 = rng.gaussian_block(lv[-1].n, 12, 7)
    ev1, V1, s1 = h.solve(9, m=12, seed=7)
    ev2, V2, s2 = h.solve(9, m=12, initial_block=U0)
    # the blocks agree to ~1 ulp (device vs NumPy log/cos), which may move the
    # stopping cycle by one; both results carry the certificate
    assert abs(s1["cycles"] - s2["cycles"]) <= 1 and s1["converged"] and s2["converged"]
    assert np.max(np.abs(ev1 - ev2) / np.maximum(np.abs(ev1), 1)) < 1e-9


def test_device_and_host_outputs_agree(lib, c1):
    import torch
    h, lv, ref_ev, ref_U = c1
    ev1, V1, _ = h.solve(9, m=12)
    ev2, V2, _ = h.solve(9, m=12, evecs="device")
    torch.cuda.synchronize()
    assert np.array_equal(ev1, ev2)
    assert np.array_equal(V1, V2.cpu().numpy())


def test_noconv_returns_current_pairs(lib, c1):
    h, lv, ref_ev, ref_U = c1
    ev, U, st = h.solve(9, m=12, max_cycles=1, allow_noconv=True)
    assert st["status"] == lib.ENOCONV and st["converged"] == 0 and st["cycles"] == 1
    assert np.all(np.isfinite(ev)) and np.all(ev >= ref_ev[:9] - 1e-9)


@pytest.mark.parametrize("kw", [dict(k=0), dict(k=9, m=10), dict(k=9, m=8), dict(k=9, tol=0.0),
                                dict(k=9, sigma=float("nan")), dict(k=9, m=400),
                                dict(k=9, m=88), dict(k=9, n_c=3)])
def test_invalid_arguments(lib, c1, kw):
    h = c1[0]
    kw = dict(kw)
    k = kw.pop("k")
    with pytest.raises(lib.BMGError) as e:
        h.solve(k, **kw)
    assert e.value.status == lib.EINVAL


def test_tiny_mesh_and_k1(lib):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 1)  # 42 vertices, two levels
    h = lib.Hierarchy("sphere", 1)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 8, 0.0)
    ev, U, st = h.solve(1, m=4)
    assert st["converged"]
    _check_pairs(ev, U, lv, ref_ev, ref_U, 1)
    ev, U, st = h.solve(4, m=8, precision="mixed")
    _check_pairs(ev, U, lv, ref_ev, ref_U, 4)


def test_widest_enrichment(lib, c1):
    # n_c + m = 96, the largest Ritz problem the one-workgroup kernel takes
    h, lv, _, _ = c1
    from oracle import reference
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 84, 0.0)
    ev, U, st = h.solve(49, m=84, precision="mixed")
    assert st["converged"]
    _check_pairs(ev, U, lv, ref_ev, ref_U, 49)


def test_small_shift_cluster(lib):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 4)
    h = lib.Hierarchy("sphere", 4)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 5, 6.0)
    for prec in ("fp64", "mixed"):
        ev, U, st = h.solve(5, 6.0, m=12, precision=prec)
        assert st["converged"]
        _check_pairs(ev, U, lv, ref_ev, ref_U, 5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_parity(lib, precision):
    from oracle import bmg as ob, reference
    lv = ob.build_levels("sphere", 6)
    h = lib.Hierarchy("sphere", 6)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 32, 0.0)
    ev, U, st = h.solve(25, 0.0, 1e-8, m=32, precision=precision)
    assert st["converged"]
    _check_pairs(ev, U, lv, ref_ev, ref_U, 25)
    print(f"C2 {precision}: cycles {st['cycles']} t {st['t_solve_ms']:.1f} ms")


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_tail_and_plain_launch_paths_identical(lib, smoother, precision, monkeypatch):
    # The cycle replayed as a HIP graph, the coarse levels fused in one
    # workgroup, the fused Jacobi cycle kernels and plain per-kernel launches
    # run the same arithmetic in the same order: results must agree bit for
    # bit, over every replay of a solve.
    h = lib.Hierarchy("sphere", 5)
    runs = {}
    for name, env in (("plain", {"BMG_NO_GRAPH": "1", "BMG_NO_TAIL": "1"}),
                      ("unfused", {"BMG_NO_GRAPH": "1", "BMG_NO_TAIL": "1", "BMG_NO_FUSE": "1"}),
                      ("tail", {"BMG_NO_GRAPH": "1"}), ("graph", {}), ("graph2", {})):
        for k in ("BMG_NO_GRAPH", "BMG_NO_TAIL", "BMG_NO_FUSE"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        runs[name] = h.solve(16, m=20, smoother=smoother, precision=precision)
    ev0, V0, s0 = runs["plain"]
    for name in ("unfused", "tail", "graph", "graph2"):
        ev, V, st = runs[name]
        assert st["cycles"] == s0["cycles"], name
        assert np.array_equal(ev, ev0), name
        assert np.array_equal(V, V0), name


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tail_column_groups_identical(lib, precision, monkeypatch):
    # With m = 32 the coarse-level tail shares the columns out over several
    # workgroups (8 in FP32, 16 in FP64) and takes level 3 as well; the cycle
    # acts on each column alone, so the result must equal the per-kernel
    # launches bit for bit.
    h = lib.Hierarchy("sphere", 5)
    runs = {}
    for name, env in (("plain", {"BMG_NO_GRAPH": "1", "BMG_NO_TAIL": "1"}),
                      ("tail", {"BMG_NO_GRAPH": "1"}), ("graph", {})):
        for k in ("BMG_NO_GRAPH", "BMG_NO_TAIL", "BMG_NO_FUSE"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        runs[name] = h.solve(25, m=32, smoother="jacobi", precision=precision)
    ev0, V0, s0 = runs["plain"]
    assert s0["converged"]
    for name in ("tail", "graph"):
        ev, V, st = runs[name]
        assert st["cycles"] == s0["cycles"], name
        assert np.array_equal(ev, ev0), name
        assert np.array_equal(V, V0), name


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_storage_order(lib, precision, monkeypatch):
    # Levels of at least BMG_ROW_ORDER_MIN_ROWS rows (and never fewer than
    # 16384) are stored with their rows in a Morton order of the vertices.
    # Every row keeps its arithmetic, so a V-cycle is the same bit for bit
    # whatever the storage; reductions over rows (Gram, residual norms) are
    # grouped differently, so a solve agrees to rounding.  The sphere refined
    # 6 times has one such level (40962 rows) with threshold 0 and none with
    # the default threshold.
    import torch
    from oracle import bmg as ob, reference
    for k in ("BMG_NO_GRAPH", "BMG_NO_TAIL", "BMG_NO_FUSE"):
        monkeypatch.delenv(k, raising=False)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((40962, 32))
    dt = torch.float32 if precision == "mixed" else torch.float64
    runs = {}
    for name, thr in (("vertex", "1000000000"), ("morton", "0")):
        monkeypatch.setenv("BMG_ROW_ORDER_MIN_ROWS", thr)
        h = lib.Hierarchy("sphere", 6)  # the threshold is read when the levels are uploaded
        cyc = {}
        for sm in ("jacobi", "gs"):
            y = torch.zeros((40962, 32), dtype=dt, device="cuda")
            h.apply("vcycle", x=torch.tensor(f, dtype=dt, device="cuda"), y=y, sigma=0.0, smoother=sm, l_c=0)
            torch.cuda.synchronize()
            cyc[sm] = y.cpu().numpy()
        runs[name] = (cyc, h.solve(25, m=32, smoother="jacobi", precision=precision))
    (c0, (ev0, V0, s0)), (c1, (ev1, V1, s1)) = runs["vertex"], runs["morton"]
    for sm in ("jacobi", "gs"):
        assert np.array_equal(c0[sm], c1[sm]), sm
    assert s0["converged"] and s1["converged"]
    assert abs(s0["cycles"] - s1["cycles"]) <= 1
    lv = ob.build_levels("sphere", 6)
    rel, sine = reference.compare(ev1, V1, ev0, V0, lv[-1].M)
    # both solves follow the same iteration up to rounding; the certificates alone
    # would allow 2e-9 and 2e-7
    assert rel < 1e-10 and sine < 2e-7, (rel, sine)


def test_discretisation_rate_against_sphere_spectrum(lib):
    # End to end against the exact spectrum of the unit sphere, l(l + 1) with
    # multiplicity 2l + 1 (Sec. 5): the discrete eigenvalues of the refined
    # icosphere approach it at the optimal rate O(h^2) = O(#DoF^-1) of the a
    # priori estimate (Lemma 2.2, eq. est-ev), i.e. r = 1 in the rate measure
    # of Sec. 5 (Table 1 reports r = 1.0037, 1.0005, 1.0059 for BMG and
    # lambda = 2, 6, 12 on the authors' meshes).  Here: the 16 lowest pairs
    # (l <= 3) of the mixed-precision solve on refinements 3..6.
    import math
    errs = {1: [], 2: [], 3: []}
    ns = []
    for nref in (3, 4, 5, 6):
        ev, U, st = lib.Hierarchy("sphere", nref).solve(16, 0.0, 1e-8, precision="mixed", smoother="jacobi")
        assert st["converged"] == 1
        ns.append(lib.finest_vertices("sphere", nref))
        assert abs(ev[0]) < 1e-8
        for l, (a, b) in ((1, (1, 4)), (2, (4, 9)), (3, (9, 16))):
            cl = ev[a:b]
            if l < 3:  # icosahedral symmetry keeps l = 1 and l = 2 exactly degenerate
                assert np.ptp(cl) < 1e-9 * l * (l + 1), (nref, l, cl)
            errs[l].append(float(np.mean(cl)) - l * (l + 1))
    for l, e in errs.items():
        assert all(x > 0 for x in e), (l, e)
        rates = [math.log(e[i] / e[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(e) - 1)]
        assert all(abs(r - 1.0) < 0.01 for r in rates), (l, rates)


def _golden_eigs(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    return np.array([float(x) for x in open(path) if x.strip() and not x.startswith("#")])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_c4_against_stored_oracle_eigenvalues(lib, precision):
    # C4: sphere refined 8 times (655362 vertices), 64 pairs, 80 test vectors.
    # The stored values come from the oracle's hierarchy and an ARPACK
    # shift-invert solve; eigenvectors are checked by their certificates,
    # M-orthonormality and the residual computed on the host.
    import scipy.sparse as sp
    ref = _golden_eigs("c4_sphere_ref8_eigs.txt")
    h = lib.Hierarchy("sphere", 8)
    ev, U, st = h.solve(64, 0.0, 1e-8, m=80, precision=precision, smoother="jacobi")
    assert st["converged"] == 1
    rel = np.abs(ev - ref[:64]) / np.maximum(np.abs(ref[:64]), 1.0)
    assert rel.max() < 1e-8, rel.max()
    L = h.n_levels - 1
    cols = h.export(L, "ell_cols")
    n, W = cols.shape
    rows = np.repeat(np.arange(n), W)
    A = sp.csr_matrix((h.export(L, "ell_a").ravel(), (rows, cols.ravel())), shape=(n, n))
    M = sp.csr_matrix((h.export(L, "ell_m").ravel(), (rows, cols.ravel())), shape=(n, n))
    MU = M @ U
    assert np.max(np.abs(U.T @ MU - np.eye(64))) < 1e-10
    D = np.asarray(M.sum(axis=1)).ravel()
    R = A @ U - MU * ev[None, :]
    rho = 2 * np.sqrt(np.sum(R * R / D[:, None], axis=0))
    assert np.allclose(rho, st["rho"], rtol=1e-6, atol=1e-12)
    print(f"C4 {precision}: cycles {st['cycles']} t {st['t_solve_ms']:.1f} ms max rel {rel.max():.1e}")


def test_custom_mesh_runtime_width_solve(lib):
    # a custom closed surface whose ELL width is 9: the whole solve on the
    # kernels' runtime-width path, against the oracle's pencil of the same mesh
    from oracle import fem, mesh, reference
    from test_gpu_kernels import _bipyramid
    xyz, tri = _bipyramid(8)
    X, T = xyz, tri
    for _ in range(4):
        X, T, _par = mesh.refine(X, T, mesh.project_sphere)
    A, M = fem.assemble(X, T)
    ref_ev, ref_U = reference.discrete_eigs(A, M, 16, 0.0)
    h = lib.Hierarchy("custom", 4, xyz=xyz, tri=tri, project=mesh.project_sphere)
    for prec, sm in (("fp64", "gs"), ("mixed", "jacobi")):
        ev, U, st = h.solve(9, m=12, precision=prec, smoother=sm)
        assert st["converged"] == 1

        class _L:
            pass
        lv = [_L()]
        lv[0].M = M
        _check_pairs(ev, U, lv, ref_ev, ref_U, 9)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_torus_64x32_coarse_grid(lib, precision):
    # The benchmark torus: R = 1, r = 0.4, a 64 x 32 parametric grid (2048
    # vertices, the level-0 eigensolve runs on the device) refined once; the
    # 32 coarse eigenvectors nearest sigma enrich the Ritz space.
    from oracle import bmg as ob, reference
    lv = ob.build_levels("torus", 1)
    ref_ev, ref_U = reference.discrete_eigs(lv[-1].A, lv[-1].M, 24, 0.0)
    h = lib.Hierarchy("torus", 1)
    lam0, phi0 = h.export(0, "coarse_eig")
    import scipy.linalg as sla
    w = sla.eigh(lv[0].A.toarray(), lv[0].M.toarray(), eigvals_only=True)
    assert np.max(np.abs(lam0 - w) / np.maximum(np.abs(w), 1.0)) < 1e-10
    assert np.max(np.abs(phi0.T @ (lv[0].M @ phi0) - np.eye(len(w)))) < 1e-10
    ev, U, st = h.solve(12, 0.0, 1e-8, m=16, precision=precision, smoother="jacobi")
    assert st["converged"] == 1 and st["n_c"] == 32
    _check_pairs(ev, U, lv, ref_ev, ref_U, 12)
