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
    # workgroup, and plain per-kernel launches run the same arithmetic in the
    # same order: results must agree bit for bit, over every replay of a solve.
    h = lib.Hierarchy("sphere", 5)
    runs = {}
    for name, env in (("plain", {"BMG_NO_GRAPH": "1", "BMG_NO_TAIL": "1"}),
                      ("tail", {"BMG_NO_GRAPH": "1"}), ("graph", {}), ("graph2", {})):
        for k in ("BMG_NO_GRAPH", "BMG_NO_TAIL"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        runs[name] = h.solve(16, m=20, smoother=smoother, precision=precision)
    ev0, V0, s0 = runs["plain"]
    for name in ("tail", "graph", "graph2"):
        ev, V, st = runs[name]
        assert st["cycles"] == s0["cycles"], name
        assert np.array_equal(ev, ev0), name
        assert np.array_equal(V, V0), name
