"""Per-kernel parity: each HIP operator (through the C ABI) against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1511_07042_amd as p
    from oracle import bmg as ob
    h = p.Hierarchy("sphere", 4)
    lv = ob.build_levels("sphere", 4)
    return torch, p, h, lv


def _dev(torch, x, dt=None):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt or torch.float64, device="cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(got, ref, scale):
    return float(np.max(np.abs(got - ref) / scale))


@pytest.mark.parametrize("m", [4, 12, 32, 80])
def test_spmm_A_M_fp64(env, m):
    torch, p, h, lv = env
    L = lv[-1]
    x = np.random.default_rng(m).standard_normal((L.n, m))
    for op, Mat in (("A", L.A), ("M", L.M)):
        y = torch.zeros((L.n, m), dtype=torch.float64, device="cuda")
        h.apply(op, x=_dev(torch, x), y=y)
        torch.cuda.synchronize()
        scale = abs(Mat) @ np.abs(x) + 1e-300
        err = _rel(_host(y), Mat @ x, scale)
        assert err < 1e-14, (op, err)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-14), ("f32", 3e-6)])
@pytest.mark.parametrize("sigma", [0.0, 7.5])
def test_shifted_and_residual(env, dtype, tol, sigma):
    torch, p, h, lv = env
    L = lv[-1]
    dt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(1)
    x, f = rng.standard_normal((L.n, 12)), rng.standard_normal((L.n, 12))
    xd, fd = _dev(torch, x, dt), _dev(torch, f, dt)
    S = (L.A - sigma * L.M).tocsr()
    scale = (abs(L.A) + sigma * abs(L.M)) @ np.abs(x) + np.abs(f)
    y = torch.zeros_like(xd)
    h.apply("shifted", x=xd, y=y, sigma=sigma)
    torch.cuda.synchronize()
    err = _rel(_host(y), S @ _host(xd), scale)
    assert err < tol, err
    h.apply("residual", x=xd, f=fd, y=y, sigma=sigma)
    torch.cuda.synchronize()
    err = _rel(_host(y), _host(fd) - S @ _host(xd), scale)
    assert err < tol, err


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
@pytest.mark.parametrize("forward", [True, False])
@pytest.mark.parametrize("level", [1, 4])
def test_smoothing_sweep(env, smoother, forward, level):
    torch, p, h, lv = env
    from oracle import bmg as ob
    L = lv[level]
    sm = ob.Smoother(L, 2.0, smoother, 2.0 / 3.0)
    rng = np.random.default_rng(level)
    e, f = rng.standard_normal((L.n, 8)), rng.standard_normal((L.n, 8))
    ref = sm.sweep(e, f, forward=forward)
    op = "smooth_fwd" if forward else "smooth_bwd"
    fd = _dev(torch, f)
    if smoother == "gs":
        y = _dev(torch, e)
        h.apply(op, f=fd, y=y, level=level, sigma=2.0, smoother="gs")
    else:
        y = torch.zeros((L.n, 8), dtype=torch.float64, device="cuda")
        h.apply(op, x=_dev(torch, e), f=fd, y=y, level=level, sigma=2.0, smoother="jacobi",
                omega=2.0 / 3.0)
    torch.cuda.synchronize()
    assert np.max(np.abs(_host(y) - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_transfers(env, dt_name):
    torch, p, h, lv = env
    dt = torch.float64 if dt_name == "f64" else torch.float32
    tol = 1e-15 if dt_name == "f64" else 1e-6
    for level in (1, 4):
        P = lv[level].P
        nf, nc = P.shape
        rng = np.random.default_rng(level)
        xf = rng.standard_normal((nf, 8))
        xc = rng.standard_normal((nc, 8))
        y = torch.zeros((nc, 8), dtype=dt, device="cuda")
        xfd = _dev(torch, xf, dt)
        h.apply("restrict", x=xfd, y=y, level=level)
        torch.cuda.synchronize()
        ref = P.T @ _host(xfd)
        assert np.max(np.abs(_host(y) - ref)) < tol * np.max(np.abs(ref)) * 8
        y0 = rng.standard_normal((nf, 8))
        yf = _dev(torch, y0, dt)
        xcd = _dev(torch, xc, dt)
        h.apply("prolong_add", x=xcd, y=yf, level=level)
        torch.cuda.synchronize()
        ref = _host(_dev(torch, y0, dt)) + P @ _host(xcd)
        assert np.max(np.abs(_host(yf) - ref)) < tol * np.max(np.abs(ref)) * 8


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
@pytest.mark.parametrize("sigma", [0.0, 6.0])
def test_vcycle(env, smoother, sigma):
    torch, p, h, lv = env
    from oracle import bmg as ob
    m = 12
    bm = ob.BMG(lv, sigma, m, 2, 2, smoother, 2.0 / 3.0)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((lv[-1].n, m))
    ref = bm.vcycle(len(lv) - 1, f)
    for dt_name, tol in (("f64", 1e-10), ("f32", 2e-4)):
        dt = torch.float64 if dt_name == "f64" else torch.float32
        y = torch.zeros((lv[-1].n, m), dtype=dt, device="cuda")
        h.apply("vcycle", x=_dev(torch, f, dt), y=y, sigma=sigma, smoother=smoother, l_c=bm.l_c,
                omega=2.0 / 3.0)
        torch.cuda.synchronize()
        err = np.max(np.abs(_host(y) - ref)) / np.max(np.abs(ref))
        assert err < tol, (dt_name, err)


def test_gaussian_block(env):
    torch, p, h, lv = env
    from oracle import rng
    for m, seed in ((12, 0), (80, 12345)):
        y = torch.zeros((lv[-1].n, m), dtype=torch.float64, device="cuda")
        h.apply("gaussian", y=y, m=m, seed=seed)
        torch.cuda.synchronize()
        ref = rng.gaussian_block(lv[-1].n, m, seed)
        assert np.max(np.abs(_host(y) - ref)) < 1e-13


@pytest.mark.parametrize("level", [0, 1, 4])
# 13 x 7 and 45 x 33: output counts that leave a ragged last block of the
# partial-sum reduction (16 outputs per block)
@pytest.mark.parametrize("wx,wf", [(1, 1), (20, 40), (44, 64), (92, 160), (96, 192), (13, 7), (45, 33)])
def test_gram_mfma(env, level, wx, wf):
    torch, p, h, lv = env
    n = lv[level].n
    rng = np.random.default_rng(wx * 1000 + wf)
    x, f = rng.standard_normal((n, wx)), rng.standard_normal((n, wf))
    y = torch.zeros((wx, wf), dtype=torch.float64, device="cuda")
    h.apply("gram", x=_dev(torch, x), f=_dev(torch, f), y=y, m=wx, m2=wf, level=level)
    torch.cuda.synchronize()
    ref = x.T @ f
    scale = np.abs(x).T @ np.abs(f)
    err = _rel(_host(y), ref, scale)
    assert err < 1e-14, err


@pytest.mark.parametrize("n", [1, 2, 7, 44, 92, 96])
def test_syev_one_workgroup(env, n):
    torch, p, h, lv = env
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    A = B + B.T
    if n >= 44:  # clustered spectrum like the Ritz problem: near-degenerate groups
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        w = np.repeat(np.arange(n // 4 + 1, dtype=float), 4)[:n] * 3.0 + 1e-9 * rng.standard_normal(n)
        A = (Q * w) @ Q.T
    out = torch.zeros(n + n * n, dtype=torch.float64, device="cuda")
    h.apply("syev", x=_dev(torch, A), y=out, m=n)
    torch.cuda.synchronize()
    o = _host(out)
    w, V = o[:n], o[n:].reshape(n, n)
    wr = np.linalg.eigvalsh(A)
    nrm = np.linalg.norm(A, 2)
    assert np.max(np.abs(w - wr)) < 1e-14 * n * nrm
    assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-13 * n
    assert np.max(np.abs(A @ V - V * w)) < 1e-14 * n * nrm


@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_eigen_residual(env, dt_name):
    torch, p, h, lv = env
    L = lv[-1]
    rng = np.random.default_rng(9)
    x = rng.standard_normal((L.n, 12))
    th = np.sort(rng.uniform(0, 30, 12))
    dt = torch.float64 if dt_name == "f64" else torch.float32
    y = torch.zeros((L.n, 12), dtype=dt, device="cuda")
    h.apply("eigres", x=_dev(torch, x), f=_dev(torch, th), y=y, dtype=0 if dt_name == "f64" else 1)
    torch.cuda.synchronize()
    ref = L.A @ x - (L.M @ x) * th[None, :]
    scale = abs(L.A) @ np.abs(x) + (abs(L.M) @ np.abs(x)) * th[None, :]
    tol = 1e-14 if dt_name == "f64" else 1e-7
    err = _rel(_host(y), ref, scale)
    assert err < tol, err


@pytest.mark.parametrize("level", [0, 2, 4])
# nz = m2 + m = 48 and 49 sit on either side of the kernel's 12 / 24 k-step
# register variants (49 also has an odd W width)
@pytest.mark.parametrize("m2,m", [(12, 12), (12, 32), (0, 8), (12, 80), (16, 80), (32, 40), (4, 92),
                                  (16, 32), (17, 32)])
def test_update_in_place(env, level, m2, m):
    # U <- [W | U] Y in place: the Ritz update of the iterate block
    torch, p, h, lv = env
    n = lv[level].n
    rng = np.random.default_rng(100 * m2 + m + level)
    W, U, Y = rng.standard_normal((n, m2)), rng.standard_normal((n, m)), rng.standard_normal((m2 + m, m))
    Ud = _dev(torch, U)
    h.apply("update", x=_dev(torch, W) if m2 else None, f=_dev(torch, Y), y=Ud, m=m, m2=m2,
            level=level)
    torch.cuda.synchronize()
    Z = np.hstack([W, U])
    err = _rel(_host(Ud), Z @ Y, np.abs(Z) @ np.abs(Y))
    assert err < 1e-14, err


def _bipyramid(k=8):
    # closed surface with two vertices of valence k (ELL width k + 1 != 7):
    # exercises the kernels' runtime-width path
    ang = 2 * np.pi * np.arange(k) / k
    xyz = np.vstack([[0, 0, 1.0], [0, 0, -1.0], np.c_[np.cos(ang), np.sin(ang), np.zeros(k)]])
    tri = []
    for i in range(k):
        a, b = 2 + i, 2 + (i + 1) % k
        for t in ((0, a, b), (1, b, a)):
            p0, p1, p2 = xyz[list(t)]
            if np.dot(np.cross(p1 - p0, p2 - p0), p0 + p1 + p2) < 0:
                t = (t[0], t[2], t[1])
            tri.append(t)
    return xyz, np.array(tri, dtype=np.int32)


def test_runtime_width_kernels(env):
    torch, p, _, _ = env
    from oracle import fem, mesh
    xyz, tri = _bipyramid(8)
    h = p.Hierarchy("custom", 3, xyz=xyz, tri=tri, project=mesh.project_sphere)
    L = h.n_levels - 1
    assert h.info(L)["ell_width"] == 9
    X, T = xyz, tri
    for _ in range(3):
        X, T, _par = mesh.refine(X, T, mesh.project_sphere)
    A, M = fem.assemble(X, T)
    n, m = A.shape[0], 12
    rng = np.random.default_rng(3)
    x, f = rng.standard_normal((n, m)), rng.standard_normal((n, m))
    for op, Mat in (("A", A), ("M", M)):
        y = torch.zeros((n, m), dtype=torch.float64, device="cuda")
        h.apply(op, x=_dev(torch, x), y=y)
        torch.cuda.synchronize()
        assert _rel(_host(y), Mat @ x, abs(Mat) @ np.abs(x) + 1e-300) < 1e-14, op
    sigma = 3.0
    S = (A - sigma * M).tocsr()
    scale = (abs(A) + sigma * abs(M)) @ np.abs(x) + np.abs(f)
    y = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    h.apply("residual", x=_dev(torch, x), f=_dev(torch, f), y=y, sigma=sigma)
    torch.cuda.synchronize()
    assert _rel(_host(y), f - S @ x, scale) < 1e-14
    d = S.diagonal()
    h.apply("smooth_fwd", x=_dev(torch, x), f=_dev(torch, f), y=y, sigma=sigma, smoother="jacobi",
            omega=2.0 / 3.0)
    torch.cuda.synchronize()
    ref = x + (2.0 / 3.0) * (f - S @ x) / d[:, None]
    assert _rel(_host(y), ref, np.abs(x) + scale / np.abs(d)[:, None]) < 1e-13
    th = np.sort(rng.uniform(0, 30, m))
    h.apply("eigres", x=_dev(torch, x), f=_dev(torch, th), y=y)
    torch.cuda.synchronize()
    ref = A @ x - (M @ x) * th[None, :]
    assert _rel(_host(y), ref, abs(A) @ np.abs(x) + (abs(M) @ np.abs(x)) * th[None, :]) < 1e-14


@pytest.mark.parametrize("level", [1, 4])
@pytest.mark.parametrize("m2,m", [(0, 8), (12, 32), (12, 80), (32, 40), (4, 92), (5, 6)])
def test_gram_fused_products(env, level, m2, m):
    # [W | U]^T [A U | M U] with A U and M U formed inside the Gram kernel
    torch, p, h, lv = env
    L = lv[level]
    rng = np.random.default_rng(7 * m + m2 + level)
    W, U = rng.standard_normal((L.n, m2)), rng.standard_normal((L.n, m))
    y = torch.zeros((m2 + m, 2 * m), dtype=torch.float64, device="cuda")
    h.apply("gram_am", x=_dev(torch, W) if m2 else None, f=_dev(torch, U), y=y, m=m, m2=m2,
            level=level)
    torch.cuda.synchronize()
    Z = np.hstack([W, U])
    Y = np.hstack([L.A @ U, L.M @ U])
    scale = np.abs(Z).T @ np.hstack([abs(L.A) @ np.abs(U), abs(L.M) @ np.abs(U)])
    err = _rel(_host(y), Z.T @ Y, scale)
    assert err < 1e-14, err
    # the symmetric blocks U^T A U and U^T M U come out exactly symmetric
    g = _host(y)[m2:]
    assert np.array_equal(g[:, :m], g[:, :m].T) and np.array_equal(g[:, m:], g[:, m:].T)


def test_gram_fused_runtime_width(env):
    torch, p, _, _ = env
    from oracle import fem, mesh
    xyz, tri = _bipyramid(8)
    h = p.Hierarchy("custom", 3, xyz=xyz, tri=tri, project=mesh.project_sphere)
    X, T = xyz, tri
    for _ in range(3):
        X, T, _par = mesh.refine(X, T, mesh.project_sphere)
    A, M = fem.assemble(X, T)
    rng = np.random.default_rng(5)
    W, U = rng.standard_normal((A.shape[0], 10)), rng.standard_normal((A.shape[0], 12))
    y = torch.zeros((22, 24), dtype=torch.float64, device="cuda")
    h.apply("gram_am", x=_dev(torch, W), f=_dev(torch, U), y=y, m=12, m2=10)
    torch.cuda.synchronize()
    Z = np.hstack([W, U])
    scale = np.abs(Z).T @ np.hstack([abs(A) @ np.abs(U), abs(M) @ np.abs(U)])
    assert _rel(_host(y), Z.T @ np.hstack([A @ U, M @ U]), scale) < 1e-14
