"""ctypes binding of libbmg (include/bmg.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts Python
arguments to the C structures and back.  torch is used for device memory
(torch.cuda tensors) and for the current HIP stream.  If the library is not
built, importing the package raises; nothing falls back to a CPU path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBUSY, ECANCELED = 0, -1, -2, -3, -4, -5, -6
KINDS = {"sphere": 0, "ellipsoid": 1, "torus": 2, "custom": 3}
SMOOTHERS = {"gs": 0, "jacobi": 1, "kaczmarz": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
SCHEMES = {"auto": 0, "enriched": 1, "shifted": 2}
EXPORTS = {"xyz": 0, "tri": 1, "parents": 2, "ell_cols": 3, "ell_a": 4, "ell_m": 5, "colours": 6,
           "lumped": 7, "coarse_eig": 8, "colours2": 9}
KERNEL_CLASSES = {"eigres": 0, "spmm_am": 1, "smooth": 2, "residual": 3, "restrict": 4,
                  "prolong": 5, "gram": 6, "update": 7, "ritz": 8, "smooth_pair": 9,
                  "restrict_res": 10, "prolong_smooth": 11, "smooth_add": 12}
# operators whose output y is in the operator's precision (dtype 0: FP64, 1: FP32)
T_OUT_OPS = {"A", "M", "shifted", "residual", "smooth_fwd", "smooth_bwd", "restrict", "prolong_add",
             "vcycle", "eigres", "coarse_solve"}
OPS = {"A": 0, "M": 1, "shifted": 2, "residual": 3, "smooth_fwd": 4, "smooth_bwd": 5,
       "restrict": 6, "prolong_add": 7, "vcycle": 8, "gaussian": 9, "gram": 10, "syev": 11,
       "eigres": 12, "update": 13, "gram_am": 14, "coarse_solve": 15, "shift_offsets": 16}

PROJECT_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_void_p)


class SurfaceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axes", C.c_double * 3), ("R", C.c_double), ("r", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32), ("n_vert", C.c_int32), ("n_tri", C.c_int32),
                ("xyz", C.POINTER(C.c_double)), ("tri", C.POINTER(C.c_int32)),
                ("project", PROJECT_FN), ("ctx", C.c_void_p)]


class LevelInfo(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level", C.c_int32), ("n_vert", C.c_int64),
                ("n_tri", C.c_int64), ("nnz", C.c_int64), ("ell_width", C.c_int32),
                ("n_colours", C.c_int32), ("area", C.c_double), ("device_bytes", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32), ("smoother", C.c_int32),
                ("precision", C.c_int32), ("max_cycles", C.c_int32), ("n_c", C.c_int32),
                ("l_c", C.c_int32), ("omega", C.c_double), ("angle_tol", C.c_double),
                ("seed", C.c_uint64), ("initial_block", C.POINTER(C.c_double)),
                ("timed_kernel", C.c_int32), ("scheme", C.c_int32), ("ramp_cycles", C.c_int32),
                ("ramp_level", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("converged", C.c_int32), ("m", C.c_int32),
                ("n_c", C.c_int32), ("l_c", C.c_int32), ("group_size", C.c_int32),
                ("t_solve_ms", C.c_double), ("max_rho_over_delta", C.c_double),
                ("max_kato_temple", C.c_double), ("rho", C.POINTER(C.c_double)),
                ("delta", C.POINTER(C.c_double)), ("timed_kernel_ms", C.c_double),
                ("timed_kernel_bytes", C.c_double), ("timed_kernel_units", C.c_int64),
                ("ritz_sweeps_max", C.c_int32), ("ritz_fallbacks", C.c_int32),
                ("scheme", C.c_int32), ("reserved2", C.c_int32), ("coarse_eig_ms", C.c_double),
                ("lc_shift", C.c_double), ("ramp_evals", C.POINTER(C.c_double)),
                ("ramp_start", C.c_int32), ("reserved3", C.c_int32)]


class GroupRequest(C.Structure):
    _fields_ = [("k", C.c_int32), ("tol", C.c_double), ("opts", C.POINTER(SolveOpts)),
                ("evals", C.POINTER(C.c_double)), ("evecs", C.c_void_p), ("ld", C.c_int64),
                ("evecs_on_device", C.c_int32), ("status", C.c_int32), ("stats", C.POINTER(SolveStats))]


class ApplyArgs(C.Structure):
    _fields_ = [("level", C.c_int32), ("op", C.c_int32), ("dtype", C.c_int32), ("m", C.c_int32),
                ("m2", C.c_int32), ("smoother", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("l_c", C.c_int32), ("reserved", C.c_int32), ("sigma", C.c_double),
                ("omega", C.c_double), ("seed", C.c_uint64)]


_H = C.c_void_p
_sig = {
    "bmg_build_hierarchy": (C.c_int, [C.POINTER(SurfaceDesc), C.c_int32, C.c_void_p, C.POINTER(_H)]),
    "bmg_build_hierarchy_host": (C.c_int, [C.POINTER(SurfaceDesc), C.c_int32, C.POINTER(_H)]),
    "bmg_free_hierarchy": (None, [_H]),
    "bmg_hierarchy_info": (C.c_int, [_H, C.c_int32, C.POINTER(LevelInfo)]),
    "bmg_hierarchy_export": (C.c_int, [_H, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_int64)]),
    "bmg_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
    "bmg_solve": (C.c_int, [_H, C.c_int32, C.c_double, C.c_double, C.POINTER(SolveOpts),
                            C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                            C.POINTER(SolveStats)]),
    "bmg_solve_group": (C.c_int, [_H, C.c_double, C.c_int32, C.POINTER(GroupRequest), C.c_void_p]),
    "bmg_apply": (C.c_int, [_H, C.POINTER(ApplyArgs), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bmg_estimate": (C.c_int, [_H, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_void_p, C.c_int64,
                               C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "bmg_two_grid": (C.c_int, [_H, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                               C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "bmg_gram_am_noalloc": (C.c_int, [_H, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.c_void_p]),
    "bmg_server_create": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]),
    "bmg_server_submit": (C.c_int, [C.c_void_p, C.POINTER(SurfaceDesc), C.c_int32, C.c_int32,
                                    C.c_double, C.c_double, C.POINTER(SolveOpts),
                                    C.POINTER(C.c_uint64)]),
    "bmg_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.c_int64, C.POINTER(SolveStats), C.POINTER(C.c_double)]),
    "bmg_server_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "bmg_server_destroy": (None, [C.c_void_p]),
    "bmg_status_string": (C.c_char_p, [C.c_int]),
    "bmg_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


class BMGError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.bmg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.bmg_status_string(status).decode()} ({status}): {msg}")


def _check(st, where, allow=()):
    if st != OK and st not in allow:
        raise BMGError(st, where)
    return st


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def surface_desc(kind="sphere", axes=(1.0, 1.0, 1.0), R=1.0, r=0.4, nu=64, nv=32, xyz=None, tri=None,
                 project=None):
    """Build a SurfaceDesc; returns (desc, keepalive) (keep both alive during the call)."""
    d = SurfaceDesc()
    d.kind = KINDS[kind]
    d.axes = (C.c_double * 3)(*[float(a) for a in axes])
    d.R, d.r, d.nu, d.nv = float(R), float(r), int(nu), int(nv)
    keep = []
    if kind == "custom":
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        keep += [xyz, tri]
        d.n_vert, d.n_tri = len(xyz), len(tri)
        d.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
        d.tri = tri.ctypes.data_as(C.POINTER(C.c_int32))
        if project is not None:
            def _cb(p, ctx):
                arr = np.ctypeslib.as_array(p, shape=(3,))
                arr[:] = project(arr.copy())
            cb = PROJECT_FN(_cb)
            keep.append(cb)
            d.project = cb
    return d, keep


class Hierarchy:
    """A device-resident (or host-only) BMG hierarchy of one surface."""

    def __init__(self, kind="sphere", n_refine=3, axes=(1.0, 1.0, 1.0), R=1.0, r=0.4, nu=64, nv=32,
                 xyz=None, tri=None, project=None, device=True, stream=None):
        d, keep = surface_desc(kind, axes, R, r, nu, nv, xyz, tri, project)
        h = _H()
        if device:
            st = _lib.bmg_build_hierarchy(C.byref(d), int(n_refine), _stream_ptr(stream), C.byref(h))
        else:
            st = _lib.bmg_build_hierarchy_host(C.byref(d), int(n_refine), C.byref(h))
        _check(st, "bmg_build_hierarchy")
        self._h = h
        self.device = device
        self.n_levels = self.info(0)["n_levels"]
        self.N = self.info(self.n_levels - 1)["n_vert"]

    def close(self):
        if getattr(self, "_h", None):
            _lib.bmg_free_hierarchy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self, level):
        out = LevelInfo()
        _check(_lib.bmg_hierarchy_info(self._h, int(level), C.byref(out)), "bmg_hierarchy_info")
        return {f: getattr(out, f) for f, _ in LevelInfo._fields_}

    def export(self, level, what):
        need = C.c_int64(0)
        _lib.bmg_hierarchy_export(self._h, int(level), EXPORTS[what], None, 0, C.byref(need))
        inf = self.info(level)
        n, W = inf["n_vert"], inf["ell_width"]
        if what in ("xyz",):
            arr = np.empty((n, 3), np.float64)
        elif what == "tri":
            arr = np.empty((inf["n_tri"], 3), np.int32)
        elif what == "parents":
            arr = np.empty((need.value // 8, 2), np.int32)
        elif what == "ell_cols":
            arr = np.empty((n, W), np.int32)
        elif what in ("ell_a", "ell_m"):
            arr = np.empty((n, W), np.float64)
        elif what in ("colours", "colours2"):
            arr = np.empty(n, np.int32)
        elif what == "lumped":
            arr = np.empty(n, np.float64)
        elif what == "coarse_eig":
            arr = np.empty(need.value // 8, np.float64)
        else:
            raise KeyError(what)
        _check(_lib.bmg_hierarchy_export(self._h, int(level), EXPORTS[what], arr.ctypes.data,
                                         arr.nbytes, C.byref(need)), "bmg_hierarchy_export")
        if what == "coarse_eig":
            n0 = n
            return arr[:n0], arr[n0:].reshape(n0, n0)
        return arr

    def solve(self, k, sigma=0.0, tol=1e-8, m=0, nu1=2, nu2=2, smoother="gs", precision="fp64",
              max_cycles=200, n_c=0, l_c=-1, omega=0.85, angle_tol=1e-7, seed=0,
              initial_block=None, evecs="host", stream=None, allow_noconv=False, timed_kernel=None,
              scheme="auto", ramp_cycles=0, ramp_level=-1):
        """Returns (evals [k], evecs [N, k] or None, stats dict).

        evecs: "host" -> numpy array, "device" -> torch.cuda tensor view, None.
        """
        o = SolveOpts()
        _lib.bmg_solve_opts_default(C.byref(o))
        o.m, o.nu1, o.nu2 = int(m), int(nu1), int(nu2)
        o.smoother = SMOOTHERS[smoother]
        o.precision = PRECISIONS[precision]
        o.max_cycles, o.n_c, o.l_c = int(max_cycles), int(n_c), int(l_c)
        o.omega, o.angle_tol, o.seed = float(omega), float(angle_tol), int(seed)
        if timed_kernel is None:
            o.timed_kernel = -1
        elif isinstance(timed_kernel, tuple):  # (class, level): that level's launches only
            o.timed_kernel = KERNEL_CLASSES[timed_kernel[0]] + 256 * (int(timed_kernel[1]) + 1)
        else:
            o.timed_kernel = KERNEL_CLASSES[timed_kernel]
        o.scheme = SCHEMES[scheme]
        o.ramp_cycles, o.ramp_level = int(ramp_cycles), int(ramp_level)
        keep = None
        if initial_block is not None:
            keep = np.ascontiguousarray(initial_block, dtype=np.float64)
            o.initial_block = keep.ctypes.data_as(C.POINTER(C.c_double))
        evals = np.zeros(k, np.float64)
        rho = np.zeros(k, np.float64)
        delta = np.zeros(k, np.float64)
        st = SolveStats()
        st.rho = rho.ctypes.data_as(C.POINTER(C.c_double))
        st.delta = delta.ctypes.data_as(C.POINTER(C.c_double))
        ramp = np.full((self.n_levels, k), np.nan)
        st.ramp_evals = ramp.ctypes.data_as(C.POINTER(C.c_double))
        out = None
        ptr, on_dev = None, 0
        if evecs == "host":
            out = np.zeros((k, self.N), np.float64)
            ptr = out.ctypes.data
        elif evecs == "device":
            import torch
            out = torch.empty((k, self.N), dtype=torch.float64, device="cuda")
            ptr, on_dev = out.data_ptr(), 1
        status = _lib.bmg_solve(self._h, int(k), float(sigma), float(tol), C.byref(o),
                                evals.ctypes.data_as(C.POINTER(C.c_double)), ptr, int(self.N),
                                on_dev, _stream_ptr(stream) if self.device else None, C.byref(st))
        _check(status, "bmg_solve", allow=(ENOCONV,) if allow_noconv else ())
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_
                 if f not in ("rho", "delta", "ramp_evals")}
        stats.update(rho=rho, delta=delta, status=status, ramp_evals=ramp)
        V = None if out is None else out.T
        return evals, V, stats

    def solve_group(self, requests, sigma=0.0, nu1=2, nu2=2, smoother="jacobi", precision="mixed",
                    n_c=0, l_c=-1, omega=0.85, evecs="host", stream=None, allow_noconv=False,
                    scheme="auto"):
        """bmg_solve_group: requests is a list of dicts with k and optionally m,
        seed, tol (1e-8), max_cycles (200), angle_tol (1e-7).  Returns a list of
        (evals [k], evecs [N, k] or None, stats dict), one per request."""
        n = len(requests)
        arr = (GroupRequest * n)()
        keep = []
        for i, q in enumerate(requests):
            o = SolveOpts()
            _lib.bmg_solve_opts_default(C.byref(o))
            o.m, o.nu1, o.nu2 = int(q.get("m", 0)), int(nu1), int(nu2)
            o.smoother, o.precision = SMOOTHERS[smoother], PRECISIONS[precision]
            o.max_cycles, o.n_c, o.l_c = int(q.get("max_cycles", 200)), int(n_c), int(l_c)
            o.omega, o.angle_tol, o.seed = float(omega), float(q.get("angle_tol", 1e-7)), int(q.get("seed", 0))
            o.timed_kernel = -1
            o.scheme = SCHEMES[scheme]
            k = int(q["k"])
            ev = np.zeros(k, np.float64)
            rho, delta = np.zeros(k, np.float64), np.zeros(k, np.float64)
            st = SolveStats()
            st.rho = rho.ctypes.data_as(C.POINTER(C.c_double))
            st.delta = delta.ctypes.data_as(C.POINTER(C.c_double))
            out, ptr, on_dev = None, None, 0
            if evecs == "host":
                out = np.zeros((k, self.N), np.float64)
                ptr = out.ctypes.data
            elif evecs == "device":
                import torch
                out = torch.empty((k, self.N), dtype=torch.float64, device="cuda")
                ptr, on_dev = out.data_ptr(), 1
            keep.append((o, ev, rho, delta, st, out))
            arr[i].k, arr[i].tol = k, float(q.get("tol", 1e-8))
            arr[i].opts = C.pointer(o)
            arr[i].evals = ev.ctypes.data_as(C.POINTER(C.c_double))
            arr[i].evecs, arr[i].ld, arr[i].evecs_on_device = ptr, int(self.N), on_dev
            arr[i].stats = C.pointer(st)
        status = _lib.bmg_solve_group(self._h, float(sigma), n, arr, _stream_ptr(stream))
        _check(status, "bmg_solve_group", allow=(ENOCONV,) if allow_noconv else ())
        res = []
        for i, (o, ev, rho, delta, st, out) in enumerate(keep):
            stats = {f: getattr(st, f) for f, _ in SolveStats._fields_ if f not in ("rho", "delta", "ramp_evals")}
            stats.update(rho=rho, delta=delta, status=arr[i].status)
            res.append((ev, None if out is None else out.T, stats))
        return res

    def estimate(self, evals, evecs, level=None, per_triangle=False, stream=None):
        """bmg_estimate on a torch.cuda FP64 tensor evecs [N, k] (columns
        contiguous, as solve(evecs="device") returns).  Returns (eta [k],
        parts [3, k], eta2_T [F] torch tensor or None)."""
        import torch
        lvl = self.n_levels - 1 if level is None else int(level)
        evals = np.ascontiguousarray(evals, dtype=np.float64)
        k = len(evals)
        V = evecs.T
        assert V.is_cuda and V.dtype == torch.float64 and V.is_contiguous(), \
            "evecs must be an [N, k] view of a contiguous [k, N] FP64 CUDA tensor"
        ld = V.shape[1]
        eta = np.zeros(k)
        parts = np.zeros((3, k))
        e2 = None
        if per_triangle:
            e2 = torch.zeros(self.info(lvl)["n_tri"], dtype=torch.float64, device=V.device)
        _check(_lib.bmg_estimate(self._h, lvl, k, evals.ctypes.data_as(C.POINTER(C.c_double)),
                                 C.c_void_p(V.data_ptr()), int(ld), eta.ctypes.data_as(C.POINTER(C.c_double)),
                                 parts.ctypes.data_as(C.POINTER(C.c_double)),
                                 None if e2 is None else C.c_void_p(e2.data_ptr()), _stream_ptr(stream)),
               "bmg_estimate")
        return eta, parts, e2

    def two_grid(self, level_H, idx, top=-1, nu=5, evecs=True, stream=None):
        """Cascade of the two-grid Alg. 1 from level_H (see bmg_two_grid).

        Returns (rows [n_levels, n] with NaN outside level_H..top, vectors
        [N_top, n] or None)."""
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        n = len(idx)
        rows = np.full((self.n_levels, n), np.nan)
        top_l = self.n_levels - 1 if top < 0 else int(top)
        V = np.zeros((n, self.info(top_l)["n_vert"])) if evecs else None
        _check(_lib.bmg_two_grid(self._h, int(level_H), n, idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                 int(top), int(nu), rows.ctypes.data_as(C.POINTER(C.c_double)),
                                 None if V is None else V.ctypes.data, _stream_ptr(stream)),
               "bmg_two_grid")
        return rows, (None if V is None else V.T)

    def apply(self, op, x=None, f=None, y=None, level=None, m=None, m2=0, dtype=None, sigma=0.0,
              smoother="gs", nu1=2, nu2=2, l_c=-1, omega=0.85, seed=0, stream=None):
        """Enqueue one operator on torch.cuda tensors (see bmg_op in include/bmg.h)."""
        import torch
        a = ApplyArgs()
        a.level = self.n_levels - 1 if level is None else int(level)
        a.op = OPS[op]
        ref = x if x is not None else y
        if dtype is None:
            if op in T_OUT_OPS and x is not None and y is not None and x.dtype != y.dtype:
                raise ValueError(f"{op}: x is {x.dtype} and y is {y.dtype}; pass dtype explicitly")
            dtype = 1 if ref.dtype == torch.float32 else 0
        if op in T_OUT_OPS and y is not None and y.dtype != (torch.float32 if dtype else torch.float64):
            # the library writes y in the operator's precision and cannot see its size
            raise ValueError(f"{op}: y is {y.dtype} but the operator writes "
                             f"{'float32' if dtype else 'float64'}")
        a.dtype = int(dtype)
        a.m = int(m if m is not None else ref.shape[-1])
        a.m2 = int(m2)
        a.smoother = SMOOTHERS[smoother]
        a.nu1, a.nu2, a.l_c = int(nu1), int(nu2), int(l_c)
        a.sigma, a.omega, a.seed = float(sigma), float(omega), int(seed)
        for t in (x, f, y):
            if t is not None:
                assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
        p = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        _check(_lib.bmg_apply(self._h, C.byref(a), p(x), p(f), p(y), _stream_ptr(stream)), f"bmg_apply({op})")
        return y


def gram_am_noalloc(h, u, G, w=None, level=None, stream=None):
    """bmg_gram_am_noalloc on torch.cuda FP64 tensors: G = [w | u]^T [A u | M u]."""
    lvl = h.n_levels - 1 if level is None else int(level)
    m = int(u.shape[-1])
    m2 = 0 if w is None else int(w.shape[-1])
    for t in (u, G, w):
        if t is not None:
            assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    _check(_lib.bmg_gram_am_noalloc(h._h, lvl, None if w is None else C.c_void_p(w.data_ptr()), m2,
                                    C.c_void_p(u.data_ptr()), m, C.c_void_p(G.data_ptr()),
                                    _stream_ptr(stream)), "bmg_gram_am_noalloc")
    return G


def finest_vertices(kind="sphere", n_refine=0, nu=64, nv=32, n_vert=0, n_tri=0):
    """Vertices of the finest level of a uniformly refined hierarchy (each edge
    gains a midpoint, each triangle splits into four)."""
    if kind in ("sphere", "ellipsoid"):
        n, e, f = 12, 30, 20
    elif kind == "torus":
        n = nu * nv
        e, f = 3 * n, 2 * n
    else:
        n, f = n_vert, n_tri
        e = 3 * n_tri // 2
    for _ in range(int(n_refine)):
        n, e, f = n + e, 2 * e + 3 * f, 4 * f
    return n


def _opts(m=0, nu1=2, nu2=2, smoother="jacobi", precision="mixed", max_cycles=200, n_c=0, l_c=-1,
          omega=0.85, angle_tol=1e-7, seed=0, scheme="auto"):
    o = SolveOpts()
    _lib.bmg_solve_opts_default(C.byref(o))
    o.m, o.nu1, o.nu2 = int(m), int(nu1), int(nu2)
    o.smoother = SMOOTHERS[smoother]
    o.precision = PRECISIONS[precision]
    o.max_cycles, o.n_c, o.l_c = int(max_cycles), int(n_c), int(l_c)
    o.omega, o.angle_tol, o.seed = float(omega), float(angle_tol), int(seed)
    o.scheme = SCHEMES[scheme]
    return o


class Server:
    """Continuous-batching server over bmg_server_* (see include/bmg.h)."""

    def __init__(self, hbm_budget_bytes, max_slots=8):
        s = C.c_void_p()
        _check(_lib.bmg_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(s)),
               "bmg_server_create")
        self._s = s
        self._n = {}

    def submit(self, kind="sphere", n_refine=3, k=8, sigma=0.0, tol=1e-8, axes=(1.0, 1.0, 1.0),
               R=1.0, r=0.4, nu=64, nv=32, xyz=None, tri=None, project=None, **solve_opts):
        """Queue one request; returns its id.  solve_opts as in Hierarchy.solve."""
        d, keep = surface_desc(kind, axes, R, r, nu, nv, xyz, tri, project)
        o = _opts(**solve_opts)
        rid = C.c_uint64(0)
        _check(_lib.bmg_server_submit(self._s, C.byref(d), int(n_refine), int(k), float(sigma),
                                      float(tol), C.byref(o), C.byref(rid)), "bmg_server_submit")
        nvtx = finest_vertices(kind, n_refine, nu, nv, d.n_vert, d.n_tri)
        self._n[rid.value] = (int(k), nvtx, keep)
        return rid.value

    def poll(self, rid, evecs=True):
        """None while the request runs; else a dict with status, evals, evecs
        ([N, k] numpy or None), stats and latency_ms."""
        k, n, _ = self._n[rid]
        evals = np.zeros(k, np.float64)
        V = np.zeros((k, n), np.float64) if evecs else None
        rho = np.zeros(k, np.float64)
        delta = np.zeros(k, np.float64)
        st = SolveStats()
        st.rho = rho.ctypes.data_as(C.POINTER(C.c_double))
        st.delta = delta.ctypes.data_as(C.POINTER(C.c_double))
        lat = C.c_double(0.0)
        status = _lib.bmg_server_poll(self._s, C.c_uint64(rid), evals.ctypes.data_as(C.POINTER(C.c_double)),
                                      None if V is None else V.ctypes.data_as(C.POINTER(C.c_double)),
                                      int(n), C.byref(st), C.byref(lat))
        if status == EBUSY:
            return None
        del self._n[rid]
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_
                 if f not in ("rho", "delta", "ramp_evals")}
        stats.update(rho=rho, delta=delta)
        err = _lib.bmg_last_error().decode(errors="replace") if status != OK else ""
        return dict(status=status, evals=evals, evecs=None if V is None else V.T, stats=stats,
                    latency_ms=lat.value, error=err)

    def wait(self, rid, evecs=True, poll_s=0.0005):
        import time
        while True:
            res = self.poll(rid, evecs)
            if res is not None:
                return res
            time.sleep(poll_s)

    def cancel(self, rid):
        _check(_lib.bmg_server_cancel(self._s, C.c_uint64(rid)), "bmg_server_cancel")

    def close(self):
        if getattr(self, "_s", None):
            _lib.bmg_server_destroy(self._s)
            self._s = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def status_string(st):
    return _lib.bmg_status_string(int(st)).decode()
