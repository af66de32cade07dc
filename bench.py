#!/usr/bin/env python3
"""Benchmark of the BMG eigensolver hot path on one MI355X.

A step is one complete solve: the k eigenpairs nearest sigma of the workload's
finest-level pencil, iterated to the 1e-8 certificate (every row of the cycle:
residual SpMM, correction V-cycle, Gram, Ritz, update) and written out as
M-orthonormal eigenvectors in device memory.  The hierarchy and matrices are
resident in HBM before the timed region; the test vectors are drawn on the
device from the step's seed (seeds 0..steps-1).  `value` is converged
eigenpairs per second of the FP32/FP64 mixed path on the largest single-GPU
workload, the sphere refined 8 times (655362 vertices, k = 64, m = 80); the
plain FP64 GPU path is timed beside it.

Beside the timed solves the JSON line carries:
  per_pair_rel_err  each returned eigenvalue against the stored oracle
                    eigenvalues of the same pencil (tests/golden);
  roofline          the kernel class with the largest total time in the mixed
                    breakdown, timed with HIP events recorded at its own
                    launches on the solve's stream; roofline_finest_sweep: the
                    Jacobi sweep on the finest level alone;
  breakdown         per kernel class (each timed in an extra solve);
  c3                the ellipsoid (1, 1.5, 2) refined 7 times, the 16 eigenpairs
                    nearest sigma = 100 (interior-shift scheme);
  c2                the sphere refined 6 times (k = 25), and 16 of its solves
                    run concurrently through the serving API;
  serving           a seeded request stream through the continuous-batching server;
  cpu_baseline      the oracle (plain FP64 CPU implementation) on the headline
                    workload: its start and a few cycles timed, the full solve
                    extrapolated to the GPU's cycle count.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Kernel classes: bound and whether the library's figure counts bytes or flops.
KCLASS = {"eigres": ("hbm", "GB/s"), "spmm_am": ("hbm", "GB/s"), "smooth": ("hbm", "GB/s"),
          "residual": ("hbm", "GB/s"), "restrict": ("hbm", "GB/s"), "prolong": ("hbm", "GB/s"),
          "gram": ("mfma", "TFLOP/s"), "update": ("mfma", "TFLOP/s"), "ritz": ("latency", "us"),
          "smooth_pair": ("hbm", "GB/s"), "restrict_res": ("hbm", "GB/s"),
          "prolong_smooth": ("hbm", "GB/s"), "smooth_add": ("hbm", "GB/s")}

# Kernel symbols of the classes (template arguments of the mixed / FP64 paths).
KSYMBOL = {"smooth": "k_rowop<{T}, 2, 7>", "residual": "k_rowop<{T}, 1, 7>",
           "restrict": "k_restrict<{T}>", "prolong": "k_prolong_add<{T}>",
           "smooth_pair": "k_jacobi2z<{T}, 7>", "restrict_res": "k_resrestrict<{T}, 7>",
           "prolong_smooth": "k_prolong_jacobi<{T}, 7>", "eigres": "k_eigres<{T}, 7>",
           "spmm_am": "k_spmm_am<7>", "gram": "k_gram_sym1 + k_gram_sym_reduce", "update": "k_update_zy",
           "ritz": "k_ritz", "smooth_add": "k_rowop<{T}, 4, 7>"}

# Committed HBM-traffic summaries (two rocprofv3 --pmc passes each).
TRAFFIC_FILES = {
    ("smooth", "c4_sphere_ref8", "mixed"): "profiles/jacobi_sweep_c4_sphere_ref8_traffic.txt",
    ("gram", "c4_sphere_ref8", "mixed"): "profiles/gram_c4_sphere_ref8_traffic.txt",
}
ROW_KERNELS = "paper_1511_07042_amd/csrc/kernels_sparse.hip"

# Stored eigenvalues of each workload's pencil (written from the oracle by
# tests/golden/make_reference_eigs.py): the per-pair error of the timed solves.
GOLDEN = {"c4_sphere_ref8": "tests/golden/c4_sphere_ref8_eigs.txt",
          "c3_ellipsoid_ref7_sigma100": "tests/golden/c3_ellipsoid_ref7_eigs.txt",
          "c2_sphere_ref6": "tests/golden/c2_sphere_ref6_eigs.txt"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_sphere_ref8")
    ap.add_argument("--smoother", default="jacobi", choices=["gs", "jacobi"])
    ap.add_argument("--only", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--timed-kernel", default=None,
                    help="kernel class for the roofline (default: the bandwidth-bound class "
                         "with the largest total time in the mixed breakdown)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the interior-shift section")
    ap.add_argument("--no-c2", action="store_true", help="skip the 40962-vertex section")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the 16 concurrent C2 solves through the serving API")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the per-class breakdown")
    ap.add_argument("--serving", type=int, default=256, metavar="N",
                    help="requests in the serving section (0: skip it)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving stream and print its JSON line")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--serving-no-shift", action="store_true",
                    help="all requests at sigma = 0 (no interior shifts)")
    ap.add_argument("--serving-kinds", default="sphere,ellipsoid,torus")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (5 times) and exit: the "
                         "reference for scaling hardware byte counters")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 5}))


def kernel_source_hash(rel=ROW_KERNELS):
    """sha256 of a kernel source file: traffic summaries taken with other
    kernel code are not reported."""
    src = open(os.path.join(ROOT, rel), "rb").read()
    return hashlib.sha256(src).hexdigest()


def measured_traffic(kclass, workload, prec, per_unit):
    """HBM bytes per launch from committed counter runs, or None when there are
    none for this kernel and workload, the kernel source changed since, or the
    launches it averages over differ from this run's (their algorithmic bytes
    per launch, per_unit, must match the recorded ones)."""
    rel = TRAFFIC_FILES.get((kclass, workload, prec))
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    kv = {}
    for line in open(os.path.join(ROOT, rel)):
        if "=" in line and not line.startswith("#"):
            key, val = line.split("=", 1)
            kv[key.strip()] = val.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash(kv.get("kernel_source", ROW_KERNELS)):
        return None
    # the amount the roofline counts per launch (bytes, or flops for a matrix-core class)
    algo = float(kv.get("algorithmic_per_launch", kv.get("algorithmic_bytes_per_launch", "nan")))
    if not abs(algo - per_unit) <= 0.5:
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(kclass, ms, amount, units, prec="mixed"):
    bound, unit = KCLASS[kclass]
    name = KSYMBOL[kclass].format(T="float" if prec == "mixed" else "double")
    if units == 0 or ms <= 0:
        return None
    if bound == "hbm":
        achieved = amount / (ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    elif bound == "mfma":
        achieved = amount / (ms * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS
    else:
        return {"bound": "latency", "kernel": name, "class": kclass, "units": int(units),
                "avg_unit_us": round(1e3 * ms / units, 3)}
    return {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": None, "kernel": name, "class": kclass,
            "units": int(units), "avg_unit_us": round(1e3 * ms / units, 3),
            "per_unit": round(amount / units, 1)}


def timed_solves(h, cfg, precision, smoother, steps, warmup, timed_kernel=None, evecs="device"):
    """W untimed warm-up solves, then exactly `steps` solves between two device
    synchronisations, each writing its eigenvectors to device memory.
    Returns (seconds, per-solve stats, per-solve eigenvalues)."""
    import torch
    kw = dict(m=cfg["m"], nu1=cfg["nu1"], nu2=cfg["nu2"], smoother=smoother, precision=precision,
              evecs=evecs, timed_kernel=timed_kernel)
    for s in range(warmup):
        h.solve(cfg["k"], cfg["sigma"], cfg["tol"], seed=1000 + s, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, evals = [], []
    for s in range(steps):
        ev, _, st = h.solve(cfg["k"], cfg["sigma"], cfg["tol"], seed=s, **kw)
        assert st["converged"] == 1, st
        stats.append(st)
        evals.append(ev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, stats, evals


def per_pair_error(name, cfg, evals):
    """Relative error max(|lambda|, 1) of every returned eigenvalue against the
    stored oracle eigenvalues (the k nearest sigma among them)."""
    import numpy as np
    rel = GOLDEN.get(name)
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    ref = np.array([float(x) for x in open(os.path.join(ROOT, rel)) if not x.startswith("#")])
    near = np.sort(ref[np.sort(np.argsort(np.abs(ref - cfg["sigma"]), kind="stable")[:cfg["k"]])])
    errs = [np.abs(np.asarray(ev) - near) / np.maximum(np.abs(near), 1.0) for ev in evals]
    return {"max": float(max(e.max() for e in errs)),
            "seed0": [float("%.3g" % v) for v in errs[0]],
            "reference": rel, "note": "relative to max(|lambda|, 1); every timed seed checked"}


def breakdown(h, cfg, prec, smoother):
    """Every kernel class timed with events in one extra solve (seed 0)."""
    bd = {}
    for kc in KCLASS:
        _, st, _ = timed_solves(h, cfg, prec, smoother, 1, 0, kc, evecs=None)
        r = roofline(kc, st[0]["timed_kernel_ms"], st[0]["timed_kernel_bytes"],
                     st[0]["timed_kernel_units"], prec)
        if r is not None:  # classes fused away in this configuration are absent
            bd[kc] = dict(ms_per_solve=round(st[0]["timed_kernel_ms"], 3), **r)
    return bd


def class_roofline(h, name, cfg, prec, smoother, steps, kc, level=None):
    """Events around each launch of one kernel class (on one level if given),
    in solves of the same workload and seeds as the timed region."""
    tk = kc if level is None else (kc, level)
    _, tst, _ = timed_solves(h, cfg, prec, smoother, steps, 0, tk, evecs=None)
    roof = roofline(kc, sum(s["timed_kernel_ms"] for s in tst),
                    sum(s["timed_kernel_bytes"] for s in tst),
                    sum(s["timed_kernel_units"] for s in tst), prec)
    if roof is not None and "frac" in roof:
        roof["traffic"] = measured_traffic(kc, name, prec, roof["per_unit"]) if level is None else None
        if level is not None:
            roof["level"] = level
    return roof


def bench_workload(bmg, name, cfg, precs, steps, warmup, smoother, timed_kernel, with_breakdown=True):
    """Timed solves of one workload for each precision, the per-pair error, the
    breakdown, and the roofline of the dominant kernel class."""
    import torch
    t0 = time.perf_counter()
    h = bmg.Hierarchy(cfg["kind"], cfg["n_refine"], axes=cfg["axes"])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    out = {"hierarchy_build_s": round(build_s, 3)}
    for prec in precs:
        dt, stats, evals = timed_solves(h, cfg, prec, smoother, steps, warmup)
        r = dict(value=round(steps * cfg["k"] / dt, 3), ms_per_step=round(1e3 * dt / steps, 3),
                 cycles=[s["cycles"] for s in stats],
                 t_solve_ms=[round(s["t_solve_ms"], 3) for s in stats],
                 scheme=["", "enriched", "shifted"][stats[0]["scheme"]], l_c=stats[0]["l_c"],
                 coarse_eig_ms=round(max(s["coarse_eig_ms"] for s in stats), 1),
                 ritz_sweeps_max=max(s["ritz_sweeps_max"] for s in stats),
                 ritz_fallbacks=sum(s["ritz_fallbacks"] for s in stats))
        r["per_pair_rel_err"] = per_pair_error(name, cfg, evals)
        kc = timed_kernel
        if with_breakdown:
            r["breakdown"] = breakdown(h, cfg, prec, smoother)
            if kc is None:
                timed = [(v["ms_per_solve"], k) for k, v in r["breakdown"].items()
                         if v["bound"] in ("hbm", "mfma")]
                kc = max(timed)[1]
        if kc is None:
            kc = "smooth"
        r["roofline"] = class_roofline(h, name, cfg, prec, smoother, steps, kc)
        if smoother == "jacobi":
            L = cfg["n_refine"]
            r["roofline_finest_sweep"] = class_roofline(h, name, cfg, prec, smoother, steps, "smooth", L)
        out[prec] = r
        print(f"# {name} {prec}: {r['value']} eigenpairs/s, {r['ms_per_step']} ms/solve, "
              f"cycles {r['cycles']}, roofline {r['roofline']}", file=sys.stderr, flush=True)
    h.close()
    return out


def cpu_baseline(cfg, smoother, gpu_cycles, budget_s=20.0, max_solves=4):
    """The oracle on the host cores, on the headline workload.  Its start
    (coarse vectors, seeded block, first Ritz step) and one cycle are timed; if
    a full solve fits budget_s, full solves (seeds 0, 1, ...) are timed instead,
    else the full solve is extrapolated as start + cycles x cycle time with the
    GPU's FP64 cycle count for the same seed."""
    import threadpoolctl
    from oracle import bmg as ob
    lv = ob.build_levels(cfg["kind"], cfg["n_refine"], axes=cfg["axes"])
    kw = dict(m=cfg["m"], nu1=cfg["nu1"], nu2=cfg["nu2"], smoother=smoother)
    t0 = time.perf_counter()
    ob.solve(lv, cfg["k"], cfg["sigma"], cfg["tol"], seed=0, max_cycles=0, **kw)
    t_start = time.perf_counter() - t0
    t0 = time.perf_counter()
    ob.solve(lv, cfg["k"], cfg["sigma"], cfg["tol"], seed=0, max_cycles=1, **kw)
    t_cycle = max(time.perf_counter() - t0 - t_start, 1e-9)
    est = t_start + gpu_cycles * t_cycle
    blas = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=1)
    threads = (f"dense BLAS on {blas} threads, scipy.sparse products single-threaded; "
               f"host os.cpu_count() = {os.cpu_count()}")
    if est <= budget_s:
        t0 = time.perf_counter()
        n, cycles = 0, []
        while n < max_solves and (n == 0 or time.perf_counter() - t0 < budget_s):
            _, _, info = ob.solve(lv, cfg["k"], cfg["sigma"], cfg["tol"], seed=n, **kw)
            cycles.append(info["cycles"])
            n += 1
        dt = time.perf_counter() - t0
        return dict(value=round(n * cfg["k"] / dt, 4), unit="eigenpairs/s", cores=int(blas),
                    kind="oracle", extrapolated=False,
                    sample=f"{n} full oracle solves of the same workload, seeds 0..{n - 1} "
                           f"({cycles} cycles, {dt:.1f} s); {threads}")
    return dict(value=round(cfg["k"] / est, 5), unit="eigenpairs/s", cores=int(blas), kind="oracle",
                extrapolated=True, start_s=round(t_start, 2), cycle_s=round(t_cycle, 2),
                cycles=int(gpu_cycles),
                sample=f"the oracle's start (coarse vectors, seeded block, first Ritz step: "
                       f"{t_start:.1f} s) and one cycle ({t_cycle:.1f} s) on the same workload, seed 0; "
                       f"the full solve extrapolated to the {gpu_cycles} cycles the GPU's FP64 path "
                       f"takes for that seed ({est:.0f} s); hierarchy build excluded; {threads}")


def _serve(bmg, reqs, slots, budget, timed, smoother):
    """Submit the requests at their arrival times (all at once unless timed)
    and collect every result.  Returns (results, makespan_s)."""
    t_arr = [r["arrival_s"] if timed else 0.0 for r in reqs]
    out = [None] * len(reqs)
    ids = {}
    with bmg.Server(budget, max_slots=slots) as srv:
        t0 = time.perf_counter()
        nxt = 0
        while nxt < len(reqs) or ids:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and t_arr[nxt] <= now:
                r = reqs[nxt]
                ids[srv.submit(r["kind"], r["n_refine"], r["k"], r["sigma"], r["tol"], axes=r["axes"],
                               smoother=smoother, precision="mixed", seed=r["seed"])] = nxt
                nxt += 1
            for rid in list(ids):
                res = srv.poll(rid, evecs=False)
                if res is not None:
                    out[ids.pop(rid)] = res
                    done = sum(o is not None for o in out)
                    if done % 32 == 0 or done == len(reqs):
                        print(f"# serving ({'timed' if timed else 'capacity'}): {done}/{len(reqs)} requests "
                              f"done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            time.sleep(0.0005)
        makespan = time.perf_counter() - t0
    return out, makespan


def serving(a, bmg):
    """Seeded request stream (surface, level, k, shift per request as drawn by
    workloads.serving_stream); Poisson arrivals at 0.8x the capacity measured
    on the same requests submitted all at once."""
    import numpy as np
    from workloads import serving_stream
    kinds = set(a.serving_kinds.split(","))
    full = serving_stream(4 * a.serving, seed=0, rate_per_s=1.0, sigma_positive=not a.serving_no_shift)
    reqs = [r for r in full if r["kind"] in kinds][:a.serving]
    budget = int(a.serving_budget_gib * (1 << 30))
    _, span = _serve(bmg, reqs, a.serving_slots, budget, False, a.smoother)
    capacity = len(reqs) / span
    rate = 0.8 * capacity
    gaps = np.diff([0.0] + [r["arrival_s"] for r in reqs])
    for r, ti in zip(reqs, np.cumsum(gaps / rate)):
        r["arrival_s"] = float(ti)
    res, span = _serve(bmg, reqs, a.serving_slots, budget, True, a.smoother)
    lat = np.array([r["latency_ms"] for r in res])
    ok = [r["status"] == 0 for r in res]
    status, by_kind = {}, {}
    for q, r in zip(reqs, res):
        s = bmg.status_string(r["status"])
        status[s] = status.get(s, 0) + 1
        d = by_kind.setdefault(q["kind"] + ("/shift" if q["sigma"] else ""), {"n": 0, "ok": 0, "lat": []})
        d["n"] += 1
        d["ok"] += int(r["status"] == 0)
        d["lat"].append(r["latency_ms"])
    for d in by_kind.values():
        d["p50_ms"] = round(float(np.percentile(d.pop("lat"), 50)), 2)
    okl = lat[np.array(ok)] if any(ok) else lat
    return {
        "metric": "serving: converged eigenpairs/s and request latency (BMG, mixed precision)",
        "value": round(sum(q["k"] for q, g in zip(reqs, ok) if g) / span, 3), "unit": "eigenpairs/s",
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "p50_ms_converged": round(float(np.percentile(okl, 50)), 2),
        "p99_ms_converged": round(float(np.percentile(okl, 99)), 2),
        "requests": len(reqs), "converged": int(sum(ok)), "status": status, "by_kind": by_kind,
        "rate_req_s": round(rate, 3), "capacity_req_s": round(capacity, 3),
        "makespan_s": round(span, 3), "slots": a.serving_slots, "budget_gib": a.serving_budget_gib,
        "seed": 0, "data": "synthetic",
        "cycles_p50": float(np.percentile([r["stats"]["cycles"] for r in res], 50)),
        "grouped_requests": int(sum(r["stats"]["group_size"] > 1 for r in res)),
        "max_group_size": int(max(r["stats"]["group_size"] for r in res)),
        "config": {"workload": "c5_serving_stream", "kinds": sorted(kinds),
                   "shifts": not a.serving_no_shift, "smoother": a.smoother},
    }


def concurrent(bmg, cfg, smoother, n_req=16, slots=8, grouping=True):
    """Independent solves of one workload (seeds 0..n_req-1) through the server
    at once: whole-device throughput when several solves share the device, as
    grouped solves (compatible requests waiting together run as one
    concatenated block) or, with grouping off, side by side on their own
    streams.  Reported beside `value`, not as it."""
    kw = dict(m=cfg["m"], nu1=cfg["nu1"], nu2=cfg["nu2"], smoother=smoother, precision="mixed")
    if grouping:
        os.environ.pop("BMG_NO_GROUP", None)
    else:
        os.environ["BMG_NO_GROUP"] = "1"  # read when the server is created
    def batch(srv, seed0):
        t0 = time.perf_counter()
        ids = [srv.submit(cfg["kind"], cfg["n_refine"], cfg["k"], cfg["sigma"], cfg["tol"],
                          axes=cfg["axes"], seed=seed0 + s, **kw) for s in range(n_req)]
        res = [srv.wait(i, evecs=False) for i in ids]
        return time.perf_counter() - t0, res

    with bmg.Server(64 << 30, max_slots=slots) as srv:
        # an untimed batch first: builds the hierarchy and the solo and grouped
        # workspaces (and their graphs), as the warm-up steps do for `value`
        batch(srv, 1000)
        runs = [batch(srv, 0) for _ in range(3)]
    os.environ.pop("BMG_NO_GROUP", None)
    dts = [dt for dt, _ in runs]
    dt, res = sorted(runs, key=lambda r: r[0])[1]  # the median batch
    ok = sum(r["status"] == 0 for r in res)
    return {"value": round(ok * cfg["k"] / dt, 3), "unit": "eigenpairs/s", "solves": n_req,
            "converged": ok, "slots": slots, "seconds": round(dt, 4),
            "seconds_all": [round(t, 4) for t in dts], "grouping": grouping,
            "group_sizes": sorted((r["stats"]["group_size"] for r in res), reverse=True),
            "note": "independent solves run concurrently through the serving API (median of "
                    "three batches after an untimed one); not the single-solve `value`"}


def section(bmg, name, precs, steps, warmup, smoother, with_breakdown=False):
    """A secondary workload: timed solves and the roofline of its dominant class."""
    from workloads import CONFIGS
    cfg = CONFIGS[name]
    res = bench_workload(bmg, name, cfg, precs, steps, warmup, smoother, None, with_breakdown)
    mp = "mixed" if "mixed" in res else precs[0]
    return {"config": {"workload": name, **cfg}, "value": res[mp]["value"], "unit": "eigenpairs/s",
            "ms_per_step": res[mp]["ms_per_step"], "roofline": res[mp]["roofline"],
            "per_pair_rel_err_max": (res[mp]["per_pair_rel_err"] or {}).get("max"),
            "mixed_vs_fp64": (round(res["mixed"]["value"] / res["fp64"]["value"], 3)
                              if "mixed" in res and "fp64" in res else None),
            "hierarchy_build_s": res["hierarchy_build_s"],
            "fp64_path": res.get("fp64"), "mixed_path": res.get("mixed")}


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    import paper_1511_07042_amd as bmg
    from workloads import CONFIGS
    if a.serving_only:
        print(json.dumps(serving(a, bmg)), flush=True)
        return
    precs = ["fp64", "mixed"] if a.only == "both" else [a.only]
    cfg = CONFIGS[a.workload]
    main_res = bench_workload(bmg, a.workload, cfg, precs, a.steps, a.warmup, a.smoother,
                              a.timed_kernel, not a.no_breakdown)
    mp = "mixed" if "mixed" in main_res else a.only
    out = {
        "metric": "converged eigenpairs/s at 1e-8 rel (FP32/FP64 mixed BMG)",
        "value": main_res[mp]["value"],
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_res[mp]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mp == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, **{k: v for k, v in cfg.items()}, "smoother": a.smoother,
                   "hierarchy_build_s": main_res["hierarchy_build_s"],
                   "evecs": "written to device memory in every timed solve"},
        "per_pair_rel_err": main_res[mp]["per_pair_rel_err"],
        "roofline": main_res[mp]["roofline"],
        "roofline_finest_sweep": main_res[mp].get("roofline_finest_sweep"),
        "mixed_vs_fp64": (round(main_res["mixed"]["value"] / main_res["fp64"]["value"], 3)
                          if a.only == "both" else None),
        "fp64_path": main_res.get("fp64"),
        "mixed_path": main_res.get("mixed"),
    }
    if not a.no_c3 and a.workload != "c3_ellipsoid_ref7_sigma100":
        out["c3"] = section(bmg, "c3_ellipsoid_ref7_sigma100", precs, a.steps, 1, a.smoother)
    if not a.no_c2 and a.workload != "c2_sphere_ref6":
        out["c2"] = section(bmg, "c2_sphere_ref6", precs, a.steps, 1, a.smoother)
        if a.only in ("both", "mixed") and not a.no_concurrent:
            out["c2"]["concurrent"] = concurrent(bmg, CONFIGS["c2_sphere_ref6"], a.smoother)
            out["c2"]["concurrent_ungrouped"] = concurrent(bmg, CONFIGS["c2_sphere_ref6"], a.smoother,
                                                           grouping=False)
    if a.serving > 0:
        out["serving"] = serving(a, bmg)
    if not a.no_cpu_baseline:
        fp = main_res.get("fp64") or main_res[mp]
        out["cpu_baseline"] = cpu_baseline(cfg, a.smoother, fp["cycles"][0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
