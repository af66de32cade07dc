#!/usr/bin/env python3
"""Benchmark of the BMG eigensolver hot path on one MI355X.

A step is one complete solve: the k eigenpairs nearest sigma of the workload's
finest-level pencil, iterated to the 1e-8 certificate (every row of the cycle:
residual SpMM, correction V-cycle, Gram, Ritz, update).  The inputs (hierarchy
and matrices) are resident in HBM before the timed region; the test vectors are
drawn on the device from the step's seed.  `value` is converged eigenpairs per
second of the FP32/FP64 mixed path; the plain FP64 GPU path is timed beside it.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_sphere_ref6")
    ap.add_argument("--smoother", default="jacobi", choices=["gs", "jacobi"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--timed-kernel", default="smooth",
                    help="kernel class timed with HIP events inside the timed region (roofline)")
    ap.add_argument("--breakdown", action="store_true",
                    help="after the timed region, time every kernel class in extra solves")
    ap.add_argument("--serving", type=int, default=0, metavar="N",
                    help="instead of the solve benchmark, serve a seeded stream of N requests "
                         "(Poisson arrivals at 0.8x the measured capacity) and report latency")
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


# Kernel classes: bound and whether the library's figure counts bytes or flops.
KCLASS = {"eigres": ("hbm", "GB/s"), "spmm_am": ("hbm", "GB/s"), "smooth": ("hbm", "GB/s"),
          "residual": ("hbm", "GB/s"), "restrict": ("hbm", "GB/s"), "prolong": ("hbm", "GB/s"),
          "gram": ("mfma", "TFLOP/s"), "update": ("mfma", "TFLOP/s"), "ritz": ("latency", "us"),
          "smooth_pair": ("hbm", "GB/s"), "restrict_res": ("hbm", "GB/s"),
          "prolong_smooth": ("hbm", "GB/s")}
FP64_PEAK_TFLOPS = 78.6


TRAFFIC_FILES = {("smooth", "jacobi", "c2_sphere_ref6", "mixed"):
                 "profiles/jacobi_sweep_c2_sphere_ref6_traffic.txt"}


def kernel_source_hash():
    """sha256 of the weighted-Jacobi row kernel's source text (its template)."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_1511_07042_amd", "csrc", "kernels_sparse.hip")).read()
    m = re.search(r"template <typename T, int MODE, bool FUSE>\n__global__.*?\n}\n", src, re.S)
    return hashlib.sha256(m.group(0).encode()).hexdigest() if m else None


def measured_traffic(kclass, smoother, workload, prec):
    """HBM bytes per launch from committed counter runs, or None when there are
    none for this kernel and workload or the kernel changed since they were taken."""
    rel = TRAFFIC_FILES.get((kclass, smoother, workload, prec))
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    kv = {}
    for line in open(os.path.join(ROOT, rel)):
        if "=" in line and not line.startswith("#"):
            key, val = line.split("=", 1)
            kv[key.strip()] = val.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(kclass, ms, amount, units):
    bound, unit = KCLASS[kclass]
    if bound == "hbm":
        achieved = amount / (ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    elif bound == "mfma":
        achieved = amount / (ms * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS
    else:
        return {"bound": "latency", "kernel": kclass, "avg_us": 1e3 * ms / max(units, 1)}
    return {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": None, "kernel": kclass,
            "units": int(units), "avg_unit_us": round(1e3 * ms / max(units, 1), 3),
            "per_unit": round(amount / max(units, 1), 1)}


def timed_solves(h, cfg, precision, smoother, steps, warmup, timed_kernel=None):
    import torch
    kw = dict(m=cfg["m"], nu1=cfg["nu1"], nu2=cfg["nu2"], smoother=smoother, precision=precision,
              evecs=None, timed_kernel=timed_kernel)
    for s in range(warmup):
        h.solve(cfg["k"], cfg["sigma"], cfg["tol"], seed=1000 + s, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for s in range(steps):
        _, _, st = h.solve(cfg["k"], cfg["sigma"], cfg["tol"], seed=s, **kw)
        assert st["converged"] == 1, st
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, stats


def cpu_baseline(cfg, smoother):
    """The oracle on the host cores: one solve of the same workload (seed 0)."""
    import threadpoolctl
    from oracle import bmg as ob
    lv = ob.build_levels(cfg["kind"], cfg["n_refine"], axes=cfg["axes"])
    t0 = time.perf_counter()
    ev, _, info = ob.solve(lv, cfg["k"], cfg["sigma"], cfg["tol"], m=cfg["m"], nu1=cfg["nu1"],
                           nu2=cfg["nu2"], smoother=smoother)
    dt = time.perf_counter() - t0
    blas = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=1)
    return dict(value=cfg["k"] / dt, unit="eigenpairs/s", cores=int(blas), kind="oracle",
                sample=f"one full oracle solve of the same workload, seed 0 ({info['cycles']} cycles, "
                       f"{dt:.1f} s; dense BLAS on {blas} threads, scipy.sparse products single-threaded)")


def _serve(bmg, reqs, slots, budget, rate=None, smoother="jacobi"):
    """Submit the requests at their arrival times (all at once if rate is None)
    and collect every result.  Returns (results, makespan_s)."""
    import numpy as np
    t_arr = [0.0] * len(reqs) if rate is None else [r["arrival_s"] for r in reqs]
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
            time.sleep(0.0005)
        makespan = time.perf_counter() - t0
    return out, makespan


def serving(a):
    """Serving stream (seeded): surface, level, k and shift per request drawn as
    in workloads.serving_stream; arrivals Poisson at 0.8x the capacity measured
    on the same stream submitted all at once."""
    import numpy as np
    import torch
    import paper_1511_07042_amd as bmg
    from workloads import serving_stream
    torch.cuda.set_device(0)
    kinds = set(a.serving_kinds.split(","))
    full = serving_stream(4 * a.serving, seed=0, rate_per_s=1.0, sigma_positive=not a.serving_no_shift)
    reqs = [r for r in full if r["kind"] in kinds][:a.serving]
    budget = int(a.serving_budget_gib * (1 << 30))
    # capacity: every request submitted at t = 0, hierarchies built on demand
    res, span = _serve(bmg, reqs, a.serving_slots, budget, None, a.smoother)
    capacity = len(reqs) / span
    rate = 0.8 * capacity
    print(f"# capacity {capacity:.2f} req/s over {span:.2f} s; serving at {rate:.2f} req/s",
          file=sys.stderr, flush=True)
    # timed run: Poisson arrivals (the stream's seeded exponential gaps, rescaled)
    gaps = np.diff([0.0] + [r["arrival_s"] for r in reqs])
    t = np.cumsum(gaps / rate)
    for r, ti in zip(reqs, t):
        r["arrival_s"] = float(ti)
    res, span = _serve(bmg, reqs, a.serving_slots, budget, rate, a.smoother)
    lat = np.array([r["latency_ms"] for r in res])
    ok = [r["status"] == 0 for r in res]
    pairs = sum(q["k"] for q, good in zip(reqs, ok) if good)
    status = {}
    for r in res:
        status[bmg.status_string(r["status"])] = status.get(bmg.status_string(r["status"]), 0) + 1
    by_kind = {}
    for q, r in zip(reqs, res):
        d = by_kind.setdefault(q["kind"] + ("/shift" if q["sigma"] else ""), {"n": 0, "ok": 0, "lat": []})
        d["n"] += 1
        d["ok"] += int(r["status"] == 0)
        d["lat"].append(r["latency_ms"])
    for d in by_kind.values():
        d["p50_ms"] = round(float(np.percentile(d.pop("lat"), 50)), 2)
    out = {
        "metric": "serving: converged eigenpairs/s and request latency (BMG, mixed precision)",
        "value": round(pairs / span, 3), "unit": "eigenpairs/s", "n_gpus": 1,
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "requests": len(reqs), "converged": int(sum(ok)), "status": status, "by_kind": by_kind,
        "rate_req_s": round(rate, 3), "capacity_req_s": round(capacity, 3),
        "makespan_s": round(span, 3), "slots": a.serving_slots,
        "budget_gib": a.serving_budget_gib, "seed": 0, "data": "synthetic",
        "cycles_p50": float(np.percentile([r["stats"]["cycles"] for r in res], 50)),
        "config": {"workload": "c5_serving_stream", "kinds": sorted(kinds),
                   "shifts": not a.serving_no_shift, "smoother": a.smoother},
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.serving:
        serving(a)
        return
    import torch
    import paper_1511_07042_amd as bmg
    from workloads import CONFIGS
    cfg = CONFIGS[a.workload]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    h = bmg.Hierarchy(cfg["kind"], cfg["n_refine"], axes=cfg["axes"])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    res = {}
    roof = {}
    for prec in (["fp64", "mixed"] if a.only == "both" else [a.only]):
        # timed region: the production path (cycle replayed as a HIP graph)
        dt, stats = timed_solves(h, cfg, prec, a.smoother, a.steps, a.warmup)
        res[prec] = dict(value=a.steps * cfg["k"] / dt, ms_per_step=1e3 * dt / a.steps,
                         cycles=[s["cycles"] for s in stats],
                         t_solve_ms=[round(s["t_solve_ms"], 3) for s in stats],
                         ritz_sweeps_max=max(s["ritz_sweeps_max"] for s in stats),
                         ritz_fallbacks=sum(s["ritz_fallbacks"] for s in stats))
        # roofline kernel: HIP events around each of its launches on the solve's
        # stream, in solves of the same workload and seeds (plain launches)
        _, tst = timed_solves(h, cfg, prec, a.smoother, a.steps, 0, a.timed_kernel)
        roof[prec] = roofline(a.timed_kernel, sum(s["timed_kernel_ms"] for s in tst),
                              sum(s["timed_kernel_bytes"] for s in tst),
                              sum(s["timed_kernel_units"] for s in tst))
        if "frac" in roof[prec]:
            roof[prec]["traffic"] = measured_traffic(a.timed_kernel, a.smoother, a.workload, prec)
            tb = "float" if prec == "mixed" else "double"
            roof[prec]["kernel"] = (f"k_rowop<{tb}, 2, false> (weighted-Jacobi sweep, levels >= 3)"
                                    if a.timed_kernel == "smooth" and a.smoother == "jacobi" else a.timed_kernel)
        print(f"# {prec}: {res[prec]} roofline {roof[prec]}", file=sys.stderr, flush=True)
        if a.breakdown:
            bd = {}
            for kc in KCLASS:
                _, st = timed_solves(h, cfg, prec, a.smoother, 1, 0, kc)
                if st[0]["timed_kernel_units"] == 0:
                    continue  # not launched in this configuration (fused away)
                bd[kc] = dict(ms=round(st[0]["timed_kernel_ms"], 3), **roofline(
                    kc, st[0]["timed_kernel_ms"], st[0]["timed_kernel_bytes"], st[0]["timed_kernel_units"]))
            res[prec]["breakdown"] = bd
            print(f"# {prec} breakdown: {json.dumps(bd)}", file=sys.stderr, flush=True)
    main_prec = "mixed" if "mixed" in res else a.only
    out = {
        "metric": "converged eigenpairs/s at 1e-8 rel (FP32/FP64 mixed BMG)",
        "value": round(res[main_prec]["value"], 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(res[main_prec]["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, **{k: v for k, v in cfg.items()}, "smoother": a.smoother,
                   "hierarchy_build_s": round(build_s, 3)},
        "roofline": roof[main_prec],
        "fp64_path": res.get("fp64"),
        "mixed_path": res.get("mixed"),
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, a.smoother)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
