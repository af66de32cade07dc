"""Build libbmg.so (HIP for gfx950) in-tree.

Every source is compiled by hipcc for gfx950 only; packed FP32 instructions are
disabled for all device code.  Objects go to _build/ at the repository root;
the shared library is written next to this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libbmg.so")

SOURCES = ["mesh.cpp", "assemble.cpp", "dense_host.cpp", "order.cpp", "hierarchy.cpp", "twogrid.cpp", "estimate.cpp", "solver.cpp",
           "capi.cpp", "server.cpp", "dense_device.cpp", "kernels_sparse.hip", "kernels_gram.hip",
           "kernels_dense.hip", "kernels_tail.hip", "kernels_coarse.hip", "kernels_estimate.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    return src, obj, p.returncode, out


def build(verbose=False, jobs=8):
    """Compile every source and link libbmg.so; raises RuntimeError on failure."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    errs = [(s, o) for s, _, rc, o in results if rc != 0]
    for s, _, rc, o in results:
        if o.strip() and (verbose or rc != 0):
            print(f"--- {s}\n{o}", file=sys.stderr)
    if errs:
        raise RuntimeError("compilation failed: " + ", ".join(s for s, _ in errs))
    objs = [o for _, o, _, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + \
        ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-ldl"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
