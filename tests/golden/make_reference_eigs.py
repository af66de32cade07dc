"""Write stored reference eigenvalues for the full-size parity tests.

Calls only the oracle: the hierarchy and P1 matrices of oracle.bmg and the
library eigensolver wrapper oracle.reference.discrete_eigs (ARPACK
shift-invert).  Usage:  python tests/golden/make_reference_eigs.py c4
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bmg, reference  # noqa: E402

CASES = {
    # name: (surface, axes, n_refine, count, sigma)
    "c4": ("sphere", (1.0, 1.0, 1.0), 8, 80, 0.0),
}


def main(name):
    kind, axes, nref, count, sigma = CASES[name]
    t0 = time.time()
    lv = bmg.build_levels(kind, nref, axes=axes)
    ev, _ = reference.discrete_eigs(lv[-1].A, lv[-1].M, count, sigma, extra=16)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_{kind}_ref{nref}_eigs.txt")
    with open(out, "w") as f:
        f.write(f"# {count} eigenvalues of the P1 pencil (A_L, M_L) nearest sigma = {sigma}, ascending;\n")
        f.write(f"# {kind} axes {axes}, icosahedron refined {nref} times ({lv[-1].n} vertices).\n")
        f.write("# Written by tests/golden/make_reference_eigs.py (oracle hierarchy + ARPACK shift-invert,\n")
        f.write(f"# tol 1e-14) in {time.time() - t0:.0f} s.\n")
        for v in ev:
            f.write(f"{v:.17e}\n")
    print(out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c4")
