"""Write stored reference eigenvalues for the full-size parity tests.

Calls only the oracle: the hierarchy and P1 matrices of oracle.bmg and the
library eigensolver wrapper oracle.reference.discrete_eigs (ARPACK
shift-invert), and for interior shifts the oracle's own BMG solve, whose
cycle count and largest deviation from ARPACK go into the file's header.
Usage:  python tests/golden/make_reference_eigs.py c4|c3|c2
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import bmg, reference  # noqa: E402

CASES = {
    # name: (surface, axes, n_refine, count, sigma)
    "c4": ("sphere", (1.0, 1.0, 1.0), 8, 80, 0.0),
    "c3": ("ellipsoid", (1.0, 1.5, 2.0), 7, 40, 100.0),
    "c2": ("sphere", (1.0, 1.0, 1.0), 6, 40, 0.0),
}


def main(name):
    kind, axes, nref, count, sigma = CASES[name]
    t0 = time.time()
    lv = bmg.build_levels(kind, nref, axes=axes)
    ev, _ = reference.discrete_eigs(lv[-1].A, lv[-1].M, count, sigma, extra=16)
    t_ref = time.time() - t0
    note = []
    if sigma > 0:
        # the oracle's interior-shift BMG on the same pencil (16 pairs, 24 vectors)
        t1 = time.time()
        bev, _, info = bmg.solve(lv, 16, sigma, 1e-8, m=24, smoother="jacobi")
        near = ev[np.sort(np.argsort(abs(ev - sigma), kind="stable")[:16])]
        dev = float(np.max(abs(bev - near) / np.maximum(abs(near), 1.0)))
        note.append(f"# Oracle BMG (shifted scheme, weighted Jacobi, 16 pairs, m = 24): converged = "
                    f"{info['converged']} after {info['cycles']} cycles (l_c = {info['l_c']}), "
                    f"max relative deviation {dev:.1e}, {time.time() - t1:.0f} s.\n")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_{kind}_ref{nref}_eigs.txt")
    with open(out, "w") as f:
        f.write(f"# {count} eigenvalues of the P1 pencil (A_L, M_L) nearest sigma = {sigma}, ascending;\n")
        f.write(f"# {kind} axes {axes}, icosahedron refined {nref} times ({lv[-1].n} vertices).\n")
        f.write("# Written by tests/golden/make_reference_eigs.py (oracle hierarchy + ARPACK shift-invert,\n")
        f.write(f"# tol 1e-14) in {t_ref:.0f} s.\n")
        for line in note:
            f.write(line)
        for v in ev:
            f.write(f"{v:.17e}\n")
    print(out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c4")
