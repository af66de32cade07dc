"""Plain FP64 CPU oracle of the bootstrap multigrid (BMG) eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product library
(``paper_1511_07042_amd``) never imports, links or calls anything here, and
nothing here imports the product library.

Paper: J. Brannick and S. Cao, "A Bootstrap Multigrid Eigensolver"
(arXiv:1511.07042).  Every module cites the section / equation / algorithm it
follows.  Where the paper is silent the reading used is stated in the module
docstring of the function concerned.

Modules
-------
mesh       surface meshes and uniform refinement with projected midpoints (Sec. 3)
fem        P1 surface-FEM stiffness and mass matrices (Sec. 2, eqs. bl-dis, pb-eig-fea)
transfer   geometric prolongation P_h and restriction P_h^T (Sec. 3, eq. proj-1)
colour     greedy vertex colouring for the multicolour Gauss-Seidel smoother
rng        counter-based Gaussian test vectors (SplitMix64 + Box-Muller)
bmg        the BMG cycle iterated to a residual certificate (Alg. 2/3, Remark 3.2),
           the level ramp (Alg. 4) and the smoothers (Jacobi, GS, Kaczmarz)
twogrid    the two-grid Alg. 1 applied in a cascade (Remark 3.1)
estimator  the a posteriori error estimator eta_T (Sec. 5, eq. est-res)
reference  the plain definition of the result: library generalized eigensolves

Parity status: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants or library
eigensolvers.  The only unpinned items are the paper's own worked numbers that
need the authors' Distmesh mesh (not available); they are not computed here.
"""
