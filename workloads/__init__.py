"""Benchmark and test workloads: seeded, synthetic problem descriptions.

This module holds only the descriptions of the inputs (surface, refinement
level, number of eigenpairs, block width, shift, tolerance) and the seeded
generators of request streams.  It contains none of the solver's arithmetic,
so both the oracle-based tests and the GPU path can use it.

The paper's experiments use a Distmesh sphere with 54 vertices that is not
available; these icosphere / ellipsoid / torus families stand in for it.
"""
import numpy as np

# sphere: icosahedron inscribed in the unit sphere, refined n_refine times
# ellipsoid: the same hierarchy mapped by x -> (a0 x, a1 y, a2 z)
CONFIGS = {
    "c1_sphere_ref3": dict(kind="sphere", axes=(1.0, 1.0, 1.0), n_refine=3, k=9, m=12,
                           sigma=0.0, tol=1e-8, nu1=2, nu2=2),
    "c2_sphere_ref6": dict(kind="sphere", axes=(1.0, 1.0, 1.0), n_refine=6, k=25, m=32,
                           sigma=0.0, tol=1e-8, nu1=2, nu2=2),
    "c3_ellipsoid_ref7_sigma100": dict(kind="ellipsoid", axes=(1.0, 1.5, 2.0), n_refine=7, k=16,
                                       m=24, sigma=100.0, tol=1e-8, nu1=2, nu2=2),
    "c4_sphere_ref8": dict(kind="sphere", axes=(1.0, 1.0, 1.0), n_refine=8, k=64, m=80,
                           sigma=0.0, tol=1e-8, nu1=2, nu2=2),
}


def icosphere_vertices(n_refine):
    return 10 * 4 ** n_refine + 2


def serving_stream(n_requests=256, seed=0, rate_per_s=100.0, sigma_positive=False):
    """Seeded request stream: Poisson arrivals and random problem descriptions.

    Each request: surface uniform over {sphere, ellipsoid with axes U[1,2]^3,
    torus R=1, r=0.4}; icosphere refinement U{3..7} (torus refinements U{1..4});
    k ~ U{4..32}; sigma = 0, or U[10,200] with probability 1/2 when
    sigma_positive is set.
    """
    rs = np.random.default_rng(seed)
    t = np.cumsum(rs.exponential(1.0 / rate_per_s, n_requests))
    reqs = []
    for i in range(n_requests):
        kind = ["sphere", "ellipsoid", "torus"][rs.integers(3)]
        axes = tuple(rs.uniform(1.0, 2.0, 3)) if kind == "ellipsoid" else (1.0, 1.0, 1.0)
        n_refine = int(rs.integers(1, 5)) if kind == "torus" else int(rs.integers(3, 8))
        k = int(rs.integers(4, 33))
        sigma = float(rs.uniform(10, 200)) if (sigma_positive and rs.random() < 0.5) else 0.0
        reqs.append(dict(id=i, arrival_s=float(t[i]), kind=kind, axes=axes, n_refine=n_refine,
                         k=k, sigma=sigma, tol=1e-8, seed=i))
    return reqs
