"""Pins of the counter-based test-vector generator (SplitMix64 + Box-Muller)."""
import os

import numpy as np

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_stream():
    ref = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if l[0] != "#"]
    got = [int(x) for x in rng.splitmix64_stream(1234567, len(ref))]
    assert got == ref


def test_uniforms_in_unit_interval_and_counter_layout():
    u = rng.uniform01(3, np.arange(100000, dtype=np.uint64))
    assert u.min() > 0 and u.max() <= 1.0
    g = rng.gaussian_block(300, 8, 5)
    # element (i, j) depends only on (seed, i*m + j)
    c = np.array([7 * 8 + 3], dtype=np.uint64)
    u1 = rng.uniform01(5, 2 * c)
    u2 = rng.uniform01(5, 2 * c + 1)
    z = np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    assert g[7, 3] == z[0]


def test_gaussian_moments():
    g = rng.gaussian_block(2000, 50, 11).ravel()
    n = g.size
    assert abs(g.mean()) < 5 / np.sqrt(n)
    assert abs(g.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(g ** 4) - 3) < 0.1
