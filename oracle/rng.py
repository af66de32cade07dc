"""Counter-based Gaussian test vectors.

The paper starts BFMG from prolongated coarse eigenfunctions (Alg. 4, step 1);
the benchmark workloads instead draw the initial block of test vectors from
N(0, 1) with a seed, in the spirit of the random test vectors of the BAMG setup
(Sec. 1.1).  To let an independent implementation draw the very same block, the
generator is defined element by element:

  * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output of the
    generator whose state was just advanced to x is mix(x + 0x9E3779B97F4A7C15),
    mix(z) = z ^ (z >> 31) after z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 and
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB (all modulo 2^64);
  * element (i, j) of an N x m block uses counter c = i*m + j and the two
    uniforms u1 = ((splitmix64(seed ^ 2c) >> 11) + 1) * 2^-53 and
    u2 = ((splitmix64(seed ^ (2c+1)) >> 11) + 1) * 2^-53, both in (0, 1];
  * Box-Muller (1958): z = sqrt(-2 ln u1) * cos(2 pi u2).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output for state values x (uint64 array), i.e. mix(x + gamma)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed, count):
    """The first `count` outputs of a SplitMix64 generator started at `seed`."""
    with np.errstate(over="ignore"):
        states = np.uint64(seed) + np.arange(count, dtype=np.uint64) * _GOLDEN
    return splitmix64(states)


def uniform01(seed, counters):
    """((splitmix64(seed ^ c) >> 11) + 1) * 2^-53, in (0, 1]."""
    c = np.asarray(counters, dtype=np.uint64)
    bits = splitmix64(np.uint64(seed) ^ c) >> np.uint64(11)
    return (bits.astype(np.float64) + 1.0) * 2.0 ** -53


def gaussian_block(n, m, seed):
    """N x m block of N(0,1) entries, element (i, j) from counter i*m + j."""
    c = np.arange(n * m, dtype=np.uint64)
    u1 = uniform01(seed, np.uint64(2) * c)
    u2 = uniform01(seed, np.uint64(2) * c + np.uint64(1))
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(n, m)
