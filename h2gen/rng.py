"""Seeded counter-based random numbers for every synthetic input.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state_i = seed + (i+1) * 0x9E3779B97F4A7C15 (mod 2^64),
followed by the published 64-bit finaliser.  Uniforms in [0, 1) take the top
53 bits; normals use the Box-Muller transform on consecutive pairs.

This module holds no arithmetic of the solver: it only produces the points
and right-hand sides that both the oracle and the GPU path consume.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_finalize(z):
    """The SplitMix64 output mix applied elementwise to uint64 values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64(seed, n):
    """First n outputs of SplitMix64 started from `seed`."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + i * _GAMMA
    return splitmix64_finalize(state)


def uniform01(seed, n):
    """n doubles in [0, 1): (z >> 11) * 2^-53."""
    z = splitmix64(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed, n):
    """n standard normals by Box-Muller on consecutive uniform pairs."""
    m = (n + 1) // 2
    u = uniform01(seed, 2 * m)
    r = np.sqrt(-2.0 * np.log1p(-u[0::2]))
    th = 2.0 * np.pi * u[1::2]
    out = np.empty(2 * m)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:n]


def points(seed, n, dim):
    """n points uniform in the unit cube [0,1)^dim, row-major n x dim."""
    return uniform01(seed, n * dim).reshape(n, dim)


def grid_points(n, dim):
    """The n = s^dim cell centres ((i + 1/2)/s, ...) of the uniform grid on [0,1)^dim,
    row-major n x dim, the first coordinate fastest (no random draw)."""
    s = int(round(n ** (1.0 / dim)))
    if s ** dim != n:
        raise ValueError(f"{n} points do not form a {dim}-dimensional grid")
    c = (np.arange(s, dtype=np.float64) + 0.5) / s
    axes = np.meshgrid(*([c] * dim), indexing="ij")
    return np.stack([a.reshape(-1, order="F") for a in axes], axis=1)


def rhs(seed, n, nrhs):
    """n x nrhs right-hand sides with N(0,1) entries, column j = draws j*n..(j+1)*n-1."""
    return np.asfortranarray(normal(seed, n * nrhs).reshape(nrhs, n).T)
