"""Seeded synthetic inputs for the Poisson workloads (host side, numpy).

This module generates right-hand sides only; it holds none of the solver's
arithmetic. Both the oracle-based tests and the GPU benchmarks draw their
inputs from here, so the two sides see the same bits.

Generators
----------
* ``uniform(seed, n)``: f = 2u - 1 with u = (splitmix64(key(seed) + (i+1)*G) >> 11) * 2^-53,
  i the linear (x-fastest) index. splitmix64 is the finaliser of Steele, Lea and
  Flood, "Fast splittable pseudorandom number generators" (OOPSLA 2014);
  G = 0x9E3779B97F4A7C15 and key(seed) = splitmix64(seed). The GPU library
  implements the same published generator for on-device request generation.
* ``gaussian(seed, n)``: Box-Muller on the uniforms of indices 2i and 2i+1 (host only).
* ``manufactured(shape)``: f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) on the unit
  cube, node (i, j, k) at ((i+1)h, (j+1)h, (k+1)h), h = 1/(n+1); its continuous
  solution is u = sin(pi x) sin(pi y) sin(pi z).

Arrays are shaped (nz, ny, nx) so that C order is x-fastest.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def key(seed):
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed) + GAMMA)


def uniform_bits(seed, start, count):
    idx = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key(seed) + (idx + np.uint64(1)) * GAMMA)


def uniform(seed, n, start=0):
    """n values of f ~ U[-1, 1) (exact multiples of 2^-52)."""
    u = (uniform_bits(seed, start, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def uniform_grid(seed, shape):
    nx, ny, nz = shape
    return uniform(seed, nx * ny * nz).reshape(nz, ny, nx)


def gaussian(seed, n):
    bits = uniform_bits(seed, 0, 2 * n)
    u = (bits >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u1, u2 = u[0::2], u[1::2]
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def nodes(n):
    h = 1.0 / (n + 1)
    return (np.arange(n) + 1) * h


def manufactured_u(shape):
    nx, ny, nz = shape
    sx, sy, sz = (np.sin(np.pi * nodes(n)) for n in (nx, ny, nz))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def manufactured(shape):
    return 3.0 * np.pi ** 2 * manufactured_u(shape)


def manufactured_noisy(shape, seed, sigma=1e-3):
    nx, ny, nz = shape
    return manufactured(shape) + sigma * gaussian(seed, nx * ny * nz).reshape(nz, ny, nx)


def spacing(n):
    """Interior-unknown convention on the unit cube: h = 1/(n+1)."""
    return 1.0 / (n + 1)
