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


# The test problem of the paper's Experimental Setup: -lap(phi) = sin x + cos y +
# 3 sin z - 2yz + 2 on [3, 28.5] x [2.5, 28] x [10, 35.5] with spacing 0.1 (256
# nodes per axis including the boundary), Dirichlet on x-, y+, z+ and Neumann on
# x+, y-, z-. The boundary values are not given in the paper; here they are
# homogeneous. Unknowns: a Dirichlet boundary node is not an unknown, a Neumann
# one is, so every axis has 255 unknowns.
PAPER_BC = 2 | 4 | 16          # Neumann on x+, y-, z- (bit f = face x-, x+, y-, y+, z-, z+)
PAPER_H = 0.1


def paper_problem():
    """(f, shape, h, bc) of the paper's test problem on 255^3 unknowns."""
    n = 255
    x = 3.0 + (np.arange(n) + 1) * PAPER_H      # x- Dirichlet node excluded, x+ included
    y = 2.5 + np.arange(n) * PAPER_H            # y- Neumann node included, y+ excluded
    z = 10.0 + np.arange(n) * PAPER_H           # z- Neumann node included, z+ excluded
    f = (np.sin(x)[None, None, :] + np.cos(y)[None, :, None] + 3.0 * np.sin(z)[:, None, None]
         - 2.0 * y[None, :, None] * z[:, None, None] + 2.0)
    return np.ascontiguousarray(f), (n, n, n), PAPER_H, PAPER_BC
