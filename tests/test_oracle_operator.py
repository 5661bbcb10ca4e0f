"""Pins for the oracle's grid operator and eigenvalue interval.

The operator is eq. matrix_p (Background section) with the Dirichlet matrix D of
eq. matrix_dirichlet on every axis; the interval is eqs. lambdaMin/lambdaMax with
the eigenvalues of eq. eigenvaluesPoissonDirichletMatrix. Pins: a dense
Kronecker-product assembly built here with numpy, dense eigenvalues, discrete
sine modes and exactness on tensor quadratics."""
import numpy as np
import pytest

import oracle


def D(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def dense_P(shape, h):
    nx, ny, nz = shape
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, D(nx))) + np.kron(Iz, np.kron(D(ny), Ix)) +
            np.kron(D(nz), np.kron(Iy, Ix))) / h ** 2


def block_ids(shape, bs):
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((k // bs) * 10000 + (j // bs) * 100 + i // bs).ravel()


SHAPES = [(1, 1, 1), (2, 3, 4), (5, 7, 6), (8, 3, 5), (6, 6, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("h", [0.1, 0.37])
def test_apply_matches_dense_kronecker(shape, h):
    rng = np.random.default_rng(hash(shape) % 1000)
    nx, ny, nz = shape
    u = rng.standard_normal((nz, ny, nx))
    ref = dense_P(shape, h) @ u.ravel()
    got = oracle.apply_A(u, h).ravel()
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("shape,bs", [((5, 7, 6), 3), ((8, 8, 4), 4), ((6, 5, 7), 2)])
def test_block_apply_is_block_diagonal_part(shape, bs):
    rng = np.random.default_rng(3)
    nx, ny, nz = shape
    h = 0.2
    P = dense_P(shape, h)
    ids = block_ids(shape, bs)
    Pb = np.where(ids[:, None] == ids[None, :], P, 0.0)
    u = rng.standard_normal((nz, ny, nx))
    got = oracle.apply_A(u, h, block=bs).ravel()
    assert np.allclose(got, Pb @ u.ravel(), rtol=0, atol=1e-13 * np.abs(got).max())
    # and it differs from the global operator when blocks exist
    assert not np.allclose(got, P @ u.ravel())


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 7, 6), (8, 8, 8), (7, 1, 3)])
def test_interval_matches_dense_eigenvalues(shape):
    h = 0.25
    ev = np.linalg.eigvalsh(dense_P(shape, h))
    lo, hi = oracle.interval(shape, h)
    assert abs(lo - ev[0]) <= 1e-11 * ev[-1]
    assert abs(hi - ev[-1]) <= 1e-11 * ev[-1]


@pytest.mark.parametrize("shape,bs", [((8, 8, 8), 4), ((7, 5, 6), 3), ((9, 2, 9), 4)])
def test_block_interval_is_one_block_spectrum(shape, bs):
    h = 0.5
    bshape = tuple(min(n, bs) for n in shape)
    ev = np.linalg.eigvalsh(dense_P(bshape, h))
    lo, hi = oracle.interval(shape, h, block=bs)
    assert abs(lo - ev[0]) <= 1e-11 * ev[-1] and abs(hi - ev[-1]) <= 1e-11 * ev[-1]
    # every block, including clipped edge blocks, has its spectrum inside
    P = dense_P(shape, h)
    ids = block_ids(shape, bs)
    for b in np.unique(ids):
        sel = ids == b
        e = np.linalg.eigvalsh(P[np.ix_(sel, sel)])
        assert e[0] >= lo * (1 - 1e-12) and e[-1] <= hi * (1 + 1e-12)


def test_dirichlet_eigs_match_dense():
    for n in (1, 2, 5, 9):
        ev = np.linalg.eigvalsh(D(n))
        got = [oracle.dirichlet_eig(i, n) for i in range(1, n + 1)]
        assert np.allclose(got, ev, rtol=1e-13, atol=1e-14)


def sine_mode(shape, ks):
    nx, ny, nz = shape
    f = [np.sin(k * np.pi * (np.arange(n) + 1) / (n + 1)) for k, n in zip(ks, shape)]
    return f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]


@pytest.mark.parametrize("shape,ks", [((17, 12, 9), (1, 1, 1)), ((17, 12, 9), (3, 5, 2)),
                                      ((33, 33, 33), (1, 2, 33)), ((40, 31, 29), (40, 31, 29))])
def test_sine_modes_are_eigenvectors(shape, ks):
    """Textbook closed form of the discrete Dirichlet Laplacian's eigenpairs."""
    h = 0.03
    u = sine_mode(shape, ks)
    lam = sum(4 * np.sin(k * np.pi / (2 * (n + 1))) ** 2 for k, n in zip(ks, shape)) / h ** 2
    got = oracle.apply_A(u, h)
    assert np.abs(got - lam * u).max() <= 2e-14 * lam


def test_tensor_quadratic_is_exact():
    """u = x(1-x)y(1-y)z(1-z): second differences of quadratics are exact."""
    n = 20
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1) * h
    q = t * (1 - t)
    u = q[:, None, None] * q[None, :, None] * q[None, None, :]
    f = 2 * (q[None, :, None] * q[None, None, :] + q[:, None, None] * q[None, None, :] +
             q[:, None, None] * q[None, :, None]) * np.ones((n, n, n))
    got = oracle.apply_A(u, h)
    assert np.abs(got - f).max() <= 1e-12 * np.abs(f).max()
