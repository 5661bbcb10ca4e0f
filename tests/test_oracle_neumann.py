"""Pins for the oracle's Neumann and mixed boundary conditions.

Eq. matrix_neuman: a Neumann end of an axis replaces the first (last) row of D
by (2, -2) ((-2, 2)). The operator is checked against a dense Kronecker
assembly of those matrices, the interval against dense (non-symmetric)
eigenvalues, and the one-sided closed form through its cosine eigenvectors."""
import itertools

import numpy as np
import pytest

import oracle
from tests.test_oracle_chebyshev import q as cheb_q

PAPER_BC = 2 | 4 | 16  # Neumann on x+, y-, z-; Dirichlet on x-, y+, z+ (Experimental Setup)


def O(n, neu_lo, neu_hi):
    m = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    if neu_lo and n > 1:
        m[0, 1] = -2
    if neu_hi and n > 1:
        m[-1, -2] = -2
    return m


def dense(shape, h, bc):
    nx, ny, nz = shape
    ox = O(nx, bc & 1, bc & 2)
    oy = O(ny, bc & 4, bc & 8)
    oz = O(nz, bc & 16, bc & 32)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, ox)) + np.kron(Iz, np.kron(oy, Ix)) +
            np.kron(oz, np.kron(Iy, Ix))) / h ** 2


@pytest.mark.parametrize("bc", range(64))
def test_operator_matches_dense_all_face_combinations(bc):
    shape = (5, 4, 6)
    h = 0.3
    rng = np.random.default_rng(bc)
    u = rng.standard_normal((6, 4, 5))
    ref = dense(shape, h, bc) @ u.ravel()
    got = oracle.apply_A(u, h, bc=bc).ravel()
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("bc", [1, 2, 3, 5, 12, 22, 42, 21, 63 - 3])
@pytest.mark.parametrize("shape", [(6, 5, 7), (8, 3, 4)])
def test_interval_matches_dense_eigenvalues(bc, shape):
    h = 0.2
    ev = np.linalg.eigvals(dense(shape, h, bc))
    assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max()  # N is similar to a symmetric matrix
    ev = np.sort(ev.real)
    lo, hi = oracle.interval(shape, h, bc=bc)
    assert abs(lo - ev[0]) <= 1e-10 * ev[-1] and abs(hi - ev[-1]) <= 1e-10 * ev[-1]


def test_block_interval_contains_every_block_with_neumann_faces():
    shape, bs, h = (9, 7, 8), 3, 0.25
    for bc in (PAPER_BC, 3, 48, 1 | 8 | 32):
        P = dense(shape, h, bc)
        lo, hi = oracle.interval(shape, h, block=bs, bc=bc)
        nx, ny, nz = shape
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ids = ((k // bs) * 10000 + (j // bs) * 100 + i // bs).ravel()
        for b in np.unique(ids):
            sel = ids == b
            e = np.sort(np.linalg.eigvals(P[np.ix_(sel, sel)]).real)
            assert e[0] >= lo * (1 - 1e-10) and e[-1] <= hi * (1 + 1e-10)


def axis_mode(n, k, neu_lo, neu_hi):
    """Eigenvector and eigenvalue of one axis (one-sided closed forms)."""
    j = np.arange(n)
    if not neu_lo and not neu_hi:
        return np.sin(k * np.pi * (j + 1) / (n + 1)), 4 * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    th = (2 * k - 1) * np.pi / (2 * n)
    v = np.cos(th * j) if neu_lo else np.cos(th * (n - 1 - j))
    return v, 4 * np.sin(th / 2) ** 2


@pytest.mark.parametrize("ks", [(1, 1, 1), (2, 3, 1), (4, 2, 5)])
def test_mixed_bc_modes_are_eigenvectors_and_chebyshev_closed_form(ks):
    shape = (12, 10, 9)
    h = 0.07
    bc = PAPER_BC
    flags = [(bc & 1, bc & 2), (bc & 4, bc & 8), (bc & 16, bc & 32)]
    vs, lam = [], 0.0
    for n, k, (a, b) in zip(shape, ks, flags):
        v, l = axis_mode(n, k, a, b)
        vs.append(v)
        lam += l / h ** 2
    u = vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :]
    assert np.abs(oracle.apply_A(u, h, bc=bc) - lam * u).max() <= 1e-12 * lam
    lo, hi = oracle.interval(shape, h, bc=bc)
    for m in (0, 1, 3, 6):
        got = oracle.chebyshev(u, h, lo, hi, m, bc=bc)
        ref = cheb_q(lam, lo, hi, m) * u
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("bc", [PAPER_BC, 1, 2 | 8 | 32, 3])
@pytest.mark.parametrize("pc,m,mixed", [(oracle.PC_NONE, 0, False), (oracle.PC_CHEBYSHEV, 4, False),
                                        (oracle.PC_BLOCK_JACOBI, 3, False),
                                        (oracle.PC_CHEBYSHEV, 4, True)])
def test_bicgstab_matches_dense_with_neumann(bc, pc, m, mixed):
    shape = (7, 6, 5)
    h = 0.15
    rng = np.random.default_rng(bc + m)
    b = rng.uniform(-1, 1, (5, 6, 7))
    P = dense(shape, h, bc)
    xd = np.linalg.solve(P, b.ravel())
    r = oracle.bicgstab(b, h, pc=pc, degree=m, mixed=mixed, tol=1e-12, maxit=2000, block=3,
                        bc=bc)
    assert r.status == oracle.OK
    assert np.linalg.norm(r.x.ravel() - xd) <= 1e-8 * np.linalg.norm(xd)


def test_dirichlet_path_unchanged_by_bc_argument():
    shape = (10, 9, 8)
    h = 0.1
    b = np.random.default_rng(1).uniform(-1, 1, (8, 9, 10))
    a = oracle.bicgstab(b, h, pc=oracle.PC_CHEBYSHEV, degree=4, tol=1e-10)
    c = oracle.bicgstab(b, h, pc=oracle.PC_CHEBYSHEV, degree=4, tol=1e-10, bc=0)
    assert np.array_equal(a.x, c.x)
    assert oracle.interval(shape, h) == oracle.interval(shape, h, bc=0)


@pytest.mark.parametrize("bc", [PAPER_BC, 1 | 8 | 32, 3, 63])
def test_block_operator_with_neumann_faces_is_block_diagonal_part(bc):
    # y has a last block one plane thick: its mirror neighbour lies in the previous block
    shape, bs, h = (9, 7, 8), 3, 0.25
    nx, ny, nz = shape
    P = dense(shape, h, bc)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ids = ((k // bs) * 10000 + (j // bs) * 100 + i // bs).ravel()
    Pb = np.where(ids[:, None] == ids[None, :], P, 0.0)
    u = np.random.default_rng(bc).standard_normal((nz, ny, nx))
    got = oracle.apply_A(u, h, block=bs, bc=bc).ravel()
    assert np.allclose(got, Pb @ u.ravel(), rtol=0, atol=1e-13 * np.abs(got).max())
