"""The Chebyshev interval, pinned to dense eigenvalues on both sides.

The interval handed to the Chebyshev iteration is the extreme eigenvalues of the
grid operator (eqs. eigenvaluesPoissonDirichletMatrix, lambdaMin, lambdaMax; the
matrix N of eq. matrix_neuman along an axis with a Neumann face). BJ(CI) uses the
spectra of the diagonal blocks R_s A R_s^T of eq. blockJacobiPreconditioner,
GNoComm(CI) the global interval (Methodology section), and the optional factors
multiply the two ends (Experimental Setup).

Here both the library's host-side interval (poisson_cheb_interval, no GPU) and
the oracle's orc_cheb_interval are compared with eigenvalues of matrices that
numpy assembles on its own: Kronecker sums of the 1D matrices, with every
coupling between different blocks deleted for BJ(CI). The closed forms never
enter the reference side.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_2503_08935_amd as P


def axis_matrix(n, neu_lo, neu_hi):
    """1D second-difference matrix: D, or N with the corner entry -2 at a Neumann end."""
    m = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    if neu_lo and n > 1:
        m[0, 1] = -2
    if neu_hi and n > 1:
        m[-1, -2] = -2
    return m


def grid_matrix(shape, h, bc):
    nx, ny, nz = shape
    ax = [axis_matrix(nx, bc & 1, bc & 2), axis_matrix(ny, bc & 4, bc & 8),
          axis_matrix(nz, bc & 16, bc & 32)]
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, ax[0])) + np.kron(Iz, np.kron(ax[1], Ix)) +
            np.kron(ax[2], np.kron(Iy, Ix))) / (h * h)


def block_ids(shape, bs):
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((k // bs) * 1_000_000 + (j // bs) * 1000 + i // bs).ravel()


def real_eigs(m):
    if np.array_equal(m, m.T):
        return np.linalg.eigvalsh(m)
    ev = np.linalg.eigvals(m)
    assert np.abs(ev.imag).max() <= 1e-9 * np.abs(ev).max()  # N is similar to a symmetric matrix
    return np.sort(ev.real)


def dense_global(shape, h, bc):
    ev = real_eigs(grid_matrix(shape, h, bc))
    return ev[0], ev[-1]


def dense_blocks(shape, h, bc, bs):
    """Extreme eigenvalues over all diagonal blocks R_s A R_s^T."""
    A = grid_matrix(shape, h, bc)
    ids = block_ids(shape, bs)
    lo, hi = np.inf, -np.inf
    for b in np.unique(ids):
        sel = ids == b
        ev = real_eigs(A[np.ix_(sel, sel)])
        lo, hi = min(lo, ev[0]), max(hi, ev[-1])
    return lo, hi


def full_block_extent(n, bs):
    """An axis longer than a block, grown to whole blocks (a clipped last block is
    bounded by the full-length block of the same kind); a shorter axis is one block."""
    return n if n <= bs else -(-n // bs) * bs


def close(a, b, scale):
    return abs(a - b) <= 1e-11 * scale


def library_interval(shape, h, bc, pc, **opts):
    with P.Solver(shape, h, bc=bc, **opts) as s:
        return s.cheb_interval(pc)


def oracle_interval(shape, h, bc, pc, block=64, bj_global=0, lmin_scale=1.0, lmax_scale=1.0):
    return oracle.cheb_interval(shape, h, pc, block=block, bj_global=bj_global,
                                lmin_scale=lmin_scale, lmax_scale=lmax_scale, bc=bc)


MASKS = [0, 1, 2, 22, 3 | 12, 48, 42, 1 | 8 | 32]
SHAPES = [(6, 5, 7), (8, 3, 4), (2, 6, 5)]


@pytest.mark.parametrize("bc", MASKS)
@pytest.mark.parametrize("shape", SHAPES)
def test_global_interval_is_dense_spectrum(shape, bc):
    h = 0.3
    lo, hi = dense_global(shape, h, bc)
    for got in (library_interval(shape, h, bc, P.PC_CHEBYSHEV),
                oracle_interval(shape, h, bc, oracle.PC_CHEBYSHEV)):
        assert close(got[0], lo, hi) and close(got[1], hi, hi), (got, lo, hi)


@pytest.mark.parametrize("bc", MASKS)
@pytest.mark.parametrize("shape,bs", [((8, 8, 4), 4), ((9, 6, 6), 3), ((6, 9, 3), 3),
                                      ((12, 4, 8), 4)])
def test_block_interval_is_block_spectrum(shape, bs, bc):
    """Every axis a whole number of blocks: the interval is exactly the extreme
    eigenvalues over the diagonal blocks."""
    h = 0.25
    lo, hi = dense_blocks(shape, h, bc, bs)
    g = dense_global(shape, h, bc)
    assert lo > g[0] * (1 + 1e-9)  # dropping the couplings moves the bottom up
    for got in (library_interval(shape, h, bc, P.PC_BLOCK_JACOBI, block=bs),
                oracle_interval(shape, h, bc, oracle.PC_BLOCK_JACOBI, block=bs)):
        assert close(got[0], lo, hi) and close(got[1], hi, hi), (got, lo, hi)


@pytest.mark.parametrize("bc", [0, 22, 2 | 8, 3])
@pytest.mark.parametrize("shape,bs", [((9, 7, 8), 3), ((7, 5, 10), 4), ((5, 11, 3), 4)])
def test_clipped_blocks(shape, bs, bc):
    """Clipped edge blocks: the interval contains every block's spectrum and is
    the spectrum of the grid grown to whole blocks (full-length block kinds)."""
    h = 0.25
    lo_c, hi_c = dense_blocks(shape, h, bc, bs)
    grown = tuple(full_block_extent(n, bs) for n in shape)
    lo, hi = dense_blocks(grown, h, bc, bs)
    for got in (library_interval(shape, h, bc, P.PC_BLOCK_JACOBI, block=bs),
                oracle_interval(shape, h, bc, oracle.PC_BLOCK_JACOBI, block=bs)):
        assert got[0] <= lo_c * (1 + 1e-11) and got[1] >= hi_c * (1 - 1e-11)
        assert close(got[0], lo, hi) and close(got[1], hi, hi), (got, lo, hi)


@pytest.mark.parametrize("bc", [0, 22, 3 | 12])
def test_gnocomm_takes_the_global_interval(bc):
    shape, bs, h = (8, 8, 4), 4, 0.2
    lo, hi = dense_global(shape, h, bc)
    blo, bhi = dense_blocks(shape, h, bc, bs)
    assert blo > lo * 1.01  # the two readings are far apart here
    for got in (library_interval(shape, h, bc, P.PC_BLOCK_JACOBI, block=bs,
                                 bj_global_interval=1),
                oracle_interval(shape, h, bc, oracle.PC_BLOCK_JACOBI, block=bs, bj_global=1)):
        assert close(got[0], lo, hi) and close(got[1], hi, hi), (got, lo, hi)


@pytest.mark.parametrize("pc,bj_global", [(P.PC_CHEBYSHEV, 0), (P.PC_BLOCK_JACOBI, 0),
                                          (P.PC_BLOCK_JACOBI, 1)])
@pytest.mark.parametrize("smin,smax", [(5.0, 1 - 1e-4), (2.0, 1.0), (0.5, 3.0)])
def test_rescaling_multiplies_the_ends(pc, bj_global, smin, smax):
    shape, bs, h, bc = (9, 6, 8), 3, 0.2, 22
    base_l = library_interval(shape, h, bc, pc, block=bs, bj_global_interval=bj_global)
    base_o = oracle_interval(shape, h, bc, pc, block=bs, bj_global=bj_global)
    got_l = library_interval(shape, h, bc, pc, block=bs, bj_global_interval=bj_global,
                             lmin_scale=smin, lmax_scale=smax)
    got_o = oracle_interval(shape, h, bc, pc, block=bs, bj_global=bj_global, lmin_scale=smin,
                            lmax_scale=smax)
    for base, got in ((base_l, got_l), (base_o, got_o)):
        assert got[0] == base[0] * smin and got[1] == base[1] * smax


def test_library_and_oracle_agree_bitwise():
    """The solve's trajectories can only agree bit for bit if the interval does;
    both sides evaluate the same closed forms of the paper in FP64."""
    shapes = [(1, 1, 3), (2, 2, 2), (7, 5, 3), (64, 64, 64), (70, 19, 13), (255, 255, 255),
              (512, 512, 512), (100, 300, 130), (129, 65, 200)]
    for shape, bc, bs, glob in itertools.product(shapes, [0, 1, 22, 3 | 12, 2 | 8 | 32],
                                                 [3, 16, 64], [0, 1]):
        if any(((bc >> (2 * d)) & 3) and shape[d] < 2 for d in range(3)):
            continue
        h = 1.0 / (shape[0] + 1)
        for pc in (P.PC_CHEBYSHEV, P.PC_BLOCK_JACOBI):
            try:
                lib = library_interval(shape, h, bc, pc, block=bs, bj_global_interval=glob)
            except P.PoissonError:
                lib = None  # degenerate interval (single point)
            orc = oracle_interval(shape, h, bc, pc, block=bs, bj_global=glob)
            if lib is None:
                assert not (0 < orc[0] < orc[1])
            else:
                assert lib == orc, (shape, bc, bs, glob, pc, lib, orc)


def test_degenerate_and_invalid_queries():
    with P.Solver((1, 1, 1), 0.5) as s:
        with pytest.raises(P.PoissonError):
            s.cheb_interval(P.PC_CHEBYSHEV)
    with P.Solver((4, 4, 4), 0.2) as s:
        with pytest.raises(P.PoissonError):
            s.cheb_interval(P.PC_JACOBI)
        lo, hi = s.cheb_interval(P.PC_CHEBYSHEV)
        assert 0 < lo < hi
