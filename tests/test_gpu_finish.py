"""The finish of a solve (the true residual and the statistics), checked against
values the host computes on its own from the returned x.

The stopping test of Alg. 1 uses the recursively updated residual; the solver
then reports ||b - A x|| / ||b|| recomputed from x (Experimental Setup: the
tolerances are relative). Here the host recomputes that quotient from the GPU's
x with the oracle's operator and exact dot products, and requires the reported
value to be the same double: the GPU applies the same operator in the same
order, and its double-double sum equals the exact sum rounded once away from
rounding ties. The recursive residual and the history must follow the oracle's
trajectory of r.r, and the interval the Chebyshev iteration used must be the
extreme eigenvalues of densely assembled matrices (global, Block-Jacobi blocks,
GNoComm(CI), rescaled)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads
from test_interval import dense_blocks, dense_global, full_block_extent

pytestmark = pytest.mark.gpu

OPC = {P.PC_NONE: oracle.PC_NONE, P.PC_JACOBI: oracle.PC_JACOBI,
       P.PC_CHEBYSHEV: oracle.PC_CHEBYSHEV, P.PC_BLOCK_JACOBI: oracle.PC_BLOCK_JACOBI}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host_relres(f, x, h, bc):
    """||b - A x||_2 / ||b||_2 from x alone: the oracle's operator, exact dots."""
    r = f - oracle.apply_A(x.reshape(f.shape), h, bc=bc)
    bb = oracle.dot(f, f)
    return math.sqrt(oracle.dot(r, r) / bb), bb


CASES = [
    # shape, bc, pc, degree, mixed, block, tol, maxit, x0 seed
    ((61, 47, 35), 0, P.PC_CHEBYSHEV, 8, False, 64, 1e-8, 5000, None),
    ((61, 47, 35), 0, P.PC_CHEBYSHEV, 8, True, 64, 1e-8, 5000, None),
    ((40, 21, 18), 22, P.PC_CHEBYSHEV, 4, False, 64, 1e-9, 5000, None),
    ((37, 30, 26), 1 | 8 | 32, P.PC_BLOCK_JACOBI, 5, True, 16, 1e-8, 5000, None),
    ((70, 19, 13), 0, P.PC_BLOCK_JACOBI, 6, False, 7, 1e-8, 5000, 5),
    ((33, 21, 50), 0, P.PC_NONE, 0, False, 64, 1e-8, 5000, None),
    ((33, 21, 50), 0, P.PC_JACOBI, 0, True, 64, 1e-10, 5000, None),
    ((129, 40, 24), 2 | 4, P.PC_CHEBYSHEV, 7, False, 64, 1e-12, 9, 3),  # NOT_CONVERGED
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-bc{c[1]}-pc{c[2]}-m{c[3]}"
                         f"-{'mixed' if c[4] else 'fp64'}-it{c[7]}")
def test_true_residual_and_stats_match_host(gpu, case):
    shape, bc, pc, m, mixed, block, tol, maxit, x0seed = case
    h = 1.0 / (shape[0] + 1)
    f = workloads.uniform_grid(50 + bc, shape)
    x0 = workloads.uniform_grid(x0seed, shape) if x0seed is not None else np.zeros_like(f)
    with P.Solver(shape, h, bc=bc, precision=P.MIXED if mixed else P.FP64, block=block) as s:
        x = dev(x0)
        st = s.solve(dev(f), x, pc, m, tol, maxit)
        torch.cuda.synchronize()
        stats, tr = s.stats(), s.trace()
        xg = x.cpu().numpy().reshape(f.shape)
    ref = oracle.bicgstab(f, h, pc=OPC[pc], degree=m, mixed=mixed, tol=tol, maxit=maxit,
                          x0=x0, block=block, bc=bc)
    assert st == ref.status and stats["iterations"] == ref.iterations
    assert np.array_equal(xg, ref.x)
    relres, bb = host_relres(f, xg, h, bc)
    assert stats["relres_true"] == relres, (stats["relres_true"], relres)
    # the recursive residual is the last r.r (s.s at a half-step exit) of the trajectory
    its = ref.iterations
    assert stats["relres_recursive"] == math.sqrt(ref.rr[its - 1] / bb)
    hist = stats["history"]
    assert len(hist) == its + 1
    assert hist[0] == math.sqrt(ref.rr0 / bb)
    assert hist[1:] == [math.sqrt(v / bb) for v in ref.rr]
    assert np.array_equal(tr[:, 3], ref.rr)
    if st == P.OK:
        assert relres < 1.2 * tol


def test_true_residual_is_not_the_recursive_one(gpu):
    """A solve stopped after 3 iterations from a far-off x0: the true residual of the
    returned x equals the host's recomputation, whatever the recursion says."""
    shape, h = (50, 40, 30), 1.0 / 51
    f = workloads.uniform_grid(61, shape)
    x0 = 1e3 * workloads.uniform_grid(62, shape)
    with P.Solver(shape, h) as s:
        x = dev(x0)
        st = s.solve(dev(f), x, P.PC_CHEBYSHEV, 3, 1e-12, 3)
        torch.cuda.synchronize()
        stats = s.stats()
        xg = x.cpu().numpy().reshape(f.shape)
    assert st == P.NOT_CONVERGED
    relres, _ = host_relres(f, xg, h, 0)
    assert stats["relres_true"] == relres and relres > 1e-6


INTERVALS = [
    # shape, bc, pc, block, bj_global, lmin_scale, lmax_scale
    ((6, 5, 7), 0, P.PC_CHEBYSHEV, 64, 0, 1.0, 1.0),
    ((6, 5, 7), 1, P.PC_CHEBYSHEV, 64, 0, 1.0, 1.0),
    ((8, 3, 4), 22, P.PC_CHEBYSHEV, 64, 0, 1.0, 1.0),
    ((6, 5, 7), 3 | 12, P.PC_CHEBYSHEV, 64, 0, 1.0, 1.0),
    ((8, 8, 4), 0, P.PC_BLOCK_JACOBI, 4, 0, 1.0, 1.0),
    ((9, 6, 6), 22, P.PC_BLOCK_JACOBI, 3, 0, 1.0, 1.0),
    ((9, 7, 8), 0, P.PC_BLOCK_JACOBI, 3, 0, 1.0, 1.0),      # clipped edge blocks
    ((7, 5, 10), 22, P.PC_BLOCK_JACOBI, 4, 0, 1.0, 1.0),    # clipped, Neumann faces
    ((8, 8, 4), 3 | 12, P.PC_BLOCK_JACOBI, 4, 1, 1.0, 1.0),  # GNoComm(CI)
    ((9, 6, 8), 22, P.PC_BLOCK_JACOBI, 3, 1, 10.0, 1 - 1e-4),
    ((9, 6, 8), 1, P.PC_BLOCK_JACOBI, 3, 0, 2.0, 1.0),
    ((6, 5, 7), 0, P.PC_CHEBYSHEV, 64, 0, 10.0, 1 - 1e-4),
]


@pytest.mark.parametrize("case", INTERVALS, ids=lambda c: f"{c[0]}-bc{c[1]}-pc{c[2]}-b{c[3]}"
                         f"-g{c[4]}-s{c[5]}")
def test_solve_reports_dense_interval(gpu, case):
    """lambda_min / lambda_max of the stats after a solve: the dense spectrum of the
    grid matrix (G(CI), GNoComm(CI)) or the extreme eigenvalues over the diagonal
    blocks (BJ(CI); a clipped block is bounded by its whole-block kind), each end
    multiplied by its factor."""
    shape, bc, pc, block, glob, smin, smax = case
    h = 0.25
    if pc == P.PC_CHEBYSHEV or glob:
        lo, hi = dense_global(shape, h, bc)
    else:
        grown = tuple(full_block_extent(n, block) for n in shape)
        lo, hi = dense_blocks(grown, h, bc, block)
    f = workloads.uniform_grid(70, shape)
    with P.Solver(shape, h, bc=bc, block=block, bj_global_interval=glob, lmin_scale=smin,
                  lmax_scale=smax) as s:
        x = torch.zeros(f.size, dtype=torch.float64, device="cuda:0")
        st = s.solve(dev(f), x, pc, 4, 1e-8, 2)
        torch.cuda.synchronize()
        stats = s.stats()
    assert st in (P.OK, P.NOT_CONVERGED)
    assert abs(stats["lambda_min"] - smin * lo) <= 1e-11 * hi, (stats["lambda_min"], smin * lo)
    assert abs(stats["lambda_max"] - smax * hi) <= 1e-11 * hi, (stats["lambda_max"], smax * hi)
