"""Four Chebyshev steps per pass (the LDS-staged k_cheb_steps_lds with S = 4: in
the mixed mode POISSON_OPT_FUSE = 3, the default, in FP64 as well with 4): the
same arithmetic per point as one step per pass (Alg. 2's loop body), so every
preconditioner apply and every solve must give the bits of the plan with two
steps per pass and of the oracle (its FP32 emulation in the mixed mode),
whatever the tile raggedness, face types, block masks and degree (the apply's
steps split into a first four-step pass and then fours, triples, pairs or a
single step)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu

CONFIGS = [
    dict(bc=0, pc=P.PC_CHEBYSHEV, block=64),            # select-free body
    dict(bc=2 | 4 | 16, pc=P.PC_CHEBYSHEV, block=64),   # the paper's faces: mirror selects
    dict(bc=1 | 32, pc=P.PC_CHEBYSHEV, block=64),
    dict(bc=0, pc=P.PC_BLOCK_JACOBI, block=16),         # block faces inside and at tile edges
    dict(bc=2 | 8 | 16, pc=P.PC_BLOCK_JACOBI, block=7),  # mask and mirror together
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda:0")


@pytest.mark.parametrize("mixed", [True, False], ids=["mixed", "fp64"])
@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"bc{c['bc']}-pc{c['pc']}-b{c['block']}")
@pytest.mark.parametrize("shape", [(200, 37, 21), (64, 32, 8), (66, 70, 19), (3, 50, 2),
                                   (257, 33, 9), (1, 1, 5), (70, 17, 40)])
def test_fours_match_pairs_and_oracle(gpu, cfg, shape, mixed):
    """Ragged x, y and z tails, a tile with grid rows on both sides, waves between
    the top and bottom one partly or wholly outside the grid, one-point axes;
    degree 4 (one pass writing w_4 only), 5-7 (a single step, pair or triple
    after the first four), 8 (two fours) and 9-11."""
    nx, ny, nz = shape
    bc, pc, block = cfg["bc"], cfg["pc"], cfg["block"]
    for axis, n in enumerate(shape):
        if bc >> (2 * axis) & 3 and n < 2:
            pytest.skip("a Neumann face needs two points on its axis")
    h = 1.0 / (nx + 1)
    v = workloads.uniform_grid(12, shape)
    dt = torch.float32 if mixed else torch.float64
    for m in (4, 5, 6, 7, 8, 9, 10, 11):
        got = []
        for fuse in ((3, 1) if mixed else (4, 1)):
            with P.Solver(shape, h, bc=bc, block=block, fuse=fuse,
                          precision=P.MIXED if mixed else P.FP64) as s:
                out = torch.empty(v.size, dtype=dt, device="cuda:0")
                s.apply_precond(pc, m, dev(v), out)
                got.append(out.cpu().numpy().astype(np.float64))
        assert np.array_equal(got[0], got[1]), m
        ref = oracle.precond(v, h, pc, degree=m, mixed=mixed, block=block, bc=bc)
        assert np.array_equal(got[0], ref.ravel()), m


@pytest.mark.parametrize("shape,pc,m,bc,block,fold,mixed", [
    ((70, 19, 13), P.PC_CHEBYSHEV, 8, 0, None, 1, True),
    ((70, 19, 13), P.PC_CHEBYSHEV, 4, 0, None, 1, True),
    ((70, 19, 13), P.PC_CHEBYSHEV, 4, 0, None, 0, True),
    ((48, 33, 35), P.PC_BLOCK_JACOBI, 7, 0, 16, 1, True),
    ((40, 21, 18), P.PC_CHEBYSHEV, 6, 22, None, 1, True),
    ((131, 45, 70), P.PC_CHEBYSHEV, 8, 0, None, 1, True),
    ((131, 45, 70), P.PC_CHEBYSHEV, 9, 0, None, 0, True),
    ((70, 19, 13), P.PC_CHEBYSHEV, 8, 0, None, 1, False),
    ((70, 19, 13), P.PC_CHEBYSHEV, 4, 0, None, 1, False),
    ((70, 19, 13), P.PC_CHEBYSHEV, 4, 0, None, 0, False),
    ((48, 33, 35), P.PC_BLOCK_JACOBI, 7, 0, 16, 1, False),
    ((40, 21, 18), P.PC_CHEBYSHEV, 6, 22, None, 1, False),
    ((131, 45, 70), P.PC_CHEBYSHEV, 8, 0, None, 1, False),
    ((131, 45, 70), P.PC_CHEBYSHEV, 10, 0, None, 0, False),
])
def test_solves_with_fours(gpu, shape, pc, m, bc, block, fold, mixed):
    """Full solves with four steps per pass, the s and p updates folded into the
    first four-step pass or standalone: iterations, trajectory and x bitwise
    those of two steps per pass and of the oracle."""
    h = workloads.spacing(shape[0])
    f = workloads.uniform_grid(40 + m, shape)
    res = []
    for fuse in ((3, 1) if mixed else (4, 1)):
        o = dict(precision=P.MIXED if mixed else P.FP64, fuse=fuse, fuse_updates=fold)
        if block:
            o["block"] = block
        with P.Solver(shape, h, bc=bc, **o) as s:
            b = dev(f)
            x = torch.zeros_like(b)
            st = s.solve(b, x, pc, m, 1e-9, 2000)
            torch.cuda.synchronize()
            res.append((st, s.stats()["iterations"], s.trace(), x.cpu().numpy()))
    a, b = res
    assert a[0] == b[0] == P.OK and a[1] == b[1] > 2
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    ref = oracle.bicgstab(f, h, pc={P.PC_CHEBYSHEV: oracle.PC_CHEBYSHEV,
                                    P.PC_BLOCK_JACOBI: oracle.PC_BLOCK_JACOBI}[pc],
                          degree=m, mixed=mixed, tol=1e-9, maxit=2000, block=block or 64, bc=bc)
    assert ref.iterations == a[1] and np.array_equal(a[3], ref.x.ravel())
