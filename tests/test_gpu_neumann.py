"""GPU parity with Neumann and mixed boundary conditions (eq. matrix_neuman):
operator, preconditioners and full solves bitwise against the oracle, on
ragged multi-tile grids and with the face layout of the paper's test problem
(Dirichlet on x-, y+, z+; Neumann on x+, y-, z-)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu

PAPER_BC = 2 | 4 | 16
BCS = [PAPER_BC, 1, 2, 1 | 8 | 32, 3 | 12, 63 - 1]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(61, 47, 35), (130, 18, 9), (2, 3, 70)])
def test_operator_bitwise(gpu, bc, shape):
    h = 0.05
    u = workloads.uniform_grid(3, shape)
    with P.Solver(shape, h, bc=bc) as s:
        out = torch.empty(u.shape, dtype=torch.float64, device=gpu)
        s.apply_operator(dev(u), out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.apply_A(u, h, bc=bc))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("pc,m,block,mixed", [(P.PC_CHEBYSHEV, 5, 64, False),
                                              (P.PC_CHEBYSHEV, 5, 64, True),
                                              (P.PC_BLOCK_JACOBI, 4, 16, False),
                                              (P.PC_BLOCK_JACOBI, 6, 10, True)])
def test_preconditioner_bitwise(gpu, bc, pc, m, block, mixed):
    shape = (61, 47, 35)
    h = 1.0 / 62
    v = workloads.uniform_grid(8, shape)
    with P.Solver(shape, h, bc=bc, block=block, precision=P.MIXED if mixed else P.FP64) as s:
        out = torch.empty(v.shape, dtype=torch.float32 if mixed else torch.float64, device=gpu)
        s.apply_precond(pc, m, dev(v), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
    ref = oracle.precond(v, h, pc, degree=m, mixed=mixed, block=block, bc=bc)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("bc", [PAPER_BC, 3 | 12])
@pytest.mark.parametrize("pc,m,mixed", [(P.PC_NONE, 0, False), (P.PC_CHEBYSHEV, 8, False),
                                        (P.PC_CHEBYSHEV, 8, True), (P.PC_BLOCK_JACOBI, 8, False)])
def test_full_solve_bitwise(gpu, bc, pc, m, mixed):
    shape = (50, 41, 37)
    h = 1.0 / 51
    f = workloads.uniform_grid(6, shape)
    with P.Solver(shape, h, bc=bc, block=16, precision=P.MIXED if mixed else P.FP64) as s:
        b = dev(f)
        x = torch.zeros_like(b)
        st = s.solve(b, x, pc, m, 1e-8, 5000)
        torch.cuda.synchronize()
        stats, tr, xg = s.stats(), s.trace(), x.cpu().numpy()
    opc = {P.PC_NONE: oracle.PC_NONE, P.PC_CHEBYSHEV: oracle.PC_CHEBYSHEV,
           P.PC_BLOCK_JACOBI: oracle.PC_BLOCK_JACOBI}[pc]
    ref = oracle.bicgstab(f, h, pc=opc, degree=m, mixed=mixed, tol=1e-8, maxit=5000, block=16,
                          bc=bc)
    assert st == ref.status == P.OK
    assert stats["iterations"] == ref.iterations
    assert np.array_equal(tr[:, 0], ref.alpha) and np.array_equal(tr[:, 3], ref.rr)
    assert np.array_equal(xg, ref.x)
    assert stats["relres_true"] < 2e-8


def test_invalid_face_masks(gpu):
    for shape, bc, code in [((1, 8, 8), 1, P.ERR_ARG), ((8, 8, 8), 63, P.ERR_UNSUPPORTED),
                            ((8, 8, 8), 64, P.ERR_ARG)]:
        with pytest.raises(P.PoissonError) as e:
            P.Solver(shape, 0.1, bc=bc)
        assert e.value.code == code
