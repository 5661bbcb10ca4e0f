"""The allocation-free solve (poisson_solve_noalloc) against poisson_solve.

Both run the same kernels on the same inputs, so x, the iteration count, the
status and the reported residuals must agree bit for bit. Two calls in a row go
through the one static scratch, the second on a smaller grid, so whatever the
first call left there must not leak into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu


def solve_both(shape, pc, deg, precision, seed, bc=0, block=None):
    dev = torch.device("cuda:0")
    f = workloads.uniform_grid(seed, shape)
    h = workloads.spacing(shape[0])
    b = torch.from_numpy(f).to(dev)
    out = {}
    opts = {"precision": precision}
    if block:
        opts["block"] = block
    with P.Solver(shape, h, bc=bc, **opts) as s:
        for name in ("solve", "solve_noalloc"):
            x = torch.zeros_like(b)
            st = getattr(s, name)(b, x, pc, deg, 1e-9, 2000)
            torch.cuda.synchronize()
            out[name] = (st, s.stats(), x.cpu().numpy())
    return out


def check_same(out):
    (st_a, sa, xa), (st_b, sb, xb) = out["solve"], out["solve_noalloc"]
    assert st_a == st_b == P.OK
    assert sa["iterations"] == sb["iterations"] > 0
    assert sa["half_step_exit"] == sb["half_step_exit"]
    assert np.array_equal(xa, xb)
    assert sa["relres_true"] == sb["relres_true"]
    assert sa["relres_recursive"] == sb["relres_recursive"]
    assert sb["history"] == []


def test_noalloc_matches_solve_twice_in_a_row(gpu):
    # the larger call first: a Chebyshev-8 FP64 plan over ragged tiles ...
    check_same(solve_both((83, 45, 37), P.PC_CHEBYSHEV, 8, P.FP64, 11))
    # ... then a smaller grid in the same scratch, mixed precision
    check_same(solve_both((29, 21, 17), P.PC_CHEBYSHEV, 5, P.MIXED, 12))


def test_noalloc_other_plans(gpu):
    check_same(solve_both((40, 21, 18), P.PC_CHEBYSHEV, 4, P.FP64, 13, bc=22))
    check_same(solve_both((48, 33, 35), P.PC_BLOCK_JACOBI, 6, P.FP64, 14, block=16))
    check_same(solve_both((37, 29, 23), P.PC_NONE, 0, P.FP64, 15))


def test_noalloc_rejects_what_does_not_fit(gpu):
    n = 96  # 96^3 * 88 B of an FP64 Chebyshev-8 workspace > 64 MiB
    dev = torch.device("cuda:0")
    b = torch.ones(n ** 3, dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)
    with P.Solver((n, n, n), workloads.spacing(n)) as s:
        with pytest.raises(P.PoissonError) as e:
            s.solve_noalloc(b, x, P.PC_CHEBYSHEV, 8, 1e-8, 10)
        assert e.value.code == P.ERR_NOMEM
        # the same call through poisson_solve allocates and works
        assert s.solve(b, x, P.PC_CHEBYSHEV, 8, 1e-8, 3) in (P.OK, P.NOT_CONVERGED)
    assert P.NOALLOC_SCRATCH_BYTES == 64 << 20


def test_noalloc_through_the_c_abi(gpu):
    L = P.lib()
    shape = (33, 31, 29)
    dev = torch.device("cuda:0")
    b = torch.from_numpy(workloads.uniform_grid(16, shape)).to(dev)
    xs = []
    for fn in (L.poisson_solve, L.poisson_solve_noalloc):
        with P.Solver(shape, workloads.spacing(shape[0])) as s:
            s._bind_stream()
            x = torch.zeros_like(b)
            rc = fn(s._ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                    P.PC_CHEBYSHEV, 6, 1e-8, 500)
            torch.cuda.synchronize()
            assert rc == P.OK
            xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
