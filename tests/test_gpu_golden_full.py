"""Full-length parity at the benchmark sizes (256^3 and 512^3) against stored
oracle solves (Alg. 1 with the scalar formulas and kernel order of Alg. 3).

The oracle takes minutes (256^3) to the better part of an hour (512^3) per
solve on the CPU, so tests/golden/make_golden.py --full runs it once and stores
every iteration's alpha, omega, rho and r.r as hex floats, the final x as its
sha256 plus sampled entries, b.b and the squared true residual ||b - A x||^2 of
the oracle's own x. The GPU solve of the same seeded problem, in the launch
configuration the benchmark times, must reproduce all of it bit for bit: the
iteration count, the half-step flag, the whole trajectory, x, and the reported
true residual. A fixture that has not been written yet is skipped.
"""
import importlib.util
import math
import os

import numpy as np
import pytest
import torch

import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
G = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(G)


def device_rhs(case):
    n, (kind, seed) = case[0], case[1]
    if kind == "uniform":
        b = torch.empty(n ** 3, dtype=torch.float64, device="cuda:0")
        P.fill_uniform(b, seed)   # the host generator's bits, checked in test_gpu_kernels
        return b
    return torch.from_numpy(workloads.manufactured_noisy((n, n, n), seed).ravel()).to("cuda:0")


@pytest.mark.parametrize("name", sorted(G.FULL))
def test_gpu_reproduces_full_solve(gpu, name):
    if not G.have(name):
        pytest.skip(f"fixture {name} not written yet (make_golden.py --full)")
    status, its, half, trace, sha, size, samples, bb, rr_true = G.read_full(name)
    case = G.FULL[name]
    n, _, pc, m, mixed, tol, maxit = case
    print(f"[golden] {name}: {its} iterations", flush=True)
    b = device_rhs(case)
    with P.Solver((n, n, n), workloads.spacing(n), precision=P.MIXED if mixed else P.FP64) as s:
        x = torch.zeros_like(b)
        st = s.solve(b, x, pc, m, tol, maxit)   # oracle.PC_* and P.PC_* share their values
        torch.cuda.synchronize()
        d, tr = s.stats(), s.trace()
    del b
    assert (st, d["iterations"], d["half_step_exit"]) == (status, its, half)
    assert np.array_equal(tr, trace)
    xs = x.cpu().numpy()
    del x
    assert xs.size == size
    for i, v in samples.items():
        assert xs[i] == v, i
    assert G.x_sha256(xs) == sha
    # the reported true residual is the oracle's ||b - A x|| / ||b|| of the same x
    assert d["relres_true"] == math.sqrt(rr_true / bb)
