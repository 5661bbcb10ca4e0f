"""Stored trajectories (tests/golden/, written from the oracle alone by
tests/golden/make_golden.py): the oracle must keep reproducing them bit for bit
(a change of its arithmetic shows here), and the GPU path must reproduce them
through the C ABI."""
import importlib.util
import os

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
G = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(G)


@pytest.mark.parametrize("name", sorted(G.CASES))
def test_oracle_reproduces_fixture(name):
    status, its, half, trace, sha, n, samples = G.read(name)
    r = G.solve(G.CASES[name])
    assert (r.status, r.iterations, r.half) == (status, its, half)
    assert np.array_equal(r.trace[:its], trace)
    assert G.x_sha256(r.x) == sha and r.x.size == n


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(G.CASES))
def test_gpu_reproduces_fixture(gpu, name):
    import torch

    import paper_2503_08935_amd as P
    from paper_2503_08935_amd import workloads
    status, its, half, trace, sha, n, samples = G.read(name)
    shape, seed, pc, m, mixed, bc, tol = G.CASES[name]
    f = workloads.uniform_grid(seed, shape)
    pcs = {oracle.PC_NONE: P.PC_NONE, oracle.PC_CHEBYSHEV: P.PC_CHEBYSHEV,
           oracle.PC_BLOCK_JACOBI: P.PC_BLOCK_JACOBI, oracle.PC_JACOBI: P.PC_JACOBI}
    with P.Solver(shape, 1.0 / (shape[0] + 1), bc=bc,
                  precision=P.MIXED if mixed else P.FP64) as s:
        b = torch.from_numpy(f.ravel()).to("cuda:0")
        x = torch.zeros_like(b)
        st = s.solve(b, x, pcs[pc], m, tol, 5000)
        torch.cuda.synchronize()
        d, tr = s.stats(), s.trace()
    xs = x.cpu().numpy()
    assert (st, d["iterations"], d["half_step_exit"]) == (status, its, half)
    assert np.array_equal(tr, trace)
    for i, v in samples.items():
        assert xs[i] == v
    assert G.x_sha256(xs) == sha
