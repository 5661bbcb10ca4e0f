#!/usr/bin/env python3
"""Write the stored trajectories under tests/golden/ from the oracle alone.

Each fixture is a seeded solve on a small grid with a ragged tile tail: the
per-iteration scalars alpha, omega, rho and r.r of right-preconditioned
Bi-CGSTAB (Alg. 1, scalar formulas of Alg. 3) as hex floats, and the final x
as the sha256 of its bytes plus 16 sampled entries, so that the bits are exact. Run from the repository root:
    python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2503_08935_amd import workloads  # noqa: E402

# name: (shape, seed, precond, degree, mixed, bc, tol)
CASES = {
    "cheb5_fp64_70x19x13": ((70, 19, 13), 41, oracle.PC_CHEBYSHEV, 5, False, 0, 1e-9),
    "cheb6_mixed_70x19x13": ((70, 19, 13), 42, oracle.PC_CHEBYSHEV, 6, True, 0, 1e-9),
    "cheb4_fp64_neumann22_40x21x18": ((40, 21, 18), 43, oracle.PC_CHEBYSHEV, 4, False, 22, 1e-9),
}


def solve(case):
    shape, seed, pc, m, mixed, bc, tol = case
    nx = shape[0]
    f = workloads.uniform_grid(seed, shape)
    return oracle.bicgstab(f, 1.0 / (nx + 1), pc=pc, degree=m, mixed=mixed, tol=tol, bc=bc)


SAMPLES = 16


def sample_indices(n):
    return [(i * 7919) % n for i in range(SAMPLES)]


def write(name, res):
    path = os.path.join(HERE, name + ".txt")
    xs = np.ascontiguousarray(res.x.ravel())
    with open(path, "w") as fh:
        fh.write("# written by tests/golden/make_golden.py from oracle/ only\n")
        fh.write(f"status {res.status} iterations {res.iterations} half {res.half}\n")
        for k in range(res.iterations):
            fh.write(" ".join(float(v).hex() for v in res.trace[k]) + "\n")
        fh.write(f"x_sha256 {hashlib.sha256(xs.tobytes()).hexdigest()} n {xs.size}\n")
        fh.write(" ".join(float(xs[i]).hex() for i in sample_indices(xs.size)) + "\n")


def read(name):
    """(status, iterations, half, trace[its, 4], x sha256, n, {index: x value})"""
    with open(os.path.join(HERE, name + ".txt")) as fh:
        lines = [ln for ln in fh.read().splitlines() if not ln.startswith("#")]
    head = lines[0].split()
    status, its, half = int(head[1]), int(head[3]), int(head[5])
    trace = np.array([[float.fromhex(t) for t in ln.split()] for ln in lines[1:1 + its]])
    tail = lines[1 + its].split()
    sha, n = tail[1], int(tail[3])
    vals = [float.fromhex(t) for t in lines[2 + its].split()]
    return status, its, half, trace.reshape(its, 4), sha, n, dict(zip(sample_indices(n), vals))


def x_sha256(x):
    return hashlib.sha256(np.ascontiguousarray(x, dtype=np.float64).ravel().tobytes()).hexdigest()


if __name__ == "__main__":
    for name, case in CASES.items():
        r = solve(case)
        write(name, r)
        print(name, r.status, r.iterations)
