#!/usr/bin/env python3
"""Write the stored trajectories under tests/golden/ from the oracle alone.

Each fixture is a seeded solve: the per-iteration scalars alpha, omega, rho and
r.r of right-preconditioned Bi-CGSTAB (Alg. 1, scalar formulas of Alg. 3) as hex
floats, and the final x as the sha256 of its bytes plus 16 sampled entries, so
that the bits are exact. The full-size fixtures also store b.b and the squared
true residual ||b - A x||^2 of the oracle's own x (exact dot products).

    python tests/golden/make_golden.py           # small grids with ragged tile tails
    python tests/golden/make_golden.py --full    # the 256^3 and 512^3 workloads

Run from the repository root. The full-size set takes hours of CPU time (about
14 GiB of memory at 512^3); a fixture already on disk is kept unless --force.
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


# Full-size workloads: name -> (n, rhs, precond, degree, mixed, tol, maxit).
# rhs is ("uniform", seed) for f ~ U[-1, 1) or ("noisy", seed) for the
# manufactured right-hand side plus 1e-3 N(0, 1) noise; zero Dirichlet faces,
# h = 1/(n+1), x0 = 0, Block-Jacobi blocks of 64^3.
FULL = {
    "full_256_none": (256, ("uniform", 2), oracle.PC_NONE, 0, False, 1e-8, 5000),
    "full_256_jacobi": (256, ("uniform", 2), oracle.PC_JACOBI, 0, False, 1e-8, 5000),
    "full_256_bj64x8": (256, ("uniform", 2), oracle.PC_BLOCK_JACOBI, 8, False, 1e-8, 5000),
    "full_256_cheb4": (256, ("uniform", 2), oracle.PC_CHEBYSHEV, 4, False, 1e-8, 5000),
    "full_256_cheb8": (256, ("uniform", 2), oracle.PC_CHEBYSHEV, 8, False, 1e-8, 5000),
    "full_512_cheb8_fp64": (512, ("uniform", 4), oracle.PC_CHEBYSHEV, 8, False, 1e-8, 5000),
    "full_512_cheb8_mixed": (512, ("uniform", 4), oracle.PC_CHEBYSHEV, 8, True, 1e-8, 5000),
    "full_512_cheb8_fp64_tol1e-10": (512, ("uniform", 4), oracle.PC_CHEBYSHEV, 8, False, 1e-10,
                                     5000),
    "full_512_cheb8_mixed_tol1e-10": (512, ("uniform", 4), oracle.PC_CHEBYSHEV, 8, True, 1e-10,
                                      5000),
    "full_512_noisy_cheb8_tol1e-10": (512, ("noisy", 3), oracle.PC_CHEBYSHEV, 8, False, 1e-10,
                                      5000),
    "full_512_noisy_bj64x8_tol1e-10": (512, ("noisy", 3), oracle.PC_BLOCK_JACOBI, 8, False,
                                       1e-10, 5000),
}


def full_rhs(case):
    n, (kind, seed) = case[0], case[1]
    shape = (n, n, n)
    if kind == "uniform":
        return workloads.uniform_grid(seed, shape)
    return workloads.manufactured_noisy(shape, seed)


def solve_full(case):
    n, _, pc, m, mixed, tol, maxit = case
    f = full_rhs(case)
    h = workloads.spacing(n)
    res = oracle.bicgstab(f, h, pc=pc, degree=m, mixed=mixed, tol=tol, maxit=maxit, block=64)
    res.bb = oracle.dot(f, f)
    r = f - oracle.apply_A(res.x, h)
    res.rr_true = oracle.dot(r, r)
    return res


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
        if hasattr(res, "rr_true"):
            fh.write(f"bb {float(res.bb).hex()} rr_true {float(res.rr_true).hex()}\n")


def read(name):
    """(status, iterations, half, trace[its, 4], x sha256, n, {index: x value})"""
    return read_full(name)[:7]


def read_full(name):
    """read() plus (b.b, ||b - A x||^2), both None where the fixture has no such line"""
    with open(os.path.join(HERE, name + ".txt")) as fh:
        lines = [ln for ln in fh.read().splitlines() if not ln.startswith("#")]
    head = lines[0].split()
    status, its, half = int(head[1]), int(head[3]), int(head[5])
    trace = np.array([[float.fromhex(t) for t in ln.split()] for ln in lines[1:1 + its]])
    tail = lines[1 + its].split()
    sha, n = tail[1], int(tail[3])
    vals = [float.fromhex(t) for t in lines[2 + its].split()]
    bb = rr_true = None
    if len(lines) > 3 + its and lines[3 + its].startswith("bb "):
        extra = lines[3 + its].split()
        bb, rr_true = float.fromhex(extra[1]), float.fromhex(extra[3])
    return (status, its, half, trace.reshape(its, 4), sha, n, dict(zip(sample_indices(n), vals)),
            bb, rr_true)


def have(name):
    return os.path.exists(os.path.join(HERE, name + ".txt"))


def x_sha256(x):
    return hashlib.sha256(np.ascontiguousarray(x, dtype=np.float64).ravel().tobytes()).hexdigest()


if __name__ == "__main__":
    import time
    force = "--force" in sys.argv
    if "--full" in sys.argv:
        only = [a for a in sys.argv[1:] if not a.startswith("--")]
        for name, case in FULL.items():
            if (only and name not in only) or (have(name) and not force):
                continue
            t0 = time.time()
            r = solve_full(case)
            write(name, r)
            print(name, r.status, r.iterations, f"{time.time() - t0:.0f} s", flush=True)
    else:
        for name, case in CASES.items():
            r = solve(case)
            write(name, r)
            print(name, r.status, r.iterations)
