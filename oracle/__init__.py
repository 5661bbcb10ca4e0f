"""Plain FP64 CPU oracle for preconditioned Bi-CGSTAB on the 3D Poisson problem.

TEST INFRASTRUCTURE. Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package. The GPU library never
imports, links or calls it, and this package imports nothing from the GPU
library. The arithmetic lives in ``oracle.c`` (plain C, OpenMP over z-planes,
exact dot products); this module only marshals numpy arrays through ctypes.

Paper: Pennati et al., "A Parallel and Highly-Portable HPC Poisson Solver:
Preconditioned Bi-CGSTAB with alpaka", arXiv 2503.08935.
  - operator: Background section, eqs. matrix_dirichlet and matrix_p
  - interval: eqs. eigenvaluesPoissonDirichletMatrix, lambdaMin, lambdaMax
  - Chebyshev preconditioner: Alg. 2 with eq. chebyshevQuantities
  - Block-Jacobi(CI) / GNoComm(CI): eqs. blockJacobiPreconditioner and
    systemBJpreconditioner, Methodology section
  - Bi-CGSTAB: Alg. 1 (half-step exit) with the scalar formulas of Alg. 3
  - Neumann faces: the one-sided matrix N of eq. matrix_neuman (mirror ghost)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PC_NONE, PC_JACOBI, PC_CHEBYSHEV, PC_BLOCK_JACOBI = 0, 1, 2, 3
OK, NOT_CONVERGED, ERR_ARG, ERR_BREAKDOWN, ERR_NONFINITE = 0, 1, -1, -5, -6

BUILD_CMD = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-o", _LIB, _SRC, "-lm"]


def build():
    """Compile oracle.c into liboracle.so next to it."""
    subprocess.check_call(BUILD_CMD)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_dot.restype = ctypes.c_double
        L.orc_dot.argtypes = [dp, dp, ctypes.c_int64]
        L.orc_dirichlet_eig.restype = ctypes.c_double
        L.orc_dirichlet_eig.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_interval.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_interval_bc.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int,
                                                            ctypes.c_uint, dp, dp])
        L.orc_apply_A_bc.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int,
                                                           ctypes.c_uint, dp, dp])
        for f in (L.orc_chebyshev_bc, L.orc_chebyshev_f32_bc):
            f.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, ctypes.c_uint,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                dp, dp])
        L.orc_precond_bc.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_uint] +
                                     [ctypes.c_int] * 5 + [ctypes.c_double] * 2 + [dp, dp])
        L.orc_cheb_interval_bc.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_uint] +
                                           [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp, dp])
        L.orc_bicgstab_bc.restype = ctypes.c_int
        L.orc_bicgstab_bc.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_uint, dp,
                                                            dp] +
                                      [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int] +
                                      [ctypes.c_double] * 2 + [ctypes.c_int] * 2 +
                                      [ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)])
        L.orc_cheb_interval.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] +
                                        [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp, dp])
        L.orc_apply_A.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp]
        for f in (L.orc_chebyshev, L.orc_chebyshev_f32):
            f.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int, dp, dp])
        L.orc_precond.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] + [ctypes.c_int] * 5 +
                                  [ctypes.c_double] * 2 + [dp, dp])
        L.orc_bicgstab.restype = ctypes.c_int
        L.orc_bicgstab.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, dp, dp] +
                                   [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int] +
                                   [ctypes.c_double] * 2 + [ctypes.c_int] * 2 +
                                   [ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)])
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


def dot(x, y):
    """Exact dot product of two float64 vectors, rounded once to float64."""
    x = _f64(x).ravel()
    y = _f64(y).ravel()
    assert x.size == y.size
    return lib().orc_dot(_dp(x), _dp(y), x.size)


def dirichlet_eig(i, n):
    return lib().orc_dirichlet_eig(int(i), int(n))


def interval(shape, h, block=0, bc=0):
    """(lambda_min, lambda_max) of the grid operator, or an interval containing the
    spectra of all its diagonal blocks. bc: bit f (x-, x+, y-, y+, z-, z+) = Neumann."""
    nx, ny, nz = shape
    lo, hi = ctypes.c_double(), ctypes.c_double()
    lib().orc_interval_bc(nx, ny, nz, h, block, bc, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def cheb_interval(shape, h, precond, block=64, bj_global=0, lmin_scale=1.0, lmax_scale=1.0,
                  bc=0):
    nx, ny, nz = shape
    lo, hi = ctypes.c_double(), ctypes.c_double()
    lib().orc_cheb_interval_bc(nx, ny, nz, h, bc, precond, block, bj_global, lmin_scale,
                               lmax_scale, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def _grid(u):
    """Arrays are indexed [k, j, i] (x fastest); returns (nx, ny, nz)."""
    nz, ny, nx = u.shape
    return nx, ny, nz


def apply_A(u, h, block=0, bc=0):
    u = _f64(u)
    out = np.empty_like(u)
    nx, ny, nz = _grid(u)
    lib().orc_apply_A_bc(nx, ny, nz, h, block, bc, _dp(u), _dp(out))
    return out


def chebyshev(b, h, lo, hi, m, block=0, mixed=False, bc=0):
    b = _f64(b)
    out = np.empty_like(b)
    nx, ny, nz = _grid(b)
    f = lib().orc_chebyshev_f32_bc if mixed else lib().orc_chebyshev_bc
    f(nx, ny, nz, h, block, bc, lo, hi, m, _dp(b), _dp(out))
    return out


def precond(v, h, pc, degree=8, mixed=False, block=64, bj_global=0, lmin_scale=1.0,
            lmax_scale=1.0, bc=0):
    v = _f64(v)
    out = np.empty_like(v)
    nx, ny, nz = _grid(v)
    lib().orc_precond_bc(nx, ny, nz, h, bc, pc, degree, int(mixed), block, bj_global,
                         lmin_scale, lmax_scale, _dp(v), _dp(out))
    return out


class Result:
    def __init__(self, x, status, iterations, half, trace, rr0):
        self.x, self.status, self.iterations, self.half = x, status, iterations, half
        self.trace, self.rr0 = trace, rr0

    @property
    def alpha(self):
        return self.trace[:self.iterations, 0]

    @property
    def omega(self):
        return self.trace[:self.iterations, 1]

    @property
    def rho(self):
        return self.trace[:self.iterations, 2]

    @property
    def rr(self):
        return self.trace[:self.iterations, 3]


def bicgstab(b, h, pc=PC_NONE, degree=8, mixed=False, tol=1e-8, maxit=5000, x0=None,
             lmin_scale=1.0, lmax_scale=1.0, block=64, bj_global=0, jacobi_diag=0.0, bc=0):
    """Right-preconditioned Bi-CGSTAB (Alg. 1); returns a Result."""
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    nx, ny, nz = _grid(b)
    trace = np.zeros((maxit, 4))
    it, half = ctypes.c_int(), ctypes.c_int()
    rr0 = ctypes.c_double()
    st = lib().orc_bicgstab_bc(nx, ny, nz, h, bc, _dp(b), _dp(x), pc, degree, int(mixed), tol,
                               maxit, lmin_scale, lmax_scale, block, bj_global, jacobi_diag,
                               _dp(trace), ctypes.byref(rr0), ctypes.byref(it),
                               ctypes.byref(half))
    return Result(x, st, it.value, half.value, trace, rr0.value)
