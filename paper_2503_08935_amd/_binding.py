"""ctypes binding of libpoisson.so (see include/poisson.h). Argument marshalling
only: every step of a solve runs in the HIP kernels of the library. PyTorch is
used for device memory and streams."""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpoisson.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED = -1, -2, -3, -4
ERR_BREAKDOWN, ERR_NONFINITE, ERR_INTERNAL = -5, -6, -7
PC_NONE, PC_JACOBI, PC_CHEBYSHEV, PC_BLOCK_JACOBI = 0, 1, 2, 3
FP64, MIXED = 0, 1
OPT_PRECISION, OPT_BLOCK, OPT_LMIN_SCALE, OPT_LMAX_SCALE = 1, 2, 3, 4
OPT_BJ_GLOBAL_INTERVAL, OPT_GRAPH_ITERS, OPT_USE_GRAPH, OPT_DEBUG_BREAKDOWN_AT = 5, 6, 7, 8
OPT_FUSE, OPT_TILE_ORDER, OPT_PAIR_LDS, OPT_FUSE_UPDATES = 9, 10, 11, 12
KERNEL_CHEB_STEP, KERNEL_STENCIL_DOT, KERNEL_UPDATE_XR, KERNEL_CHEB_PAIR = 0, 1, 2, 3
KERNEL_CHEB_TRIPLE = 4
NOALLOC_SCRATCH_BYTES = 64 << 20

# every symbol declared in include/poisson.h
EXPORTS = [
    "poisson_create", "poisson_set_option", "poisson_set_stream", "poisson_solve",
    "poisson_solve_noalloc",
    "poisson_stats", "poisson_trace", "poisson_destroy", "poisson_strerror",
    "poisson_apply_operator", "poisson_apply_precond", "poisson_dot", "poisson_kernel_bench",
    "poisson_kernel_bytes", "poisson_fill_uniform", "poisson_cheb_interval",
    "poisson_server_create", "poisson_server_set_option", "poisson_server_footprint",
    "poisson_server_submit", "poisson_server_step", "poisson_server_poll", "poisson_server_info",
    "poisson_server_destroy",
]
SERVER_OPT_USE_GRAPH, SERVER_OPT_SIZE_CLASSES, SERVER_OPT_FUSE_UPDATES = 1, 2, 3
SERVER_OPT_FOUR_STEPS = 4


class Stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("status", ctypes.c_int), ("iterations", ctypes.c_int), ("half_step_exit", ctypes.c_int),
        ("precond", ctypes.c_int), ("degree", ctypes.c_int), ("precision", ctypes.c_int),
        ("relres_recursive", ctypes.c_double), ("relres_true", ctypes.c_double),
        ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
        ("solve_ms", ctypes.c_double), ("loop_ms", ctypes.c_double),
        ("model_bytes", ctypes.c_double), ("model_gbps", ctypes.c_double),
        ("history_len", ctypes.c_int), ("history", ctypes.POINTER(ctypes.c_double)),
    ]


class ServerInfo(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t), ("queued", ctypes.c_int), ("active", ctypes.c_int),
        ("completed", ctypes.c_long), ("steps", ctypes.c_long),
        ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
        ("budget_bytes", ctypes.c_size_t), ("busy_ms", ctypes.c_double),
    ]


class PoissonError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libpoisson.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.poisson_create.argtypes = [ip, ip, ip, ctypes.c_double, ctypes.c_uint,
                                     ctypes.POINTER(vp)]
        L.poisson_set_option.argtypes = [vp, ip, ctypes.c_double]
        L.poisson_set_stream.argtypes = [vp, vp]
        L.poisson_solve.argtypes = [vp, vp, vp, ip, ip, ctypes.c_double, ip]
        L.poisson_solve_noalloc.argtypes = [vp, vp, vp, ip, ip, ctypes.c_double, ip]
        L.poisson_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.poisson_trace.argtypes = [vp, dp, ip]
        L.poisson_cheb_interval.argtypes = [vp, ip, dp, dp]
        L.poisson_destroy.argtypes = [vp]
        L.poisson_destroy.restype = None
        L.poisson_strerror.argtypes = [ip]
        L.poisson_strerror.restype = ctypes.c_char_p
        L.poisson_apply_operator.argtypes = [vp, vp, vp]
        L.poisson_apply_precond.argtypes = [vp, ip, ip, vp, vp]
        L.poisson_dot.argtypes = [vp, vp, vp, dp]
        L.poisson_kernel_bench.argtypes = [vp, ip, ip, ip]
        L.poisson_kernel_bytes.argtypes = [vp, ip, ip]
        L.poisson_kernel_bytes.restype = ctypes.c_double
        L.poisson_fill_uniform.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_uint64]
        L.poisson_server_create.argtypes = [ctypes.c_size_t, ip, vp, ctypes.POINTER(vp)]
        L.poisson_server_set_option.argtypes = [vp, ip, ctypes.c_double]
        L.poisson_server_footprint.argtypes = [ip, ip, ip, ip, ip, ip,
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.poisson_server_submit.argtypes = [vp, ip, ip, ip, ctypes.c_double, ctypes.c_uint, vp, vp,
                                            ip, ip, ip, ctypes.c_double, ip,
                                            ctypes.POINTER(ctypes.c_uint64)]
        L.poisson_server_step.argtypes = [vp, ip]
        L.poisson_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Stats)]
        L.poisson_server_info.argtypes = [vp, ctypes.POINTER(ServerInfo)]
        L.poisson_server_destroy.argtypes = [vp]
        L.poisson_server_destroy.restype = None
        _lib = L
    return _lib


def strerror(code):
    return lib().poisson_strerror(int(code)).decode()


def _check(code, what):
    if code < 0:
        raise PoissonError(code, what)
    return code


def _ptr(t, n=None, dtypes=None):
    """Device pointer of a contiguous torch tensor (marshalling only)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA/HIP tensor")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"dtype {t.dtype} not in {dtypes}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _stats_dict(s):
    d = {k: getattr(s, k) for k, _ in Stats._fields_ if k not in ("history", "struct_size")}
    d["history"] = [s.history[i] for i in range(s.history_len)] if s.history_len else []
    return d


class Solver:
    """One poisson_ctx: an nx x ny x nz interior grid with spacing h."""

    def __init__(self, shape, h, bc=0, stream=None, **options):
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.n = nx * ny * nz
        self.h = float(h)
        ctx = ctypes.c_void_p()
        _check(lib().poisson_create(nx, ny, nz, self.h, bc, ctypes.byref(ctx)), "poisson_create")
        self._ctx = ctx
        self._stream = stream
        self.precision = FP64
        for k, v in options.items():
            self.set_option(k, v)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().poisson_destroy(self._ctx)
            self._ctx = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    _OPTS = dict(precision=OPT_PRECISION, block=OPT_BLOCK, lmin_scale=OPT_LMIN_SCALE,
                 lmax_scale=OPT_LMAX_SCALE, bj_global_interval=OPT_BJ_GLOBAL_INTERVAL,
                 graph_iters=OPT_GRAPH_ITERS, use_graph=OPT_USE_GRAPH,
                 debug_breakdown_at=OPT_DEBUG_BREAKDOWN_AT, fuse=OPT_FUSE,
                 tile_order=OPT_TILE_ORDER, pair_lds=OPT_PAIR_LDS, fuse_updates=OPT_FUSE_UPDATES)

    def set_option(self, key, value):
        k = self._OPTS[key] if isinstance(key, str) else key
        _check(lib().poisson_set_option(self._ctx, k, float(value)), f"set_option({key})")
        if k == OPT_PRECISION:
            self.precision = int(value)

    def _bind_stream(self):
        lib().poisson_set_stream(self._ctx, _stream_handle(self._stream))

    def solve(self, rhs, x, precond=PC_CHEBYSHEV, degree=8, tol=1e-8, maxit=5000):
        """Solve A x = rhs in place of x; returns the status (>= 0) or raises."""
        import torch
        self._bind_stream()
        st = lib().poisson_solve(self._ctx, _ptr(rhs, self.n, (torch.float64,)),
                                 _ptr(x, self.n, (torch.float64,)), int(precond), int(degree),
                                 float(tol), int(maxit))
        if st in (ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED, ERR_INTERNAL):
            raise PoissonError(st, "poisson_solve")
        return st

    def solve_noalloc(self, rhs, x, precond=PC_CHEBYSHEV, degree=8, tol=1e-8, maxit=5000):
        """solve() through poisson_solve_noalloc: no device allocation, the
        library's static scratch (NOALLOC_SCRATCH_BYTES per GPU) instead."""
        import torch
        self._bind_stream()
        st = lib().poisson_solve_noalloc(self._ctx, _ptr(rhs, self.n, (torch.float64,)),
                                         _ptr(x, self.n, (torch.float64,)), int(precond),
                                         int(degree), float(tol), int(maxit))
        if st in (ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED, ERR_INTERNAL):
            raise PoissonError(st, "poisson_solve_noalloc")
        return st

    def stats(self):
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        _check(lib().poisson_stats(self._ctx, ctypes.byref(s)), "poisson_stats")
        return _stats_dict(s)

    def trace(self):
        import numpy as np
        n = self.stats()["iterations"]
        buf = np.zeros((max(n, 1), 4))
        got = _check(lib().poisson_trace(self._ctx, buf.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), n), "poisson_trace")
        return buf[:got]

    def cheb_interval(self, precond=PC_CHEBYSHEV):
        """(lambda_min, lambda_max) a Chebyshev / Block-Jacobi solve would use (host only)."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(lib().poisson_cheb_interval(self._ctx, int(precond), ctypes.byref(lo),
                                           ctypes.byref(hi)), "poisson_cheb_interval")
        return lo.value, hi.value

    def apply_operator(self, u, out):
        import torch
        self._bind_stream()
        _check(lib().poisson_apply_operator(self._ctx, _ptr(u, self.n, (torch.float64,)),
                                            _ptr(out, self.n, (torch.float64,))),
               "poisson_apply_operator")

    def apply_precond(self, precond, degree, v, out):
        """out = M^-1 v; out is float64 (FP64) or float32 (MIXED precision)."""
        import torch
        self._bind_stream()
        odt = torch.float32 if self.precision == MIXED else torch.float64
        _check(lib().poisson_apply_precond(self._ctx, int(precond), int(degree),
                                           _ptr(v, self.n, (torch.float64,)),
                                           _ptr(out, self.n, (odt,))),
               "poisson_apply_precond")

    def dot(self, x, y):
        import torch
        self._bind_stream()
        r = ctypes.c_double()
        _check(lib().poisson_dot(self._ctx, _ptr(x, self.n, (torch.float64,)),
                                 _ptr(y, self.n, (torch.float64,)), ctypes.byref(r)),
               "poisson_dot")
        return r.value

    def kernel_bench(self, kernel, precision, reps):
        self._bind_stream()
        _check(lib().poisson_kernel_bench(self._ctx, int(kernel), int(precision), int(reps)),
               "poisson_kernel_bench")

    def kernel_bytes(self, kernel, precision):
        return lib().poisson_kernel_bytes(self._ctx, int(kernel), int(precision))


def fill_uniform(out, seed, stream=None):
    """out[i] = 2u_i - 1 from the counter-based splitmix64 generator (device)."""
    import torch
    _check(lib().poisson_fill_uniform(_stream_handle(stream), _ptr(out, None, (torch.float64,)),
                                      out.numel(), int(seed)), "poisson_fill_uniform")


def footprint(shape, precond, degree, precision):
    """Arena bytes one request of this plan needs in a Server."""
    nx, ny, nz = shape
    b = ctypes.c_size_t()
    _check(lib().poisson_server_footprint(nx, ny, nz, int(precond), int(degree), int(precision),
                                          ctypes.byref(b)), "poisson_server_footprint")
    return b.value


class Server:
    """Continuous-batching server (poisson_server_*): FIFO admission by HBM footprint."""

    def __init__(self, budget_bytes, max_slots=64, stream=None, use_graph=True, size_classes=None,
                 fuse_updates=None, four_steps=None):
        srv = ctypes.c_void_p()
        self._stream = stream
        _check(lib().poisson_server_create(int(budget_bytes), int(max_slots),
                                           _stream_handle(stream), ctypes.byref(srv)),
               "poisson_server_create")
        self._srv = srv
        if not use_graph:
            _check(lib().poisson_server_set_option(srv, SERVER_OPT_USE_GRAPH, 0.0),
                   "poisson_server_set_option")
        if size_classes is not None:
            _check(lib().poisson_server_set_option(srv, SERVER_OPT_SIZE_CLASSES,
                                                   float(size_classes)),
                   "poisson_server_set_option")
        if fuse_updates is not None:
            _check(lib().poisson_server_set_option(srv, SERVER_OPT_FUSE_UPDATES,
                                                   float(fuse_updates)),
                   "poisson_server_set_option")
        if four_steps is not None:
            _check(lib().poisson_server_set_option(srv, SERVER_OPT_FOUR_STEPS, float(four_steps)),
                   "poisson_server_set_option")

    def close(self):
        if getattr(self, "_srv", None):
            lib().poisson_server_destroy(self._srv)
            self._srv = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, rhs, x, shape, h, precond=PC_CHEBYSHEV, degree=4, precision=MIXED, tol=1e-8,
               maxit=5000, bc=0):
        import torch
        nx, ny, nz = shape
        n = nx * ny * nz
        t = ctypes.c_uint64()
        _check(lib().poisson_server_submit(self._srv, nx, ny, nz, float(h), int(bc),
                                           _ptr(rhs, n, (torch.float64,)),
                                           _ptr(x, n, (torch.float64,)), int(precond), int(degree),
                                           int(precision), float(tol), int(maxit), ctypes.byref(t)),
               "poisson_server_submit")
        return t.value

    def step(self, iters=8):
        return _check(lib().poisson_server_step(self._srv, int(iters)), "poisson_server_step")

    def poll(self, ticket):
        """(status, stats) with status PENDING while not finished (stats None)."""
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        st = lib().poisson_server_poll(self._srv, int(ticket), ctypes.byref(s))
        if st == ERR_ARG:
            raise PoissonError(st, "poisson_server_poll")
        if st == PENDING:
            return st, None
        return st, _stats_dict(s)

    def info(self):
        i = ServerInfo()
        i.struct_size = ctypes.sizeof(ServerInfo)
        _check(lib().poisson_server_info(self._srv, ctypes.byref(i)), "poisson_server_info")
        return {k: getattr(i, k) for k, _ in ServerInfo._fields_ if k != "struct_size"}
