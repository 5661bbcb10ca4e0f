"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/poisson.h, and rejects invalid arguments
before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2503_08935_amd as P
from paper_2503_08935_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "poisson.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(poisson_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = P.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(B.EXPORTS) == names


def test_header_is_plain_c():
    text = open(os.path.join(ROOT, "include", "poisson.h")).read()
    assert 'extern "C"' in text
    for bad in ("torch", "std::", "hipStream_t", "class "):
        assert bad not in re.sub(r"/\*.*?\*/", "", text, flags=re.S)


def test_create_validation():
    L = P.lib()
    ctx = ctypes.c_void_p()
    for args in [(0, 4, 4, 0.1), (4, -1, 4, 0.1), (4, 4, 4, 0.0), (4, 4, 4, -1.0),
                 (4, 4, 4, float("nan")), (4, 4, 4, float("inf")), (1 << 13, 1 << 13, 1 << 13, 0.1),
                 (1 << 14, 1 << 14, 2, 0.1)]:
        assert L.poisson_create(*args, 0, ctypes.byref(ctx)) == P.ERR_ARG
        assert not ctx.value
    # Neumann on every face is singular; a mask above 6 bits or a Neumann face on a
    # 1-point axis is invalid
    assert L.poisson_create(4, 4, 4, 0.1, 63, ctypes.byref(ctx)) == P.ERR_UNSUPPORTED
    assert L.poisson_create(4, 4, 4, 0.1, 64, ctypes.byref(ctx)) == P.ERR_ARG
    assert L.poisson_create(1, 4, 4, 0.1, 2, ctypes.byref(ctx)) == P.ERR_ARG
    assert L.poisson_create(4, 4, 4, 0.1, 22, ctypes.byref(ctx)) == P.OK and ctx.value
    L.poisson_destroy(ctx)
    assert L.poisson_create(4, 4, 4, 0.1, 0, None) == P.ERR_ARG
    assert L.poisson_create(4, 4, 4, 0.1, 0, ctypes.byref(ctx)) == P.OK and ctx.value
    L.poisson_destroy(ctx)
    L.poisson_destroy(None)


def test_options_and_solve_argument_checks():
    L = P.lib()
    s = P.Solver((8, 6, 4), 0.1)
    c = s._ctx
    assert L.poisson_set_option(c, 999, 1.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_PRECISION, 2.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_BLOCK, 1.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_BLOCK, 3.5) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_GRAPH_ITERS, 0.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_TILE_ORDER, 2.0) == P.OK
    assert L.poisson_set_option(c, B.OPT_TILE_ORDER, 3.0) == P.ERR_ARG
    for v in (0, 1, 2):  # steps per pass: one, two, three
        assert L.poisson_set_option(c, B.OPT_FUSE, float(v)) == P.OK
    for v in (3, 4):  # four in the mixed mode, four in both
        assert L.poisson_set_option(c, B.OPT_FUSE, float(v)) == P.OK
    assert L.poisson_set_option(c, B.OPT_FUSE, 5.0) == P.ERR_ARG
    for v in (0, 1):
        assert L.poisson_set_option(c, B.OPT_PAIR_LDS, float(v)) == P.OK
    assert L.poisson_set_option(c, B.OPT_PAIR_LDS, 2.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_LMIN_SCALE, -1.0) == P.ERR_ARG
    assert L.poisson_set_option(c, B.OPT_LMIN_SCALE, float("nan")) == P.ERR_ARG
    for k, v in [(B.OPT_PRECISION, 1), (B.OPT_BLOCK, 16), (B.OPT_LMIN_SCALE, 100.0),
                 (B.OPT_LMAX_SCALE, 1 - 1e-4), (B.OPT_BJ_GLOBAL_INTERVAL, 1),
                 (B.OPT_GRAPH_ITERS, 16), (B.OPT_USE_GRAPH, 0), (B.OPT_DEBUG_BREAKDOWN_AT, -1)]:
        assert L.poisson_set_option(c, k, float(v)) == P.OK
    fake = ctypes.c_void_p(0x1000)
    # argument errors are found before any device access
    assert L.poisson_solve(c, None, fake, 2, 8, 1e-8, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 7, 8, 1e-8, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, 65, 1e-8, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, -1, 1e-8, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, 8, 0.0, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, 8, 1.0, 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, 8, float("nan"), 10) == P.ERR_ARG
    assert L.poisson_solve(c, fake, fake, 2, 8, 1e-8, 0) == P.ERR_ARG
    st = B.Stats()
    st.struct_size = ctypes.sizeof(B.Stats)
    assert L.poisson_stats(c, ctypes.byref(st)) == P.ERR_ARG  # nothing solved yet
    assert L.poisson_kernel_bench(c, 0, 0, 1) == P.ERR_ARG     # no plan yet
    s.close()


def test_degenerate_chebyshev_interval_rejected():
    L = P.lib()
    one = P.Solver((1, 1, 1), 0.5)
    fake = ctypes.c_void_p(0x1000)
    assert L.poisson_solve(one._ctx, fake, fake, P.PC_CHEBYSHEV, 4, 1e-8, 10) == P.ERR_ARG
    one.close()


def test_strerror_covers_codes():
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert P.strerror(code) != "unknown status"
    assert P.strerror(42) == "unknown status"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()


def test_server_host_side_checks():
    L = P.lib()
    srv = ctypes.c_void_p()
    assert L.poisson_server_create(100, 4, None, ctypes.byref(srv)) == P.ERR_ARG
    assert L.poisson_server_create(1 << 20, 0, None, ctypes.byref(srv)) == P.ERR_ARG
    assert L.poisson_server_create(1 << 20, 4, None, None) == P.ERR_ARG
    assert L.poisson_server_create(1 << 20, 4, None, ctypes.byref(srv)) == P.OK
    fake = ctypes.c_void_p(0x1000)
    t = ctypes.c_uint64()
    # a request larger than the whole budget is rejected before any device access
    assert L.poisson_server_submit(srv, 64, 64, 64, 1 / 65, 0, fake, fake, 2, 4, 1, 1e-8, 100,
                                   ctypes.byref(t)) == P.ERR_NOMEM
    assert L.poisson_server_submit(srv, 8, 8, 8, 1 / 9, 63, fake, fake, 2, 4, 1, 1e-8, 100,
                                   ctypes.byref(t)) == P.ERR_UNSUPPORTED
    assert L.poisson_server_submit(srv, 8, 8, 8, 1 / 9, 0, fake, fake, 2, 4, 5, 1e-8, 100,
                                   ctypes.byref(t)) == P.ERR_ARG
    assert L.poisson_server_submit(srv, 8, 8, 8, 1 / 9, 0, fake, fake, 2, 4, 1, 2.0, 100,
                                   ctypes.byref(t)) == P.ERR_ARG
    assert L.poisson_server_poll(srv, 1, None) == P.ERR_ARG       # no such ticket
    assert L.poisson_server_step(srv, 0) == P.ERR_ARG
    assert L.poisson_server_set_option(srv, 99, 1.0) == P.ERR_ARG
    assert L.poisson_server_set_option(srv, B.SERVER_OPT_FOUR_STEPS, 2.0) == P.ERR_ARG
    assert L.poisson_server_set_option(srv, B.SERVER_OPT_FOUR_STEPS, 0.0) == P.OK
    assert L.poisson_server_set_option(srv, B.SERVER_OPT_FOUR_STEPS, 1.0) == P.OK
    info = B.ServerInfo()
    info.struct_size = ctypes.sizeof(B.ServerInfo)
    assert L.poisson_server_info(srv, ctypes.byref(info)) == P.OK
    assert info.queued == 0 and info.budget_bytes == 1 << 20
    L.poisson_server_destroy(srv)
    L.poisson_server_destroy(None)


def test_footprint_model():
    # mixed Chebyshev-4: r, r~, p, w, t in FP64 and p^, s^, three Chebyshev buffers (the
    # first pair writes y_1, w_2; the pair (3, 4) one more) and the FP32 copy of the
    # input: 5*8 + 6*4 = 64 bytes per unknown; with the s and p updates folded into the
    # first passes (the server's default) s and the second p in FP64: 80; plus tile
    # partials
    n = 128
    fp = P.footprint((n, n, n), P.PC_CHEBYSHEV, 4, P.MIXED)
    assert 80 * n ** 3 <= fp <= 80 * n ** 3 + 64 * 1024 + 15 * 256
    # FP64 Chebyshev-8: 7 FP64 vectors plus a ring of 4 for the fused step pairs, plus
    # the folds' two
    fp64 = P.footprint((n, n, n), P.PC_CHEBYSHEV, 8, P.FP64)
    assert 104 * n ** 3 <= fp64 <= 104 * n ** 3 + 64 * 1024 + 16 * 256
    # no preconditioner, Jacobi and degrees below 3: no folds
    assert P.footprint((n, n, n), P.PC_NONE, 0, P.FP64) < fp
    assert P.footprint((n, n, n), P.PC_CHEBYSHEV, 2, P.FP64) < 88 * n ** 3
