"""GPU solver parity against the CPU oracle through the C ABI: full solves on
grids the oracle finishes in seconds (several tiles, ragged tails), iteration
counts, solution vectors and the per-iteration scalars alpha, omega, rho."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu

REL_TOL = 1e-9  # solution parity bar (relative 2-norm)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_solve(shape, h, f, pc, m, tol, maxit=5000, x0=None, bc=0, **opts):
    with P.Solver(shape, h, bc=bc, **opts) as s:
        b = dev(f)
        x = dev(x0) if x0 is not None else torch.zeros_like(b)
        st = s.solve(b, x, pc, m, tol, maxit)
        torch.cuda.synchronize()
        return st, s.stats(), s.trace(), x.cpu().numpy()


def oracle_pc(pc):
    return {P.PC_NONE: oracle.PC_NONE, P.PC_JACOBI: oracle.PC_JACOBI,
            P.PC_CHEBYSHEV: oracle.PC_CHEBYSHEV, P.PC_BLOCK_JACOBI: oracle.PC_BLOCK_JACOBI}[pc]


def check_parity(shape, h, f, pc, m, tol, mixed=False, block=64, bj_global=0, lmin=1.0, lmax=1.0,
                 maxit=5000):
    opts = dict(precision=P.MIXED if mixed else P.FP64, block=block, bj_global_interval=bj_global,
                lmin_scale=lmin, lmax_scale=lmax)
    st, stats, tr, x = gpu_solve(shape, h, f, pc, m, tol, maxit, **opts)
    ref = oracle.bicgstab(f, h, pc=oracle_pc(pc), degree=m, mixed=mixed, tol=tol, maxit=maxit,
                          block=block, bj_global=bj_global, lmin_scale=lmin, lmax_scale=lmax)
    assert st == ref.status
    assert abs(stats["iterations"] - ref.iterations) <= 1
    rel = np.linalg.norm(x - ref.x) / max(np.linalg.norm(ref.x), 1e-300)
    assert rel <= REL_TOL, rel
    return st, stats, tr, x, ref


def test_manufactured_32_one_iteration(gpu):
    n = 32
    h = workloads.spacing(n)
    f = workloads.manufactured((n, n, n))
    st, stats, tr, x, ref = check_parity((n, n, n), h, f, P.PC_NONE, 0, 1e-8)
    assert (st, stats["iterations"], stats["half_step_exit"]) == (P.OK, 1, 1)
    assert np.array_equal(x, ref.x)
    c = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    assert np.abs(x - c * workloads.manufactured_u((n, n, n))).max() < 1e-12


SOLVES = [
    dict(pc=P.PC_NONE, m=0),
    dict(pc=P.PC_JACOBI, m=0),
    dict(pc=P.PC_CHEBYSHEV, m=4),
    dict(pc=P.PC_CHEBYSHEV, m=8),
    dict(pc=P.PC_BLOCK_JACOBI, m=8, block=16),
    dict(pc=P.PC_BLOCK_JACOBI, m=6, block=16, bj_global=1, lmin=10.0, lmax=1 - 1e-4),
    dict(pc=P.PC_CHEBYSHEV, m=8, mixed=True),
    dict(pc=P.PC_CHEBYSHEV, m=4, mixed=True),
    dict(pc=P.PC_BLOCK_JACOBI, m=8, block=16, mixed=True),
    dict(pc=P.PC_JACOBI, m=0, mixed=True),
    dict(pc=P.PC_CHEBYSHEV, m=1),
    dict(pc=P.PC_CHEBYSHEV, m=0),
]


@pytest.mark.parametrize("case", SOLVES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_full_solve_parity_ragged(gpu, case):
    shape = (61, 47, 35)
    h = workloads.spacing(61)
    f = workloads.uniform_grid(2, shape)
    st, stats, tr, x, ref = check_parity(shape, h, f, case["pc"], case["m"], 1e-8,
                                         mixed=case.get("mixed", False),
                                         block=case.get("block", 64),
                                         bj_global=case.get("bj_global", 0),
                                         lmin=case.get("lmin", 1.0), lmax=case.get("lmax", 1.0))
    assert st == P.OK
    # the reproducible reductions make the whole trajectory identical
    assert stats["iterations"] == ref.iterations
    assert np.array_equal(tr[:, 0], ref.alpha) and np.array_equal(tr[:, 1], ref.omega)
    assert np.array_equal(tr[:, 2], ref.rho) and np.array_equal(tr[:, 3], ref.rr)
    assert np.array_equal(x, ref.x)
    assert stats["relres_true"] < 1.5e-8


def test_graph_and_poll_interval_do_not_change_bits(gpu):
    shape = (40, 33, 20)
    h = workloads.spacing(40)
    f = workloads.uniform_grid(9, shape)
    outs = []
    for use_graph, k in [(1, 8), (0, 3), (1, 1), (1, 64)]:
        st, stats, tr, x = gpu_solve(shape, h, f, P.PC_CHEBYSHEV, 4, 1e-10, use_graph=use_graph,
                                     graph_iters=k)
        outs.append((st, stats["iterations"], x))
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1] and np.array_equal(o[2], outs[0][2])


def test_special_cases(gpu):
    shape = (20, 17, 9)
    h = 0.05
    z = np.zeros((9, 17, 20))
    st, stats, tr, x = gpu_solve(shape, h, z, P.PC_CHEBYSHEV, 4, 1e-8, x0=np.ones_like(z))
    assert st == P.OK and stats["iterations"] == 0 and np.all(x == 0)
    f = workloads.uniform_grid(3, shape)
    bad = f.copy()
    bad[3, 4, 5] = np.inf
    st, stats, tr, x = gpu_solve(shape, h, bad, P.PC_CHEBYSHEV, 4, 1e-8)
    assert st == P.ERR_NONFINITE
    st, stats, tr, x = gpu_solve(shape, h, f, P.PC_NONE, 0, 1e-12, maxit=1)
    assert st == P.NOT_CONVERGED and stats["iterations"] == 1
    ref = oracle.bicgstab(f, h, pc=oracle.PC_NONE, tol=1e-12, maxit=1)
    assert np.array_equal(x, ref.x)
    # x0 already the solution: zero iterations
    xs = oracle.bicgstab(f, h, pc=oracle.PC_CHEBYSHEV, degree=4, tol=1e-13).x
    st, stats, tr, x = gpu_solve(shape, h, f, P.PC_CHEBYSHEV, 4, 1e-8, x0=xs)
    assert st == P.OK and stats["iterations"] == 0
    # forced omega = 0 at iteration 3 reports a breakdown there
    st, stats, tr, x = gpu_solve(shape, h, f, P.PC_CHEBYSHEV, 4, 1e-12, debug_breakdown_at=3)
    assert st == P.ERR_BREAKDOWN and stats["iterations"] == 3 and np.all(np.isfinite(x))


@pytest.mark.parametrize("pc,block,bc", [(P.PC_CHEBYSHEV, 64, 0), (P.PC_BLOCK_JACOBI, 16, 0),
                                         (P.PC_CHEBYSHEV, 64, 2 | 4 | 16),
                                         (P.PC_BLOCK_JACOBI, 10, 1 | 8)])
def test_fused_step_pairs_change_no_bits(gpu, pc, block, bc):
    """Two Chebyshev steps per pass (the default for FP64) against one per pass, and
    against the oracle, for every degree pattern (odd/even step counts, step 2 fused)."""
    shape = (61, 47, 35)
    h = workloads.spacing(61)
    f = workloads.uniform_grid(12, shape)
    for m in (3, 4, 5, 6, 7, 9):
        outs = []
        for fuse in (0, 1):
            st, stats, tr, x = gpu_solve(shape, h, f, pc, m, 1e-9, fuse=fuse, block=block, bc=bc)
            outs.append((st, stats["iterations"], x))
        assert outs[0][0] == outs[1][0] == P.OK
        assert outs[0][1] == outs[1][1] and np.array_equal(outs[0][2], outs[1][2]), m
    ref = oracle.bicgstab(f, h, pc=oracle_pc(pc), degree=9, tol=1e-9, block=block, bc=bc)
    assert ref.iterations == outs[1][1] and np.array_equal(ref.x, outs[1][2])


def test_kernel_bench_entry_points(gpu):
    shape = (96, 80, 70)
    h = workloads.spacing(96)
    f = workloads.uniform_grid(1, shape)
    with P.Solver(shape, h) as s:
        b = dev(f)
        x = torch.zeros_like(b)
        assert s.solve(b, x, P.PC_CHEBYSHEV, 8, 1e-8, 500) == P.OK
        x0 = x.clone()
        for k in (P.KERNEL_CHEB_STEP, P.KERNEL_CHEB_PAIR, P.KERNEL_STENCIL_DOT,
                  P.KERNEL_UPDATE_XR):
            s.kernel_bench(k, P.FP64, 3)
            assert s.kernel_bytes(k, P.FP64) > 0
        torch.cuda.synchronize()
        assert torch.equal(x, x0)  # the caller's solution is never touched
        with pytest.raises(P.PoissonError):
            s.kernel_bench(P.KERNEL_CHEB_STEP, P.MIXED, 1)  # plan is FP64


INTERIOR = [
    dict(pc=P.PC_CHEBYSHEV, m=8, bc=0),                   # fused pairs, no selects
    dict(pc=P.PC_CHEBYSHEV, m=7, bc=0, mixed=True),       # FP32 pairs of points
    dict(pc=P.PC_BLOCK_JACOBI, m=6, bc=0, block=16),      # block-face mask
    dict(pc=P.PC_CHEBYSHEV, m=5, bc=2 | 4 | 16),          # Neumann faces: selects kept
    dict(pc=P.PC_CHEBYSHEV, m=6, bc=1 | 32, mixed=True),
    dict(pc=P.PC_NONE, m=0, bc=0),
]


@pytest.mark.parametrize("nx", [128, 127])
@pytest.mark.parametrize("case", INTERIOR, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_interior_tile_paths_parity(gpu, nx, case):
    """Grids with whole 64-column tiles and interior wave rows, so the kernels'
    interior bodies (no guards, and without neighbour selects when every face is
    Dirichlet and there is no block mask) run next to the guarded edge bodies;
    nx odd takes the unpaired FP32 accesses. Bitwise against the oracle."""
    shape = (nx, 40, 24)
    h = 1.0 / 41
    f = workloads.uniform_grid(21, shape)
    mixed = case.get("mixed", False)
    block = case.get("block", 64)
    st, stats, tr, x = gpu_solve(shape, h, f, case["pc"], case["m"], 1e-9, bc=case["bc"],
                                 precision=P.MIXED if mixed else P.FP64, block=block)
    ref = oracle.bicgstab(f, h, pc=oracle_pc(case["pc"]), degree=case["m"], mixed=mixed,
                          tol=1e-9, block=block, bc=case["bc"])
    assert st == ref.status == P.OK
    assert stats["iterations"] == ref.iterations
    assert np.array_equal(tr[:, 0], ref.alpha) and np.array_equal(tr[:, 2], ref.rho)
    assert np.array_equal(x, ref.x)


@pytest.mark.parametrize("mixed", [False, True])
def test_tile_orders_change_no_bits(gpu, mixed):
    """The three tile orders (natural, x-grouped, slabs per XCD) only permute which
    workgroup takes which tile; the reductions commit per tile in tile order."""
    shape = (128, 64, 32)  # 32 tiles: every order is a full permutation
    h = 1.0 / 129
    f = workloads.uniform_grid(31, shape)
    outs = []
    for order in (0, 1, 2):
        st, stats, tr, x = gpu_solve(shape, h, f, P.PC_CHEBYSHEV, 7, 1e-9, tile_order=order,
                                     precision=P.MIXED if mixed else P.FP64)
        outs.append((st, stats["iterations"], x))
    for o in outs[1:]:
        assert o[0] == outs[0][0] == P.OK and o[1] == outs[0][1]
        assert np.array_equal(o[2], outs[0][2])


@pytest.mark.parametrize("mixed", [False, True])
def test_three_steps_per_pass_solve(gpu, mixed):
    """Full solves with three Chebyshev steps per pass: the same iterations and bits
    as the oracle."""
    shape = (130, 45, 33)
    h = 1.0 / 131
    f = workloads.uniform_grid(41, shape)
    st, stats, tr, x = gpu_solve(shape, h, f, P.PC_CHEBYSHEV, 8, 1e-9, fuse=2,
                                 precision=P.MIXED if mixed else P.FP64)
    ref = oracle.bicgstab(f, h, pc=oracle.PC_CHEBYSHEV, degree=8, mixed=mixed, tol=1e-9)
    assert st == ref.status == P.OK
    assert stats["iterations"] == ref.iterations
    assert np.array_equal(x, ref.x)


def test_byte_model_per_iteration(gpu):
    """The stats' model bytes follow the passes the plan runs: FP64 Chebyshev-8 moves
    632 B per unknown and iteration with one step per pass, 440 with two, 360 with
    steps 1-2, 3-5 and 6-8; mixed 264 with steps 1-3, 4-6, 7-8 and 224 with 1-4, 5-8.
    Folding the s and p updates into the first passes saves 8 B each: 424, 344, 248
    and 208; FP64 with 1-4, 5-8 and both folds (the default below 448^3) 264."""
    shape = (64, 48, 40)
    n = 64 * 48 * 40
    f = workloads.uniform_grid(5, shape)
    for fuse, mixed, fold, per in ((0, False, 1, 632), (1, False, 0, 440), (2, False, 0, 360),
                                   (2, True, 0, 264), (1, False, 1, 424), (2, False, 1, 344),
                                   (2, True, 1, 248), (3, True, 0, 224), (3, True, 1, 208),
                                   (3, False, 1, 264), (4, False, 1, 264)):
        st, stats, tr, x = gpu_solve(shape, 1.0 / 65, f, P.PC_CHEBYSHEV, 8, 1e-8, fuse=fuse,
                                     fuse_updates=fold, precision=P.MIXED if mixed else P.FP64)
        assert st == P.OK
        assert stats["model_bytes"] == per * n * stats["iterations"], (fuse, mixed, fold)


def test_update_folding_follows_the_grid_size(gpu):
    """By default the s and p updates are folded into first passes of two or three
    steps from 352^3 unknowns on (where it was measured faster) and not below: the
    stats' byte model shows which plan ran (344 against 360 B per unknown and
    iteration, FP64 Chebyshev-8 with three steps per pass)."""
    for shape, per in (((351, 352, 352), 360), ((352, 352, 352), 344)):
        n = shape[0] * shape[1] * shape[2]
        b = torch.empty(n, dtype=torch.float64, device="cuda:0")
        P.fill_uniform(b, 9)
        with P.Solver(shape, 1.0 / (shape[0] + 1), fuse=2) as s:
            x = torch.zeros_like(b)
            st = s.solve(b, x, P.PC_CHEBYSHEV, 8, 1e-12, 2)
            torch.cuda.synchronize()
            stats = s.stats()
        assert st == P.NOT_CONVERGED and stats["iterations"] == 2
        assert stats["model_bytes"] == per * n * 2, shape


def test_fp64_four_step_passes_follow_degree_and_size(gpu):
    """By default FP64 runs four Chebyshev steps per pass (folded: 264 B per unknown
    and iteration at degree 8) at degrees 4-7 and below 448^3 unknowns, and three
    (344 B) at degree 8 from 448^3 on, where four were not faster; a degree 4k+1
    starts with a pair and ends on a triple (degree 5: 1-2, 3-5, as with three)."""
    cases = [((447, 448, 448), 8, 264), ((448, 448, 448), 8, 344), ((448, 448, 448), 6, None),
             ((64, 48, 40), 5, None)]
    for shape, deg, per in cases:
        n = shape[0] * shape[1] * shape[2]
        b = torch.empty(n, dtype=torch.float64, device="cuda:0")
        P.fill_uniform(b, 9)
        got = {}
        for fuse in (None, 2, 4):
            opts = {} if fuse is None else dict(fuse=fuse)
            with P.Solver(shape, 1.0 / (shape[0] + 1), **opts) as s:
                x = torch.zeros_like(b)
                st = s.solve(b, x, P.PC_CHEBYSHEV, deg, 1e-12, 2)
                torch.cuda.synchronize()
                stats = s.stats()
            assert st == P.NOT_CONVERGED and stats["iterations"] == 2
            got[fuse] = (stats["model_bytes"] / (n * 2), x.cpu().numpy())
        if per is not None:
            assert got[None][0] == per, (shape, deg, got[None][0])
        if deg == 6:
            assert got[None][0] == got[4][0] < got[2][0]
        if deg == 5:
            assert got[4][0] == got[2][0]
        assert np.array_equal(got[None][1], got[2][1]) and np.array_equal(got[4][1], got[2][1])
        del b


def test_block_jacobi_four_step_passes_follow_degree_and_size(gpu):
    """By default mixed Block-Jacobi runs four Chebyshev steps per pass below 448^3
    unknowns and at degrees 4-7, three at degree 8 from 448^3 on; FP64
    Block-Jacobi always runs three (the byte model shows which plan ran)."""
    cases = [((447, 448, 448), 8, P.MIXED, 3), ((448, 448, 448), 8, P.MIXED, 2),
             ((448, 448, 448), 6, P.MIXED, 3), ((64, 48, 40), 6, P.FP64, 2)]
    for shape, deg, prec, same_as in cases:
        n = shape[0] * shape[1] * shape[2]
        b = torch.empty(n, dtype=torch.float64, device="cuda:0")
        P.fill_uniform(b, 9)
        got = {}
        for fuse in (None, 2, 3, 4):
            opts = {} if fuse is None else dict(fuse=fuse)
            with P.Solver(shape, 1.0 / (shape[0] + 1), precision=prec, block=64, **opts) as s:
                x = torch.zeros_like(b)
                st = s.solve(b, x, P.PC_BLOCK_JACOBI, deg, 1e-12, 2)
                torch.cuda.synchronize()
                stats = s.stats()
            assert st == P.NOT_CONVERGED and stats["iterations"] == 2
            got[fuse] = (stats["model_bytes"], x.cpu().numpy())
        assert got[None][0] == got[same_as][0], (shape, deg, prec)
        for f in (2, 3, 4):
            assert np.array_equal(got[None][1], got[f][1]), (shape, deg, prec, f)
        del b


def test_update_folding_with_four_step_passes(gpu):
    """A mixed plan whose applies start with a four-step pass (degree >= 4) folds the
    updates by default from 128^3 unknowns on; below 352^3 a mixed plan of degree 3
    (first pass: two steps) does not, and below 128^3 neither does."""
    for deg, folded, shape in ((8, True, (128, 128, 128)), (4, True, (128, 128, 128)),
                               (3, False, (128, 128, 128)), (8, False, (128, 128, 127))):
        f = workloads.uniform_grid(6, shape)
        got = {}
        for fold in (None, 0, 1):
            opts = {} if fold is None else dict(fuse_updates=fold)
            st, stats, tr, x = gpu_solve(shape, 1.0 / 129, f, P.PC_CHEBYSHEV, deg, 1e-12,
                                         maxit=3, precision=P.MIXED, **opts)
            assert st == P.NOT_CONVERGED and stats["iterations"] == 3
            got[fold] = (stats["model_bytes"], x)
        assert got[1][0] < got[0][0]
        assert got[None][0] == got[1 if folded else 0][0], deg
        assert np.array_equal(got[None][1], got[0][1]) and np.array_equal(got[1][1], got[0][1])
