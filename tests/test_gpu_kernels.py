"""GPU parity of single operations against the CPU oracle, element by element,
through the C ABI. Shapes span several tiles (64 x 4 columns, up to 64 planes)
with ragged tails in every direction."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_08935_amd as P
from paper_2503_08935_amd import workloads

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 32), (61, 47, 35), (130, 9, 70), (1, 1, 1), (5, 1, 300)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_fill_uniform_matches_host_generator(gpu):
    for n, seed in [(1, 0), (1000, 7), (333_333, 2**63 + 5)]:
        out = torch.empty(n, dtype=torch.float64, device=gpu)
        P.fill_uniform(out, seed)
        assert np.array_equal(host(out), workloads.uniform(seed, n))


@pytest.mark.parametrize("shape", SHAPES)
def test_operator_bitwise(gpu, shape):
    nx, ny, nz = shape
    h = 1.0 / (nx + 1)
    u = workloads.uniform_grid(11, shape)
    with P.Solver(shape, h) as s:
        out = torch.empty(u.shape, dtype=torch.float64, device=gpu)
        s.apply_operator(dev(u), out)
        assert np.array_equal(host(out), oracle.apply_A(u, h))


@pytest.mark.parametrize("shape", SHAPES[:3])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dot_is_correctly_rounded(gpu, shape, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    x = rng.standard_normal((nz, ny, nx)) * np.exp2(rng.integers(-20, 20, (nz, ny, nx)))
    y = x * (1 + 1e-10 * rng.standard_normal(x.shape)) - np.mean(x)
    with P.Solver(shape, 0.1) as s:
        for a, b in [(x, y), (x, x), (y, -x)]:
            assert s.dot(dev(a), dev(b)) == oracle.dot(a, b)


CASES = [
    (P.PC_JACOBI, 0, 0), (P.PC_CHEBYSHEV, 0, 0), (P.PC_CHEBYSHEV, 1, 0), (P.PC_CHEBYSHEV, 2, 0),
    (P.PC_CHEBYSHEV, 3, 0), (P.PC_CHEBYSHEV, 8, 0), (P.PC_BLOCK_JACOBI, 5, 16),
    (P.PC_BLOCK_JACOBI, 8, 7),
]


@pytest.mark.parametrize("pc,m,block", CASES)
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("shape", [(61, 47, 35), (130, 9, 70)])
def test_preconditioner_bitwise(gpu, pc, m, block, mixed, shape):
    nx, ny, nz = shape
    h = 1.0 / (nx + 1)
    v = workloads.uniform_grid(5, shape)
    opts = dict(precision=P.MIXED if mixed else P.FP64)
    if block:
        opts["block"] = block
    with P.Solver(shape, h, **opts) as s:
        out = torch.empty(v.shape, dtype=torch.float32 if mixed else torch.float64, device=gpu)
        s.apply_precond(pc, m, dev(v), out)
        got = host(out).astype(np.float64)
    ref = oracle.precond(v, h, pc, degree=m, mixed=mixed, block=block or 64)
    assert np.array_equal(got, ref)


LDS_CONFIGS = [
    dict(bc=0, pc=P.PC_CHEBYSHEV, block=64),            # select-free body
    dict(bc=2 | 4 | 16, pc=P.PC_CHEBYSHEV, block=64),   # the paper's faces: mirror selects
    dict(bc=1 | 32, pc=P.PC_CHEBYSHEV, block=64),
    dict(bc=1 | 2 | 4 | 8 | 16, pc=P.PC_CHEBYSHEV, block=64),
    dict(bc=0, pc=P.PC_BLOCK_JACOBI, block=16),         # block faces inside and at tile edges
    dict(bc=2 | 8 | 16, pc=P.PC_BLOCK_JACOBI, block=7),  # mask and mirror together
]


@pytest.mark.parametrize("cfg", LDS_CONFIGS, ids=lambda c: f"bc{c['bc']}-pc{c['pc']}-b{c['block']}")
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("shape", [(200, 37, 21), (128, 16, 8), (64, 16, 70), (3, 50, 2),
                                   (2, 1, 7), (257, 33, 9)])
def test_lds_pairs_match_register_pairs(gpu, cfg, mixed, shape):
    """The fused Chebyshev pairs staged in LDS over 128 x 16 (FP64) and 256 x 16 (FP32)
    tiles (the default) against the 64 x 16 register tiles and the oracle, bitwise:
    ragged x, y and z tails, a tile whose second wave column lies outside the grid,
    two-plane and single-row grids; Dirichlet, Neumann and mixed faces, Block-Jacobi
    masks; odd and even degrees (an odd degree ends with a single step, an even one
    with a pair that stores w_m only)."""
    nx, ny, nz = shape
    bc, pc, block = cfg["bc"], cfg["pc"], cfg["block"]
    for axis, n in enumerate(shape):
        if bc >> (2 * axis) & 3 and n < 2:
            pytest.skip("a Neumann face needs two points on its axis")
    h = 1.0 / (nx + 1)
    v = workloads.uniform_grid(9, shape)
    dt = torch.float32 if mixed else torch.float64
    for m in (3, 4, 8, 9):
        got = []
        for lds in (1, 0):
            with P.Solver(shape, h, bc=bc, block=block, pair_lds=lds,
                          precision=P.MIXED if mixed else P.FP64) as s:
                out = torch.empty(v.shape, dtype=dt, device=gpu)
                s.apply_precond(pc, m, dev(v), out)
                got.append(host(out).astype(np.float64))
        assert np.array_equal(got[0], got[1]), m
        ref = oracle.precond(v, h, pc, degree=m, mixed=mixed, block=block, bc=bc)
        assert np.array_equal(got[0], ref), m


@pytest.mark.parametrize("cfg", LDS_CONFIGS, ids=lambda c: f"bc{c['bc']}-pc{c['pc']}-b{c['block']}")
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("shape", [(200, 37, 21), (128, 16, 8), (64, 8, 70), (3, 50, 2),
                                   (257, 33, 9), (66, 70, 19)])
def test_triples_match_pairs(gpu, cfg, mixed, shape):
    """Three Chebyshev steps per pass (LDS-staged, 64 x 32 tiles of eight waves in FP64
    and 128 x 32 in FP32; steps 1-3 first) against two per pass and the oracle,
    bitwise, on ragged shapes (waves between the top and bottom one partly or wholly
    outside the grid; a tile row with grid rows on both sides), for every face type
    and block mask; degrees whose steps after the first triple split into triples
    only (6, 9), triples and a pair (5, 8) or triples and a single step (7, 10)."""
    nx, ny, nz = shape
    bc, pc, block = cfg["bc"], cfg["pc"], cfg["block"]
    for axis, n in enumerate(shape):
        if bc >> (2 * axis) & 3 and n < 2:
            pytest.skip("a Neumann face needs two points on its axis")
    h = 1.0 / (nx + 1)
    v = workloads.uniform_grid(10, shape)
    dt = torch.float32 if mixed else torch.float64
    for m in (5, 6, 7, 8, 9, 10):
        got = []
        for fuse in (2, 1):
            with P.Solver(shape, h, bc=bc, block=block, fuse=fuse,
                          precision=P.MIXED if mixed else P.FP64) as s:
                out = torch.empty(v.shape, dtype=dt, device=gpu)
                s.apply_precond(pc, m, dev(v), out)
                got.append(host(out).astype(np.float64))
        assert np.array_equal(got[0], got[1]), m
        ref = oracle.precond(v, h, pc, degree=m, mixed=mixed, block=block, bc=bc)
        assert np.array_equal(got[0], ref), m


@pytest.mark.parametrize("fuse", [0, 1, 2])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_fp32_operator_on_smooth_field(gpu, fuse, m):
    """Mixed mode on u = 1 + (i^2 + j^2 + k^2) 2^-23 (exact in FP32), where the
    FP32 operator's second-difference order is exact and 6u first is not: every
    FP32 kernel (one step per pass, pairs, triples) matches the oracle bit for
    bit, and the first step matches the float32 evaluation of its formula with
    A u = -6 * 2^-23 / h^2 at interior points."""
    shape = (70, 40, 36)
    nx, ny, nz = shape
    h = 1.0 / (nx + 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = 1.0 + (i * i + j * j + k * k).astype(np.float64) * 2.0 ** -23
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    with P.Solver(shape, h, precision=P.MIXED, fuse=fuse) as s:
        out = torch.empty(u.shape, dtype=torch.float32, device=gpu)
        s.apply_precond(P.PC_CHEBYSHEV, m, dev(u), out)
        got = host(out).astype(np.float64)
    assert np.array_equal(got, oracle.precond(u, h, P.PC_CHEBYSHEV, degree=m, mixed=True))
    if m == 1:
        lo, hi = oracle.interval(shape, h)
        theta, delta = (hi + lo) / 2.0, (hi - lo) / 2.0
        sigma = theta / delta
        c1 = np.float32(2.0 * (1.0 / (2.0 * sigma - 1.0 / sigma)) / delta)
        au = np.float32(-6.0 * 2.0 ** -23) * np.float32(1.0 / (h * h))
        ref = c1 * (np.float32(2.0) * u.astype(np.float32) - au / np.float32(theta))
        inner = (slice(1, -1),) * 3
        assert np.array_equal(got[inner], ref.astype(np.float64)[inner])


def test_dot_rounding_ties(gpu):
    """The rounding-tie cases the oracle's dot is pinned on, fed to the GPU's
    double-double reduction. A tie that the two words of the double-double hold
    exactly rounds to even as the exact dot does. A tie broken only by a term more
    than 106 bits below the sum (a sticky bit) is lost by the double-double, which
    then rounds the tie to even: one unit in the last place below the exact result.
    Solve data never comes that close to a tie (every trajectory test agrees bit for
    bit), but this is where the GPU's dot and the exact one differ, besides products
    that underflow below the subnormal range (there the product's error term is not
    representable)."""
    e53 = 2.0 ** -53
    cases = [
        # x, y, exact (= oracle), GPU
        ([1.0, e53], [1.0, 1.0], 1.0, 1.0),
        ([1.0, 3 * e53], [1.0, 1.0], 1.0 + 2.0 ** -51, 1.0 + 2.0 ** -51),
        ([-1.0, -e53], [1.0, 1.0], -1.0, -1.0),
        ([e53, 1.0], [1.0, 1.0], 1.0, 1.0),
        ([1.0, e53, 2.0 ** -300], [1.0, 1.0, 1.0], 1.0 + 2.0 ** -52, 1.0),
        ([1.0, e53, 2.0 ** -104], [1.0, 1.0, 1.0], 1.0 + 2.0 ** -52, 1.0 + 2.0 ** -52),
        # each product is half the smallest subnormal: the exact sum is one subnormal
        # step, while each rounded product and its FMA error term round to zero
        ([5e-324, 5e-324], [0.5, 0.5], 5e-324, 0.0),
        ([1e300, 1e300], [1e8, -1e8], 0.0, 0.0),
    ]
    for x, y, exact, want in cases:
        n = 130  # several waves; the values sit in the first and last lanes
        xs = np.zeros(n)
        ys = np.zeros(n)
        pos = [0, n - 1, 64][:len(x)]
        xs[pos], ys[pos] = x, y
        assert oracle.dot(xs, ys) == exact
        with P.Solver((n, 1, 1), 0.1) as s:
            got = s.dot(dev(xs), dev(ys))
        assert got == want, (x, y, got.hex(), want.hex())
