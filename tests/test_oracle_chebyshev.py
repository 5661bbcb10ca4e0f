"""Pins for the oracle's Chebyshev preconditioner (Alg. 2, eq. chebyshevQuantities).

m steps of the Chebyshev iteration started from zero leave the residual
polynomial T_{m+1}((theta - lambda)/delta) / T_{m+1}(sigma), so on an eigenvector
with eigenvalue lambda the preconditioner acts as the scalar
q_m(lambda) = (1 - T_{m+1}((theta - lambda)/delta) / T_{m+1}(sigma)) / lambda.
T_k is evaluated here with numpy's Chebyshev series, independently of the
oracle's three-term recurrence. The minimax property gives the spectral bound
|1 - lambda q_m(lambda)| <= 1/T_{m+1}(sigma) on [alpha, beta]."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import oracle
from tests.test_oracle_operator import block_ids, dense_P, sine_mode


def T(k, t):
    return C.chebval(t, [0] * k + [1])


def q(lam, lo, hi, m):
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    return (1 - T(m + 1, (theta - lam) / delta) / T(m + 1, theta / delta)) / lam


def mode_lambda(shape, ks, h):
    return sum(4 * np.sin(k * np.pi / (2 * (n + 1))) ** 2 for k, n in zip(ks, shape)) / h ** 2


@pytest.mark.parametrize("m", range(0, 9))
@pytest.mark.parametrize("ks", [(1, 1, 1), (2, 3, 1), (5, 4, 7), (20, 14, 11)])
def test_closed_form_on_sine_modes(m, ks):
    shape = (20, 14, 11)
    h = 1.0 / 21
    lo, hi = oracle.interval(shape, h)
    u = sine_mode(shape, ks)
    lam = mode_lambda(shape, ks, h)
    got = oracle.chebyshev(u, h, lo, hi, m)
    ref = q(lam, lo, hi, m) * u
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("m", [0, 1, 2, 4, 8])
def test_closed_form_fp32(m):
    shape = (16, 16, 16)
    h = 1.0 / 17
    lo, hi = oracle.interval(shape, h)
    for ks in [(1, 1, 1), (3, 2, 5), (16, 16, 16)]:
        u = sine_mode(shape, ks)
        lam = mode_lambda(shape, ks, h)
        got = oracle.chebyshev(u, h, lo, hi, m, mixed=True)
        ref = q(lam, lo, hi, m) * u
        assert np.abs(got - ref).max() <= 3e-5 * np.abs(ref).max()
        # the FP32 result is FP32-representable
        assert np.array_equal(got.astype(np.float32).astype(np.float64), got)


def test_interval_rescaling_changes_the_polynomial():
    shape = (12, 12, 12)
    h = 1.0 / 13
    lo, hi = oracle.interval(shape, h)
    u = sine_mode(shape, (2, 2, 2))
    lam = mode_lambda(shape, (2, 2, 2), h)
    lo2, hi2 = 100 * lo, hi * (1 - 1e-4)
    got = oracle.chebyshev(u, h, lo2, hi2, 6)
    assert np.abs(got - q(lam, lo2, hi2, 6) * u).max() <= 1e-12 * np.abs(got).max()


@pytest.mark.parametrize("m", [1, 3, 6])
def test_spectral_bound_dense(m):
    shape = (5, 4, 6)
    h = 0.2
    P = dense_P(shape, h)
    lo, hi = oracle.interval(shape, h)
    N = P.shape[0]
    Q = np.empty((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        Q[:, c] = oracle.chebyshev(e.reshape(6, 4, 5), h, lo, hi, m).ravel()
    ev = np.linalg.eigvals(P @ Q)
    bound = 1.0 / T(m + 1, (hi + lo) / (hi - lo))
    assert np.abs(ev.imag).max() < 1e-8
    assert np.abs(1 - ev.real).max() <= bound * (1 + 1e-9)
    # the preconditioner is a polynomial in P, so it commutes with it
    assert np.abs(P @ Q - Q @ P).max() <= 1e-10 * np.abs(P @ Q).max()


def test_block_jacobi_locality_and_local_closed_form():
    shape, bs = (12, 8, 8), 4
    h = 0.1
    lo, hi = oracle.interval(shape, h, block=bs)
    nx, ny, nz = shape
    # a sine mode of one 4x4x4 block, zero elsewhere
    u = np.zeros((nz, ny, nx))
    ks = (2, 1, 3)
    blk = sine_mode((bs, bs, bs), ks)
    u[4:8, 0:4, 8:12] = blk
    lam = mode_lambda((bs, bs, bs), ks, h)
    for m in (0, 1, 2, 5):
        got = oracle.chebyshev(u, h, lo, hi, m, block=bs)
        ref = np.zeros_like(u)
        ref[4:8, 0:4, 8:12] = q(lam, lo, hi, m) * blk
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # random data confined to one block stays in that block, for FP32 as well
    rng = np.random.default_rng(0)
    v = np.zeros((nz, ny, nx))
    v[0:4, 4:8, 4:8] = rng.standard_normal((4, 4, 4))
    for mixed in (False, True):
        got = oracle.chebyshev(v, h, lo, hi, 7, block=bs, mixed=mixed)
        mask = np.zeros_like(v, dtype=bool)
        mask[0:4, 4:8, 4:8] = True
        assert np.all(got[~mask] == 0.0) and np.abs(got[mask]).max() > 0


def test_block_jacobi_equals_blockwise_dense_chebyshev():
    """M_BJ^-1 = sum_s R_s^T q_m(R_s A R_s^T) R_s (eq. blockJacobiPreconditioner)."""
    shape, bs, h, m = (6, 4, 5), 3, 0.3, 4
    P = dense_P(shape, h)
    ids = block_ids(shape, bs)
    lo, hi = oracle.interval(shape, h, block=bs)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(P.shape[0])
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    ref = np.zeros_like(v)
    for b in np.unique(ids):
        sel = ids == b
        Ab = P[np.ix_(sel, sel)]
        w, V = np.linalg.eigh(Ab)
        ref[sel] = V @ (q(w, lo, hi, m) * (V.T @ v[sel]))
    got = oracle.chebyshev(v.reshape(5, 4, 6), h, lo, hi, m, block=bs).ravel()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def _first_step_fp32(u, h, lo, hi, au):
    """y = c1 (2u - A u / theta) in float32 for a given float32 A u, with c1 and
    theta computed in FP64 and rounded once (the first step of Alg. 2)."""
    theta, delta = (hi + lo) / 2.0, (hi - lo) / 2.0
    sigma = theta / delta
    rho_cur = 1.0 / (2.0 * sigma - 1.0 / sigma)
    c1 = np.float32(2.0 * rho_cur / delta)
    return c1 * (np.float32(2.0) * u.astype(np.float32) - au / np.float32(theta))


def test_fp32_operator_exact_on_smooth_quadratic():
    """The FP32 operator of the mixed mode keeps full accuracy where u is smooth.

    u = 1 + (i^2 + j^2 + k^2) 2^-23 is exact in float32, and at interior points
    (A u) = -6 * 2^-23 / h^2 exactly (each axis' second difference of i^2 is 2).
    Summing the differences (u - u_minus) + (u - u_plus) gets this exactly; 6u
    minus the neighbours would round 6u, whose bits span 2^2 .. 2^-22. The first
    Chebyshev step then equals the float32 evaluation of its formula with that
    A u, bit for bit."""
    n = 40
    shape = (n, n, n)
    h = 1.0 / (n + 1)
    ih2f = np.float32(1.0 / (h * h))
    i = np.arange(n, dtype=np.float64)
    q2 = i[:, None, None] ** 2 + i[None, :, None] ** 2 + i[None, None, :] ** 2
    u = 1.0 + q2 * 2.0 ** -23
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    lo, hi = oracle.interval(shape, h)
    got = oracle.chebyshev(u, h, lo, hi, 1, mixed=True).reshape(shape)
    au = np.float32(-6.0 * 2.0 ** -23) * ih2f
    ref = _first_step_fp32(u, h, lo, hi, au).astype(np.float64)
    inner = (slice(1, -1),) * 3
    assert np.array_equal(got[inner], ref[inner])
    # 6u first would not be exact here: the float32 rounding of 6u already moves it
    six_u = np.float32(6.0) * u.astype(np.float32)
    assert not np.array_equal(six_u.astype(np.float64), 6.0 * u)
