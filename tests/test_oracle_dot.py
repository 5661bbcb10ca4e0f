"""Pins for the oracle's dot product: the exact sum of exact products, rounded
once to the nearest double (ties to even). Checked against exact rational
arithmetic (Python Fractions), independent of the oracle's code."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def exact(x, y):
    return float(sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0)))


@pytest.mark.parametrize("seed", range(6))
def test_random_wide_range(seed):
    rng = np.random.default_rng(seed)
    n = 2000
    x = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))
    y = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))
    assert oracle.dot(x, y) == exact(x, y)


@pytest.mark.parametrize("seed", range(4))
def test_heavy_cancellation(seed):
    rng = np.random.default_rng(100 + seed)
    n = 500
    a = rng.standard_normal(n) * 1e10
    x = np.concatenate([a, -a, rng.standard_normal(7)])
    y = np.concatenate([np.ones(n), np.ones(n), rng.standard_normal(7) * 1e-20])
    perm = rng.permutation(x.size)
    x, y = x[perm], y[perm]
    naive = float(np.dot(x, y))
    ex = exact(x, y)
    assert oracle.dot(x, y) == ex
    assert ex != 0.0 and abs(ex) < 1e-15
    assert naive != ex  # plain summation loses it; the oracle does not


def test_ties_round_to_even():
    e53 = 2.0 ** -53
    # 1 + 2^-53 is half-way between 1 and 1 + 2^-52: ties to even gives 1
    assert oracle.dot([1.0, e53], [1.0, 1.0]) == 1.0
    # a sticky bit far below breaks the tie upwards
    assert oracle.dot([1.0, e53, 2.0 ** -300], [1.0, 1.0, 1.0]) == 1.0 + 2.0 ** -52
    # 1 + 3*2^-53 is half-way between 1+2^-52 and 1+2^-51: even is 1+2^-51
    assert oracle.dot([1.0, 3 * e53], [1.0, 1.0]) == 1.0 + 2.0 ** -51
    assert oracle.dot([-1.0, -e53], [1.0, 1.0]) == -1.0


def test_subnormal_and_extreme():
    tiny = 5e-324
    assert oracle.dot([tiny, tiny], [0.5, 0.5]) == exact([tiny, tiny], [0.5, 0.5])
    assert oracle.dot([tiny], [0.5]) == 0.0  # exact 2^-1075 ties to even (zero)
    assert oracle.dot([tiny], [0.75]) == tiny
    big = 1e300
    assert oracle.dot([big, big], [1e8, -1e8]) == 0.0  # exact cancellation beyond overflow
    assert math.isinf(oracle.dot([big], [1e10]))
    assert math.isnan(oracle.dot([np.inf, 1.0], [0.0, 1.0]))
    assert math.isnan(oracle.dot([np.inf, -np.inf], [1.0, 1.0]))
    assert oracle.dot([np.inf, 1.0], [1.0, 1.0]) == np.inf
    assert oracle.dot([], []) == 0.0


def test_order_and_thread_invariance():
    rng = np.random.default_rng(7)
    n = 300_000
    x = rng.uniform(-1, 1, n)
    y = x * (1 + 1e-9 * rng.standard_normal(n)) - x.mean()
    ref = oracle.dot(x, y)
    perm = rng.permutation(n)
    assert oracle.dot(x[perm], y[perm]) == ref
    old = oracle.get_threads()
    try:
        for t in (1, 3, 8):
            oracle.set_threads(t)
            assert oracle.dot(x, y) == ref
    finally:
        oracle.set_threads(old)
    # the exact result agrees with math.fsum of the exact products to within
    # the rounding of the products themselves
    assert abs(ref - math.fsum(x * y)) <= 1e-12 * np.abs(x * y).sum()
