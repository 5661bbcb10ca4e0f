"""Input generators: the counter-based uniform generator against the published
splitmix64 reference outputs, and the paper's test problem against its
definition in the Experimental Setup (domain, spacing, faces, right-hand side)."""
import math

import numpy as np

from paper_2503_08935_amd import workloads

G = 0x9E3779B97F4A7C15


def test_splitmix64_reference_outputs():
    # splitmix64 (Steele, Lea, Flood 2014): state += G; output = mix(state).
    # Reference outputs: the first output from state 0, and the first five
    # outputs from state 1234567.
    assert int(workloads._mix(np.uint64(G))) == 0xE220A8397B1DCDAF
    states = [(1234567 + (i + 1) * G) % (1 << 64) for i in range(5)]
    got = [int(workloads._mix(np.uint64(s))) for s in states]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_uniform_is_the_keyed_stream():
    seed, n = 7, 1000
    key = int(workloads.key(seed))
    assert key == int(workloads._mix(np.uint64((seed + G) % (1 << 64))))
    bits = workloads.uniform_bits(seed, 0, n)
    for i in (0, 1, 517, n - 1):
        assert int(bits[i]) == int(workloads._mix(np.uint64((key + (i + 1) * G) % (1 << 64))))
    u = workloads.uniform(seed, n)
    assert np.all(u >= -1.0) and np.all(u < 1.0)
    assert np.all(u * 2.0 ** 52 == np.round(u * 2.0 ** 52))  # multiples of 2^-52
    # an offset window is the same stream
    assert np.array_equal(workloads.uniform(seed, 10, start=500), u[500:510])


def test_uniform_moments():
    u = workloads.uniform(3, 1 << 20)
    assert abs(u.mean()) < 4.0 / math.sqrt(3 * (1 << 20))
    assert abs(u.var() - 1.0 / 3.0) < 2e-3


def test_paper_problem_definition():
    f, shape, h, bc = workloads.paper_problem()
    assert shape == (255, 255, 255) and h == 0.1 and f.shape == (255, 255, 255)
    # Neumann on x+, y-, z- (bits 1, 2, 4); Dirichlet on x-, y+, z+
    assert bc == (1 << 1) | (1 << 2) | (1 << 4)

    def rhs(x, y, z):
        return math.sin(x) + math.cos(y) + 3 * math.sin(z) - 2 * y * z + 2

    # first unknown: x = 3.1 (x- boundary node excluded), y = 2.5 and z = 10 (Neumann
    # boundary nodes included); last: x = 28.5 (Neumann node), y = 27.9, z = 35.4
    assert math.isclose(f[0, 0, 0], rhs(3.1, 2.5, 10.0), rel_tol=1e-14)
    assert math.isclose(f[-1, -1, -1], rhs(28.5, 27.9, 35.4), rel_tol=1e-14)
    assert math.isclose(f[7, 100, 31], rhs(3.0 + 3.2, 2.5 + 10.0, 10.0 + 0.7), rel_tol=1e-13)
