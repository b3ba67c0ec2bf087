"""The whole-state projections used to compare full-size states with the
oracle's (tests/golden/sketch.py): the hash is SplitMix64 as published, and
the projections are linear and see every amplitude."""
import numpy as np

from tests.golden.sketch import N_PROJ, _splitmix64, sketch


def test_splitmix64_published_values():
    # the generator seeded with 0 outputs mix(0x9E3779B97F4A7C15 * k) for
    # k = 1, 2, ...: first outputs 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4
    with np.errstate(over="ignore"):
        got = _splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert [int(v) for v in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_projection_of_basis_vectors_is_a_unit_weight():
    for x in (0, 1, 12345, (1 << 20) - 1):
        e = np.zeros(1 << 20, dtype=np.complex128)
        e[x] = 1.0
        s = sketch(e)
        assert s.shape == (N_PROJ,)
        # every weight is one of 1, i, -1, -i
        assert np.allclose(np.abs(s), 1.0, atol=0)
        assert np.all(np.isin(np.round(s.real) + 1j * np.round(s.imag), [1, 1j, -1, -1j]))


def test_projection_is_linear_and_sees_every_amplitude():
    rng = np.random.default_rng(4)
    n = 1 << 18
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2 * n)
    b = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2 * n)
    assert np.allclose(sketch(a + 2j * b), sketch(a) + 2j * sketch(b), rtol=0, atol=1e-13)
    # one amplitude off by delta moves every projection by |delta|
    for x in rng.integers(0, n, 8):
        c = a.copy()
        c[x] += 3e-9
        assert np.allclose(np.abs(sketch(c) - sketch(a)), 3e-9, rtol=1e-6, atol=0)
    # a transposition of two amplitudes is seen by some projection
    c = a.copy()
    c[[7, 8]] = c[[8, 7]]
    assert np.max(np.abs(sketch(c) - sketch(a))) > 1e-6
