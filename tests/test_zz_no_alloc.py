"""The allocation-free marginal entry point (sim_probabilities_noalloc)
against sim_probabilities on the same states, through the C ABI: bitwise
equal results, on two calls in a row where the second is smaller, and the
context's device buffers do not grow."""
import ctypes

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(sim, qubits):
    lib = qsim.load_library()
    q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.uint32))
    out = np.empty(1 << len(q), dtype=np.float64)
    st = lib.sim_probabilities_noalloc(sim._ctx, q.ctypes.data if len(q) else None, len(q), out.ctypes.data)
    assert st == qsim.OK, lib.sim_last_error(sim._ctx)
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_marginals_equal_allocating_entry_point(dtype):
    # first call: 22 qubits, a wide marginal over low and high qubits (the
    # lane-contiguous path with many partial sums); second call: a smaller
    # state and fewer bins
    cases = [(22, list(range(6)) + [20, 11, 15, 7, 19, 9, 13, 17, 21, 10]),
             (12, [3, 1])]
    for n, qs in cases:
        print(f"noalloc: n={n} dtype={dtype} qubits={qs}", flush=True)
        sim = qsim.Simulator(n, dtype=dtype, opt=qsim.OPT_ALL)
        sim.load(W.layered(n, 4, seed=n))
        sim.run()
        before = sim.device_bytes()
        got = _noalloc(sim, qs)
        assert sim.device_bytes() == before            # nothing allocated by the call
        want = sim.probabilities(qs)
        assert np.array_equal(got, want)
        assert abs(got.sum() - 1.0) < (1e-12 if dtype == "c128" else 1e-5)
        # the norm (no qubits) and a single high qubit
        assert np.array_equal(_noalloc(sim, []), sim.probabilities([]))
        assert np.array_equal(_noalloc(sim, [n - 1]), sim.probabilities([n - 1]))
        sim.close()


def test_noalloc_rejects_bad_arguments():
    sim = qsim.Simulator(10, opt=0)
    sim.load(W.layered(10, 2, seed=3))
    lib = qsim.load_library()
    out = np.empty(1 << 17, dtype=np.float64)
    q = np.arange(17, dtype=np.uint32)
    assert lib.sim_probabilities_noalloc(sim._ctx, q.ctypes.data, 3, out.ctypes.data) == qsim.E_STATE
    sim.run()
    assert lib.sim_probabilities_noalloc(sim._ctx, q.ctypes.data, 11, out.ctypes.data) == qsim.E_INVAL
    dup = np.array([1, 1], dtype=np.uint32)
    assert lib.sim_probabilities_noalloc(sim._ctx, dup.ctypes.data, 2, out.ctypes.data) == qsim.E_INVAL
    assert lib.sim_probabilities_noalloc(sim._ctx, q.ctypes.data, 2, None) == qsim.E_INVAL
    sim.close()
