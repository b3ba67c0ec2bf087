"""Host-memory offload on the GPU: the state lives in pinned host memory and
passes through two device windows (2^W amplitudes each), pass by pass.
Checked against the oracle's full state at 16 qubits (windows of 2^12 /
2^13, so every pass streams 8 or 16 windows), and at 30 qubits with 2^28
windows (a device budget of 8 GiB for a 16 GiB state) against the oracle's
stored layered-circuit values and the product and diagonal closed forms.
Tolerance: complex128 max |delta a| <= 1e-12; complex64 infidelity <= 1e-6
and max |delta a| <= 2e-5 max |a|."""
import os
import sys

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def offload_run(n, gates, dtype, window, **kw):
    import time
    t0 = time.perf_counter()
    sim = qsim.Simulator(n, dtype=dtype, opt=kw.pop("opt", qsim.OPT_ALL), offload_window=window, **kw)
    t1 = time.perf_counter()
    sim.load(gates)
    t2 = time.perf_counter()
    if n >= 24:
        say(f"  offload n={n}: host buffer {t1 - t0:.1f} s, plan {t2 - t1:.1f} s "
            f"({sim.stats()['offload_passes']} passes); running")
    sim.run()
    if n >= 24:
        st = sim.stats()
        say(f"  offload n={n}: run {st['run_ms'] / 1e3:.1f} s, "
            f"{st['pcie_bytes'] / st['run_ms'] / 1e6:.1f} GB/s over the host link")
    return sim


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_offload_full_state_16q(oracle_mod, dtype):
    from tests.test_planner_cpu import _offload_cases
    n = 16
    Wq = 12 if dtype == "c128" else 13
    for name, gates in _offload_cases(n):
        say(f"offload 16q {dtype} {name}")
        want = oracle_mod.run(n, gates)
        sim = offload_run(n, gates, dtype, Wq)
        st = sim.stats()
        assert st["window_qubits"] == Wq and st["offload_passes"] >= 1
        got = sim.amplitudes()
        if dtype == "c128":
            assert np.max(np.abs(got - want)) <= 1e-12, name
            assert abs(sim.norm() - 1) < 1e-12
        else:
            assert oracle_mod.infidelity(want, got) <= 1e-6, name
            assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(want)) + 1e-7, name
        # marginals streamed window by window through the device
        qs = [15, 0, 9, 14]
        assert np.max(np.abs(sim.probabilities(qs) - oracle_mod.marginal(want, qs))) < \
            (1e-12 if dtype == "c128" else 1e-5)
        # a second run of the same plan gives the same state
        sim.run()
        assert np.array_equal(sim.amplitudes(), got)
        sim.close()


def test_offload_unsupported_outputs_and_window_limits():
    n = 16
    sim = offload_run(n, W.layered(n, 2, 3), "c128", 12)
    with pytest.raises(qsim.QsimError):
        sim.sample(np.array([0.5]))
    with pytest.raises(qsim.QsimError):
        sim.expect_z([1])
    with pytest.raises(qsim.QsimError):
        sim.probabilities_noalloc([0])
    sim.close()
    # a window smaller than one stage chunk is refused
    with pytest.raises(qsim.QsimError):
        qsim.Simulator(n, opt=qsim.OPT_ALL, offload_window=9)
    # offload needs cache-blocked stages
    with pytest.raises(qsim.QsimError):
        qsim.Simulator(n, opt=qsim.OPT_FUSE, offload_window=12)


def golden(name):
    from tests.golden.make_golden import read
    if not os.path.exists(os.path.join(HERE, "golden", f"{name}.txt")):
        pytest.skip(f"golden file {name}.txt not generated")
    return read(name)


def test_offload_layered30_against_stored_values():
    """A 16 GiB complex128 state through 2 x 4 GiB device windows."""
    g = golden("layered30")
    n, gates = W.config_circuit("layered30")
    say("offload layered30, windows of 2^28")
    sim = offload_run(n, gates, "c128", 28)
    st = sim.stats()
    say(f"offload layered30: {st['offload_passes']} passes, run {st['run_ms']:.0f} ms, "
        f"{st['pcie_bytes'] / st['run_ms'] / 1e6:.1f} GB/s over the host link")
    assert np.max(np.abs(sim.amplitudes(g["idx"]) - g["amp"])) <= 1e-12
    assert abs(sim.norm() - g["norm"]) < 1e-12
    for qs, ref in g["marginals"].items():
        assert np.max(np.abs(sim.probabilities(list(qs)) - ref)) < 1e-12
    sim.close()


def test_offload_closed_forms_30q():
    from oracle import closed_forms as CF
    n = 30
    idx = W.sample_indices(n, 1 << 20, 31)
    gates = W.product_circuit(n, 4, seed=32)
    say("offload product 30q")
    sim = offload_run(n, gates, "c128", 28)
    assert np.max(np.abs(sim.amplitudes(idx) - CF.product_state_amplitudes(n, gates, idx))) <= 1e-12
    sim.close()
    gates = W.hadamard_diagonal_circuit(n, 300, seed=33)
    say("offload hadamard-diagonal 30q")
    sim = offload_run(n, gates, "c128", 28)
    assert np.max(np.abs(sim.amplitudes(idx) - CF.hadamard_diagonal_amplitudes(n, gates, idx))) <= 1e-12
    assert abs(sim.norm() - 1) < 1e-12
    sim.close()
