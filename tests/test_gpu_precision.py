"""The precision form at full size: complex64 storage with 5-qubit fused
gates applied as batched 32x32 complex GEMMs on FP32 MFMA (fusion products
in FP64, norms and inner products in FP64), on the 28- and 32-qubit layered
circuits, against the complex128 GPU path (itself checked against the
oracle's stored values at 28 qubits).  And the FP64-MFMA form of the same
fused gates in complex128 at 28 qubits, where every launch walks its
batches with a grid stride, against the oracle's stored values.

Tolerances: complex128 max |delta a| <= 1e-12; complex64 infidelity
1 - |<a|b>|^2 / (<a|a><b|b>) <= 1e-6 and max |delta a| <= 2e-5 max |a|."""
import os
import sys

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
FUSED5 = dict(opt=qsim.OPT_FUSE, force_fuse_k=5)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(name):
    from tests.golden.make_golden import read
    if not os.path.exists(os.path.join(HERE, "golden", f"{name}.txt")):
        pytest.skip(f"golden file {name}.txt not generated")
    return read(name)


def dense_mfma_ops(sim):
    """Full-pass dense ops of the plan with 5 qubits (the MFMA kernel)."""
    return sim.stats()["n_dense"]


def infidelity(a, b):
    ip = a.inner(b)
    return 1.0 - abs(ip) ** 2 / (a.norm() * b.norm())


@pytest.mark.parametrize("name", ["layered28", "layered32"])
def test_complex64_fused_k5_mfma_against_complex128(name):
    n, gates = W.config_circuit(name)
    say(f"{name}: complex64 forced k=5 (FP32 MFMA) vs complex128")
    ref = qsim.Simulator(n, dtype="c128", opt=qsim.OPT_ALL)
    ref.load(gates)
    ref.run()
    low = qsim.Simulator(n, dtype="c64", **FUSED5)
    low.load(gates)
    low.run()
    st = low.stats()
    # every pass is a fused dense gate; most are 5-qubit GEMMs
    assert st["n_stages"] == 0 and st["n_dense"] >= len(gates) // 40
    inf = infidelity(ref, low)
    say(f"{name}: {st['n_dense']} fused dense passes, infidelity {inf:.3e}")
    assert inf <= 1e-6
    assert abs(ref.norm() - 1) < 1e-11
    if name == "layered28":
        g = golden(name)
        got = low.amplitudes(g["idx"])
        err = float(np.max(np.abs(got - g["amp"])))
        say(f"{name}: complex64 max|delta| on {g['idx'].size} stored amplitudes {err:.3e}")
        assert err <= 2e-5 * float(np.max(np.abs(g["amp"])))
        # the complex128 reference path itself against the oracle's values
        assert float(np.max(np.abs(ref.amplitudes(g["idx"]) - g["amp"]))) <= 1e-12
    ref.close()
    low.close()


def test_complex128_fused_k5_mfma_grid_stride_28q():
    """FP64 MFMA 5-qubit fused gates at 28 qubits: 2^19 GEMM batches per
    launch, walked by a capped grid (16 batches per wave), against the
    oracle's stored amplitudes, marginals and norm."""
    g = golden("layered28")
    n, gates = W.config_circuit("layered28")
    say("layered28: complex128 forced k=5 (FP64 MFMA)")
    sim = qsim.Simulator(n, dtype="c128", **FUSED5)
    sim.load(gates)
    sim.run()
    assert sim.stats()["n_stages"] == 0
    got = sim.amplitudes(g["idx"])
    err = float(np.max(np.abs(got - g["amp"])))
    say(f"layered28 k=5 FP64 MFMA: max|delta| {err:.3e}")
    assert err <= 1e-12
    assert abs(sim.norm() - g["norm"]) < 1e-12
    for qs, ref in g["marginals"].items():
        assert np.max(np.abs(sim.probabilities(list(qs)) - ref)) < 1e-12
    sim.close()
