"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance: max |delta a| <= 1e-12 for complex128 (the accuracy target of the
simulator); complex64 states are compared by infidelity <= 1e-6 and
max |delta a| <= 2e-5 * max |a| (single precision rounding over a few
thousand gates).
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W
from paper_2604_12256_amd.workloads import Gate

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_state(n, gates, dtype="c128", **kw):
    sim = qsim.Simulator(n, dtype=dtype, **kw)
    sim.load(gates)
    sim.run()
    out = sim.amplitudes()
    st = sim.stats()
    sim.close()
    return out, st


def check128(got, want, what=""):
    err = np.max(np.abs(got - want))
    assert err <= TOL128, f"{what}: max|delta| = {err:.3e}"
    return err


def check64(got, want, oracle_mod, what=""):
    inf = oracle_mod.infidelity(want, got.astype(np.complex128))
    err = np.max(np.abs(got - want))
    assert inf <= 1e-6, f"{what}: infidelity {inf:.3e}"
    assert err <= 2e-5 * np.max(np.abs(want)) + 1e-7, f"{what}: max|delta| {err:.3e}"


def test_layered12_plain_full_state(oracle_mod):
    """12-qubit layered circuit on the plain gate-by-gate path, full state."""
    n, gates = W.config_circuit("layered12")
    say("layered12 plain")
    got, st = gpu_state(n, gates, opt=0)
    assert st["full_passes"] == 540
    check128(got, oracle_mod.run(n, gates), "layered12 plain")


@pytest.mark.parametrize("opt", [0, 1, 2, 3, 4, 6, 7, 8, 12, 14, 15])
def test_random_circuits_every_pass(oracle_mod, opt):
    for n, seed, C in ((11, 1, 10), (14, 2, 12), (16, 3, 13), (15, 4, 11)):
        gates = W.random_mixed(n, 120, seed=seed + 7 * opt, max_k=5)
        say(f"random n={n} opt={opt} C={C}")
        got, _ = gpu_state(n, gates, opt=opt, C=C)
        check128(got, oracle_mod.run(n, gates), f"n={n} opt={opt}")


@pytest.mark.parametrize("L", [1, 3, 4, 6])
def test_stage_kernel_fixed_low_qubits(oracle_mod, L):
    """Stages whose local set holds only L of the low qubits (lanes on high
    qubits, contiguous runs of 2^L amplitudes), both dtypes."""
    n = 17
    gates = W.layered(n, 6, seed=20 + L)
    want = oracle_mod.run(n, gates)
    for dtype in ("c128", "c64"):
        say(f"fixed low L={L} {dtype}")
        got, st = gpu_state(n, gates, dtype=dtype, opt=qsim.OPT_ALL, L=L)
        assert st["n_stages"] >= 2
        if dtype == "c128":
            check128(got, want, f"L={L}")
        else:
            check64(got, want, oracle_mod, f"L={L}")


@pytest.mark.parametrize("C", [10, 11, 12, 13])
def test_stage_kernel_chunk_sizes(oracle_mod, C):
    """Targets on register, lane, wave and global bits for every chunk size."""
    n = 17
    gates = W.layered(n, 6, seed=C)
    say(f"stages n={n} C={C}")
    got, st = gpu_state(n, gates, opt=qsim.OPT_STAGES | qsim.OPT_FUSE, C=C)
    assert st["n_stages"] >= 2
    check128(got, oracle_mod.run(n, gates), f"C={C}")


def test_stage_kernel_operator_paths(oracle_mod):
    """Rare stage-kernel paths against the oracle: diagonal tables with more
    than four selector bits, two-bit dense operators with selectors, whole-
    register-tile dense operators (the shapes are asserted on the CPU in
    test_planner_cpu), in both precisions and several chunk sizes."""
    from tests.test_planner_cpu import operator_path_circuit
    n = 16
    gates = operator_path_circuit(n, 3)
    want = oracle_mod.run(n, gates)
    opt = qsim.OPT_STAGES | qsim.OPT_FUSE | qsim.OPT_DIAG
    for C in (11, 12, 13):
        say(f"operator paths c128 C={C}")
        got, _ = gpu_state(n, gates, opt=opt, C=C)
        check128(got, want, f"c128 C={C}")
    for C in (12, 13, 14):
        say(f"operator paths c64 C={C}")
        got, _ = gpu_state(n, gates, dtype="c64", opt=opt, C=C)
        check64(got, want, oracle_mod, f"c64 C={C}")
    say("operator paths all passes")
    got, _ = gpu_state(n, gates, opt=qsim.OPT_ALL)
    check128(got, want, "all passes")


def test_layered_and_diag_heavy_all_opts(oracle_mod):
    for n, gates in ((18, W.layered(18, 10, 5)), (18, W.diag_heavy(18, 300, 6)), (20, W.layered(20, 5, 7))):
        want = oracle_mod.run(n, gates)
        for opt in (qsim.OPT_ALL, qsim.OPT_STAGES | qsim.OPT_FUSE, qsim.OPT_FUSE | qsim.OPT_DIAG):
            say(f"n={n} opt={opt}")
            got, _ = gpu_state(n, gates, opt=opt)
            check128(got, want, f"n={n} opt={opt}")


def test_complex64_paths(oracle_mod):
    for n, gates in ((14, W.layered(14, 10, 2)), (16, W.random_mixed(16, 150, 5, max_k=5))):
        want = oracle_mod.run(n, gates)
        for opt in (0, qsim.OPT_FUSE, qsim.OPT_ALL, qsim.OPT_STAGES | qsim.OPT_FUSE):
            say(f"c64 n={n} opt={opt}")
            got, _ = gpu_state(n, gates, dtype="c64", opt=opt, C=12 if opt & 4 else 0)
            check64(got, want, oracle_mod, f"c64 n={n} opt={opt}")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_forced_fusion_mfma(oracle_mod, k):
    """Fused 3-, 4- and 5-qubit gates run as batched GEMMs on the matrix cores."""
    n, gates = 16, W.layered(16, 6, 11)
    want = oracle_mod.run(n, gates)
    for dtype in ("c128", "c64"):
        say(f"fuse{k} {dtype}")
        got, st = gpu_state(n, gates, dtype=dtype, opt=qsim.OPT_FUSE, force_fuse_k=k)
        if dtype == "c128":
            check128(got, want, "fuse5")
        else:
            check64(got, want, oracle_mod, "fuse5 c64")


def test_qubit_reordering_permutation(oracle_mod):
    """Planner inserts in-place low/high bit exchanges; outputs are translated
    back to logical order."""
    from .test_planner_cpu import high_qubit_circuit
    for n, C in ((14, 10), (18, 12)):
        gates = high_qubit_circuit(n, 6, 2, 12, 5)
        want = oracle_mod.run(n, gates)
        sim = qsim.Simulator(n, opt=qsim.OPT_ALL, C=C, L=6)   # six idle fixed low qubits
        sim.load(gates)
        sim.run()
        st = sim.stats()
        say(f"remap n={n}: perms {st['n_perm']}")
        assert st["n_perm"] >= 1
        check128(sim.amplitudes(), want, f"remap n={n}")
        idx = W.sample_indices(n, 500, 2)
        check128(sim.amplitudes(idx), want[idx.astype(np.int64)], "remap gather")
        assert np.max(np.abs(sim.probabilities([0, 3, n - 1]) - oracle_mod.marginal(want, [0, 3, n - 1]))) < 1e-13
        plain = qsim.Simulator(n, opt=0)
        plain.load(gates)
        plain.run()
        assert abs(sim.inner(plain) - 1) < 1e-12   # inner product across different layouts
        sim.close()
        plain.close()


def test_small_and_degenerate(oracle_mod):
    for n in (1, 2, 3, 5, 9, 10):
        gates = W.random_mixed(n, 40, seed=n, max_k=min(3, n))
        for opt in (0, qsim.OPT_ALL):
            got, _ = gpu_state(n, gates, opt=opt)
            check128(got, oracle_mod.run(n, gates), f"n={n}")
    # empty circuit: |0...0>, in both precisions, planned and plain
    for n in (1, 12):
        want = np.zeros(1 << n, dtype=np.complex128)
        want[0] = 1
        for dtype in ("c128", "c64"):
            for opt in (0, qsim.OPT_ALL):
                got, _ = gpu_state(n, [], dtype=dtype, opt=opt)
                assert np.array_equal(got, want), f"empty n={n} {dtype} opt={opt}"
    # one qubit in complex64
    gates = W.random_mixed(1, 40, seed=1, max_k=1)
    for opt in (0, qsim.OPT_ALL):
        got, _ = gpu_state(1, gates, dtype="c64", opt=opt)
        check64(got, oracle_mod.run(1, gates), oracle_mod, f"n=1 c64 opt={opt}")


def test_outputs_probabilities_norm_inner(oracle_mod):
    n = 16
    gates = W.layered(n, 8, 3)
    want = oracle_mod.run(n, gates)
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    idx = W.sample_indices(n, 1000, 1)
    check128(sim.amplitudes(idx), want[idx.astype(np.int64)], "gather")
    for qs in ([], [0], [15, 3], [2, 9, 4, 0], list(range(12)), list(range(4, 16))):
        got = sim.probabilities(qs)
        ref = oracle_mod.marginal(want, qs) if qs else np.array([oracle_mod.norm(want)])
        assert np.max(np.abs(got - ref)) < 1e-13, qs
    other = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
    other.load(gates)
    other.run()
    ip = sim.inner(other)
    ref = oracle_mod.inner(want, other.amplitudes())
    assert abs(ip - ref) < 1e-12
    assert abs(abs(ip) - 1) < 1e-5
    # determinism: a second run is bitwise identical
    a1 = sim.amplitudes()
    p1 = sim.probabilities([1, 2, 3])
    sim.run()
    assert np.array_equal(a1, sim.amplitudes())
    assert np.array_equal(p1, sim.probabilities([1, 2, 3]))
    sim.close()
    other.close()


def test_errors_reported():
    sim = qsim.Simulator(8)
    with pytest.raises(qsim.QsimError) as e:
        sim.amplitudes()
    assert e.value.status == qsim.E_STATE
    with pytest.raises(qsim.QsimError) as e:
        sim.load([Gate("H", (8,))])
    assert e.value.status == qsim.E_INVAL
    sim.load([Gate("H", (0,))])
    sim.run()
    with pytest.raises(qsim.QsimError):
        sim.amplitudes(np.array([256], dtype=np.uint64))
    with pytest.raises(qsim.QsimError):
        sim.probabilities([0, 0])
    # a failed load keeps the previous circuit
    with pytest.raises(qsim.QsimError):
        sim.load([Gate("CZ", (1, 1))])
    sim.run()
    assert abs(sim.amplitudes()[1] - 1 / math.sqrt(2)) < 1e-15
    sim.close()


# ---------------------------------------------------------------- full sizes
def golden(name):
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from tests.golden.make_golden import read
    path = os.path.join(HERE, "golden", f"{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"golden file {name}.txt not generated")
    return read(name)


@pytest.mark.parametrize("name", ["layered28", "layered30", "diag30"])
def test_full_size_against_golden(name):
    """Full-size workloads in the benchmark's configuration (all passes on),
    on the oracle's stored sample amplitudes, marginals and norm, and on the
    whole state through its seeded projections: a wrong amplitude anywhere
    moves every projection by its error (bound 1e-10; rounding differences
    spread over the state move them by about 1e-13)."""
    from tests.golden.make_golden import read_sketch
    from tests.golden.sketch import sketch
    g = golden(name)
    n, gates = W.config_circuit(name)
    say(f"full size {name}")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    got = sim.amplitudes(g["idx"])
    check128(got, g["amp"], name)
    assert abs(sim.norm() - g["norm"]) < 1e-12
    for qs, ref in g["marginals"].items():
        assert np.max(np.abs(sim.probabilities(list(qs)) - ref)) < 1e-12
    s_ref = read_sketch(name)
    if s_ref is not None:
        say(f"full size {name}: whole-state projections")
        err = np.max(np.abs(sketch(sim.amplitudes()) - s_ref))
        assert err < 1e-10, f"{name}: projections differ by {err:.3e}"
    sim.close()


def test_layered22_full_state(oracle_mod):
    """The 28-qubit configuration's circuit family (40 layers, seed 1) at 22
    qubits, where the oracle's full state takes seconds: every amplitude of
    the optimised path (booster, stages over 2^10 chunks, fusion) in both
    precisions against it."""
    n = 22
    gates = W.layered(n, 40, 1)
    say("layered22 full state (oracle)")
    want = oracle_mod.run(n, gates)
    for dtype in ("c128", "c64"):
        say(f"layered22 {dtype}")
        got, st = gpu_state(n, gates, dtype=dtype, opt=qsim.OPT_ALL)
        assert st["n_stages"] >= 2
        if dtype == "c128":
            check128(got, want, "layered22")
        else:
            check64(got, want, oracle_mod, "layered22 c64")


def test_diag24_full_state_and_samples(oracle_mod):
    n, gates = W.config_circuit("diag24")
    want = oracle_mod.run(n, gates)
    say("diag24")
    got, _ = gpu_state(n, gates, opt=qsim.OPT_ALL)
    check128(got, want, "diag24")
    idx = W.sample_indices(n, 1 << 20, 3).astype(np.int64)
    check128(got[idx], want[idx], "diag24 samples")
    assert abs(oracle_mod.norm(got) - 1) < 1e-12


def test_product_state_closed_form_30q():
    """Booster + tensor product at 30 qubits: single-qubit gates only."""
    from oracle import closed_forms as CF
    n = 30
    gates = W.product_circuit(n, 4, seed=8)
    idx = W.sample_indices(n, 1 << 20, 9)
    say("product 30q")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    check128(sim.amplitudes(idx), CF.product_state_amplitudes(n, gates, idx), "product30")
    assert abs(sim.norm() - 1) < 1e-12
    sim.close()


def test_diagonal_closed_form_30q():
    """Diagonal detector + phase tables at 30 qubits: H on all, then diagonals."""
    from oracle import closed_forms as CF
    n = 30
    gates = W.hadamard_diagonal_circuit(n, 400, seed=10)
    idx = W.sample_indices(n, 1 << 20, 11)
    say("hadamard-diagonal 30q")
    for opt in (qsim.OPT_ALL, qsim.OPT_DIAG | qsim.OPT_FUSE):
        sim = qsim.Simulator(n, opt=opt)
        sim.load(gates)
        sim.run()
        check128(sim.amplitudes(idx), CF.hadamard_diagonal_amplitudes(n, gates, idx), "hdiag30")
        sim.close()


def test_complex64_32q_against_complex128():
    """32-qubit layered circuit in complex64 on the optimised path (stages,
    all passes) against the complex128 path on the same GPU.  The forced
    5-qubit fused-GEMM form is in test_gpu_precision.py."""
    n, gates = W.config_circuit("layered32")
    say("layered32 c64 vs c128")
    a = qsim.Simulator(n, dtype="c128", opt=qsim.OPT_ALL)
    a.load(gates)
    a.run()
    b = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
    b.load(gates)
    b.run()
    ip = a.inner(b)
    inf = 1 - abs(ip) ** 2 / (a.norm() * b.norm())
    say(f"layered32 infidelity {inf:.3e}")
    assert inf <= 1e-6
    assert abs(a.norm() - 1) < 1e-11
    a.close()
    b.close()


def test_batched_small_circuits(oracle_mod):
    """One launch for many small circuits (serving path): each result equals
    the oracle and its solo run."""
    import torch
    sims, wants = [], []
    for i in range(20):
        n = 4 + (i % 10)
        gates = W.layered(n, 3 + i % 5, seed=100 + i)
        sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
        sim.load(gates)
        sims.append(sim)
        wants.append(oracle_mod.run(n, gates))
    qsim.run_batch(sims)
    torch.cuda.synchronize()
    for sim, want in zip(sims, wants):
        got = sim.amplitudes()
        check128(got, want, f"batch n={sim.n}")
        sim.run()
        solo = sim.amplitudes()
        check128(solo, got, "solo vs batch")
        sim.close()
    # complex64 batch
    sims = []
    for i in range(6):
        n = 10 + i % 5
        sim = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
        gates = W.layered(n, 4, seed=200 + i)
        sim.load(gates)
        sims.append((sim, oracle_mod.run(n, gates)))
    qsim.run_batch([s for s, _ in sims])
    torch.cuda.synchronize()
    for sim, want in sims:
        check64(sim.amplitudes(), want, oracle_mod, "batch c64")
        sim.close()


def test_batched_mid_size_circuits_staged(oracle_mod):
    """States above the small-state limit in one batch: their full-state
    stages go out together (one launch per stage step, one workgroup per
    chunk), with small circuits in the same call.  Each state is bitwise its
    solo run, and equals the oracle where the oracle is cheap."""
    import torch
    cases = []
    for i, (n, dt) in enumerate([(14, "c128"), (15, "c128"), (16, "c128"), (17, "c128"), (14, "c128"),
                                 (18, "c128"), (12, "c128"), (20, "c128")]):
        gates = W.layered(n, 6 + i % 4, seed=300 + i) + W.random_mixed(n, 30, seed=400 + i, max_k=3)
        sim = qsim.Simulator(n, dtype=dt, opt=qsim.OPT_ALL)
        sim.load(gates)
        cases.append((n, gates, sim))
    say("staged batch: 8 complex128 states of 12..20 qubits")
    qsim.run_batch([c[2] for c in cases])
    torch.cuda.synchronize()
    got = [c[2].amplitudes() for c in cases]
    for (n, gates, sim), g in zip(cases, got):
        if n <= 16:
            check128(g, oracle_mod.run(n, gates), f"staged batch n={n}")
        sim.run()
        solo = sim.amplitudes()
        if n > qsim_small_max("c128"):
            assert np.array_equal(solo, g), f"staged batch n={n} differs from its solo run"
        else:
            check128(g, solo, f"small n={n}")
        sim.close()
    # complex64, and a batch with more states than one launch holds
    sims = []
    for i in range(70):
        n = 15 + i % 3
        sim = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
        sim.load(W.layered(n, 3 + i % 3, seed=500 + i))
        sims.append(sim)
    say("staged batch: 70 complex64 states of 15..17 qubits")
    qsim.run_batch(sims)
    torch.cuda.synchronize()
    got = [s.amplitudes() for s in sims]
    for sim, g in zip(sims, got):
        sim.run()
        assert np.array_equal(sim.amplitudes(), g), f"staged batch c64 n={sim.n}"
        sim.close()


def test_batched_stages_with_quadratic_phases(oracle_mod):
    """A staged batch whose stage programs hold quadratic-phase operators
    (RZZ and QFT circuits) next to ones that do not: the launches that carry
    them run the kernel variant with the operator; every state equals its
    solo run bitwise and the oracle."""
    import torch
    cases = []
    for i, n in enumerate((15, 16, 17, 16, 15)):
        gates = (W.rzz_full(n, 20 + i), W.qft(n, 30 + i), W.layered(n, 4, 40 + i),
                 W.rzz_full(n, 50 + i), W.qft(n, 60 + i))[i]
        sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
        sim.load(gates)
        cases.append((n, gates, sim))
    nquad = 0
    for n, gates, _ in cases:
        ops = qsim.Plan(n, gates).ops()
        nquad += sum(1 for o in ops if o["kind"] == "STAGE" for k in o["kernel_ops"] if k.get("quad"))
    assert nquad >= 3
    say(f"staged batch with {nquad} quadratic-phase operators")
    qsim.run_batch([c[2] for c in cases])
    torch.cuda.synchronize()
    got = [c[2].amplitudes() for c in cases]
    for (n, gates, sim), g in zip(cases, got):
        check128(g, oracle_mod.run(n, gates), f"quad batch n={n}")
        sim.run()
        assert np.array_equal(sim.amplitudes(), g), f"quad batch n={n} differs from its solo run"
        sim.close()


def qsim_small_max(dtype):
    return 13 if dtype == "c128" else 14


def test_batch_rejects_duplicates_and_mixed_dtypes():
    a = qsim.Simulator(15, opt=qsim.OPT_ALL)
    b = qsim.Simulator(15, dtype="c64", opt=qsim.OPT_ALL)
    a.load(W.layered(15, 2, seed=1))
    b.load(W.layered(15, 2, seed=2))
    with pytest.raises(qsim.QsimError):
        qsim.run_batch([a, a])
    with pytest.raises(qsim.QsimError):
        qsim.run_batch([a, b])
    c = qsim.Simulator(15, opt=qsim.OPT_ALL)  # nothing loaded
    with pytest.raises(qsim.QsimError):
        qsim.run_batch([a, c])
    for s in (a, b, c):
        s.close()


def test_stage_at_the_phase_cap(oracle_mod):
    """Stages of 96 register phases (a deep brickwork with every qubit
    local) against the oracle, both dtypes."""
    rng = np.random.default_rng(5)
    n = 12
    gates = []
    for layer in range(150):
        for a in range(layer % 2, n - 1, 2):
            gates.append(Gate("U", (a, a + 1), 0.0, W.haar_unitary(rng, 4)))
    want = oracle_mod.run(n, gates)
    for dtype in ("c128", "c64"):
        say(f"phase cap {dtype}")
        got, _ = gpu_state(n, gates, dtype=dtype, opt=qsim.OPT_STAGES | qsim.OPT_FUSE)
        if dtype == "c128":
            check128(got, want, "phase cap")
        else:
            check64(got, want, oracle_mod, "phase cap c64")


def test_ghz_30q_closed_form():
    """GHZ at 30 qubits: exactly two amplitudes of 1/sqrt(2)."""
    n = 30
    gates = [Gate("H", (0,))] + [Gate("CNOT", (q, q + 1)) for q in range(n - 1)]
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    idx = np.concatenate([np.array([0, (1 << n) - 1], dtype=np.uint64), W.sample_indices(n, 1 << 16, 4)])
    got = sim.amplitudes(idx)
    want = np.zeros(idx.size, dtype=np.complex128)
    want[(idx == 0) | (idx == (1 << n) - 1)] = 1 / math.sqrt(2)
    check128(got, want, "ghz30")
    p = sim.probabilities([0, 29])
    assert np.max(np.abs(p - np.array([0.5, 0, 0, 0.5]))) < 1e-13
    sim.close()


def test_circuit_times_inverse_28q():
    """C * C^-1 = identity at full size: |0...0> comes back."""
    from .test_oracle_pins import inverse_circuit
    n, gates = W.config_circuit("layered28")
    say("layered28 + inverse")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates + inverse_circuit(gates))
    sim.run()
    idx = np.concatenate([np.array([0], dtype=np.uint64), W.sample_indices(n, 1 << 16, 6)])
    got = sim.amplitudes(idx)
    want = np.zeros(idx.size, dtype=np.complex128)
    want[idx == 0] = 1
    check128(got, want, "C C^-1")
    assert abs(sim.norm() - 1) < 1e-12
    sim.close()


@pytest.mark.parametrize("family", ["rzz", "qft", "qaoa"])
def test_benchmark_families_full_state(oracle_mod, family):
    """The benchmark circuits of Sec. 5 (fully-connected RZZ, QFT with its
    closing SWAPs, 5-level fully-connected QAOA) at 14 and 15 qubits: full
    state on the plain, staged and fully optimised paths, and in complex64."""
    for n in (14, 15):
        _, gates = W.config_circuit(f"{family}{n}")
        want = oracle_mod.run(n, gates)
        for opt in (0, qsim.OPT_STAGES | qsim.OPT_REMAP, qsim.OPT_ALL & ~qsim.OPT_QUAD, qsim.OPT_ALL):
            say(f"{family}{n} c128 opt={opt}")
            got, _ = gpu_state(n, gates, opt=opt, C=12)
            check128(got, want, f"{family}{n} opt={opt}")
        say(f"{family}{n} c64")
        got, _ = gpu_state(n, gates, dtype="c64", opt=qsim.OPT_ALL)
        check64(got, want, oracle_mod, f"{family}{n} c64")


def test_quadratic_phase_operator(oracle_mod):
    """Complex128 stages whose register phases collect many one- and two-qubit
    diagonals apply them as one quadratic-phase operator (chunk rows,
    per-thread rows, Gray-code walk over the register tile): every chunk size
    against the oracle, with the plan checked to use the operator; complex64
    (diagonal tables) on the same circuits."""
    # (n, circuit, chunk sizes at which the complex128 plan must use the operator)
    cases = [(16, W.rzz_full(16, 4), (11, 12, 13)),
             (17, W.qft(17, 6), (10, 11, 12, 13)),
             (17, W.qaoa_full(17, 2, 3), ()),
             (15, W.diag_heavy(15, 300, 9, 0.85), ())]
    for n, gates, expect in cases:
        want = oracle_mod.run(n, gates)
        for dtype, Cs in (("c128", (10, 11, 12, 13)), ("c64", (11, 12, 13, 14))):
            for C in Cs:
                ops = qsim.Plan(n, gates, dtype=dtype, C=C).ops()
                nquad = sum(1 for o in ops if o["kind"] == "STAGE" for k in o["kernel_ops"] if k.get("quad"))
                say(f"quad n={n} {dtype} C={C}: {nquad} operators")
                got, _ = gpu_state(n, gates, dtype=dtype, opt=qsim.OPT_ALL, C=C)
                if dtype == "c128":
                    check128(got, want, f"quad n={n} C={C}")
                else:
                    check64(got, want, oracle_mod, f"quad n={n} c64 C={C}")
                if dtype == "c128" and C in expect:
                    assert nquad >= 1, (n, C)


def test_quadratic_phase_operator_complex64(oracle_mod):
    """The quadratic-phase operator in complex64 stages (FP64 factors, one
    FP32 rounding per amplitude): 22-qubit RZZ and QAOA circuits whose
    complex64 plans use it at every chunk size, against the oracle."""
    n = 22
    for name, gates in (("rzz22", W.rzz_full(n, 4)), ("qaoa22", W.qaoa_full(n, 2, 3))):
        want = oracle_mod.run(n, gates)
        for C in (11, 13, 14):
            ops = qsim.Plan(n, gates, dtype="c64", C=C).ops()
            nquad = sum(1 for o in ops if o["kind"] == "STAGE" for k in o["kernel_ops"] if k.get("quad"))
            say(f"quad {name} c64 C={C}: {nquad} operators")
            assert nquad >= 1, (name, C)
            got, _ = gpu_state(n, gates, dtype="c64", opt=qsim.OPT_ALL, C=C)
            check64(got, want, oracle_mod, f"quad {name} c64 C={C}")


@pytest.mark.parametrize("family", ["rzz", "qft", "qaoa"])
def test_benchmark_families_30q_closed_form(family):
    """The same families at 30 qubits against their closed forms (diagonal
    phases, the Fourier kernel, QAOA weight classes) on 2^20 sampled indices."""
    from oracle import closed_forms as CF
    n, gates = W.config_circuit(f"{family}30")
    idx = W.sample_indices(n, 1 << 20, 12)
    if family == "rzz":
        want = CF.hadamard_diagonal_amplitudes(n, gates, idx)
    elif family == "qft":
        want = CF.qft_amplitudes(n, CF.qft_input(n, gates), idx)
    else:
        want = CF.qaoa_amplitudes(n, gates, idx)
    say(f"{family}30 c128")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    check128(sim.amplitudes(idx), want, f"{family}30")
    assert abs(sim.norm() - 1) < 1e-12
    if family == "qaoa":
        say("qaoa30 c64 vs c128")
        b = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
        b.load(gates)
        b.run()
        inf = 1 - abs(sim.inner(b)) ** 2 / (sim.norm() * b.norm())
        say(f"qaoa30 infidelity {inf:.3e}")
        assert inf <= 1e-6
        b.close()
    sim.close()


def test_batched_small_circuits_with_swaps(oracle_mod):
    """A solo run applies SWAPs as relabellings (the plan's layout moves); a
    batched small-state run applies the gates as given.  Outputs of both are
    in logical order, and so is the inner product between the two."""
    import torch
    cases = []
    for n in (5, 9, 12, 13):
        gates = W.qft(n, n) + W.random_mixed(n, 40, seed=n, max_k=3)
        assert qsim.Plan(n, gates).layout() != list(range(n))
        sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
        sim.load(gates)
        cases.append((n, gates, sim, oracle_mod.run(n, gates)))
    say("batched small circuits with SWAPs")
    qsim.run_batch([c[2] for c in cases])
    torch.cuda.synchronize()
    for n, gates, sim, want in cases:
        check128(sim.amplitudes(), want, f"batch n={n}")
        qs = [n - 1, 0, n // 2]
        np.testing.assert_allclose(sim.probabilities(qs), oracle_mod.marginal(want, qs), atol=1e-13)
        solo = qsim.Simulator(n, opt=qsim.OPT_ALL)
        solo.load(gates)
        solo.run()
        check128(solo.amplitudes(), want, f"solo n={n}")
        assert abs(abs(sim.inner(solo)) - 1) < 1e-12
        np.testing.assert_allclose(solo.probabilities(qs), oracle_mod.marginal(want, qs), atol=1e-13)
        solo.close()
        sim.close()


def test_served_results_equal_solo_runs():
    """Serving loop: every request's final state equals its solo run (batched
    small circuits and overlapping large ones)."""
    from paper_2604_12256_amd import serve as S
    reqs = W.serving_stream(24, 500.0, 7, n_min=8, n_max=22)
    be = S.GpuBackend(qsim.OPT_ALL, n_streams=3, keep_states=True)
    res = S.serve(reqs, be, max_streams=3)
    assert sorted(r.rid for r in res) == sorted(r.rid for r in reqs)
    assert any(r.mode == "batch" for r in res) and any(r.mode == "stream" for r in res)
    for req in reqs:
        solo = qsim.Simulator(req.n, dtype=req.dtype, opt=0)
        solo.load(req.circuit())
        solo.run()
        a = solo.amplitudes()
        b = be.kept[req.rid]
        if req.dtype == "c128":
            check128(b, a, f"served rid={req.rid}")
        else:
            assert 1 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real) <= 1e-6
        solo.close()


def test_served_mix_with_large_stream_requests():
    """Serving: 20-26-qubit requests on their own streams overlap a batch of
    small circuits; every result equals its solo run (the large ones are
    compared on 2^16 seeded indices and by norm, the small ones in full)."""
    from paper_2604_12256_amd import serve as S
    rng = np.random.default_rng(41)
    reqs = []
    for i in range(14):
        n = int(rng.integers(20, 27)) if i % 3 == 0 else int(rng.integers(8, 14))
        if i == 0:
            n = 26                  # on its stream while the first batch runs
        reqs.append(W.Request(i, 1e-4 * i, n, int(rng.integers(4, 12)), "c128" if i % 2 else "c64", 100 + i))
    be = S.GpuBackend(qsim.OPT_ALL, n_streams=3, keep_states=True)
    res = S.serve(reqs, be, max_streams=3)
    by = {r.rid: r for r in res}
    large = [r for r in reqs if r.n >= 20]
    assert large and all(by[r.rid].mode == "stream" for r in large)
    assert any(by[r.rid].mode == "batch" for r in reqs)
    # at least one batch ran while a large request was on its stream
    batches = [by[r.rid] for r in reqs if by[r.rid].mode == "batch"]
    assert any(b.start < by[l.rid].done and by[l.rid].start < b.done for b in batches for l in large)
    for req in reqs:
        say(f"served mix rid={req.rid} n={req.n} {req.dtype} {by[req.rid].mode}")
        solo = qsim.Simulator(req.n, dtype=req.dtype, opt=0)
        solo.load(req.circuit())
        solo.run()
        a = solo.amplitudes()
        b = be.kept[req.rid]
        if req.n >= 20:
            idx = W.sample_indices(req.n, 1 << 16, req.rid)
            a, b = a[idx], b[idx]
        if req.dtype == "c128":
            check128(b, a, f"served rid={req.rid}")
        else:
            err = np.max(np.abs(a - b))
            assert err <= 2e-5 * np.max(np.abs(a)) + 1e-7, (req.rid, err)
        solo.close()

