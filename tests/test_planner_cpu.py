"""Host optimiser checks on the CPU (no GPU): every plan the library builds
must reproduce the oracle's state when its ops are interpreted, and the
booster / diagonal detector must behave as Sec. 4.4 and 4.5 describe."""
import itertools

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W
from paper_2604_12256_amd.workloads import Gate

from .planinterp import access_count, run_plan

ALL_OPTS = list(range(16)) + [31, 63, 16 | 4, 16 | 6, 16 | 12, 16 | 14, 32 | 6, 32 | 7, 32 | 14]


def plan_state(n, gates, **kw):
    p = qsim.Plan(n, gates, **kw)
    ops = p.ops()
    return ops, run_plan(ops, n, p.layout()), run_plan(ops, n, p.layout(), use_kernel_ops=False)


@pytest.mark.parametrize("opt", ALL_OPTS)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_every_pass_combination_matches_oracle(oracle_mod, opt, dtype):
    for n, seed in ((7, 1), (11, 2), (12, 3)):
        gates = W.random_mixed(n, 150, seed=seed + 10 * opt, max_k=4)
        want = oracle_mod.run(n, gates)
        C = 10 if dtype == "c128" else 11
        ops, got_k, got_g = plan_state(n, gates, dtype=dtype, opt=opt, C=C)
        assert np.max(np.abs(got_g - want)) < 1e-12, (n, opt)
        assert np.max(np.abs(got_k - want)) < 1e-12, (n, opt)


@pytest.mark.parametrize("opt", [qsim.OPT_ALL, qsim.OPT_STAGES, qsim.OPT_STAGES | qsim.OPT_FUSE,
                                 qsim.OPT_FUSE, qsim.OPT_BOOST | qsim.OPT_STAGES])
def test_layered_and_diag_heavy(oracle_mod, opt):
    for n, gates in ((12, W.layered(12, 8, 3)), (12, W.diag_heavy(12, 200, 5)), (13, W.layered(13, 4, 4))):
        want = oracle_mod.run(n, gates)
        for dtype, C in (("c128", 10), ("c128", 12), ("c64", 11), ("c64", 13)):
            ops, got_k, got_g = plan_state(n, gates, dtype=dtype, opt=opt, C=C)
            assert np.max(np.abs(got_k - want)) < 1e-12, (n, dtype, C)


def test_wide_gates_and_controls(oracle_mod):
    """5- and 6-qubit dense gates (beyond the register tile) and gates that
    are block diagonal in some qubits (controls) on global qubits."""
    n = 12
    rng = np.random.default_rng(3)
    gates = []
    for i in range(40):
        k = int(rng.integers(1, 7))
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        gates.append(Gate("U", qs, 0.0, W.haar_unitary(rng, 1 << k)))
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        gates.append(Gate("CNOT", (a, b)))
    want = oracle_mod.run(n, gates)
    for opt in (qsim.OPT_ALL, qsim.OPT_STAGES, qsim.OPT_FUSE):
        ops, got_k, got_g = plan_state(n, gates, opt=opt, C=10)
        assert np.max(np.abs(got_k - want)) < 1e-12


def test_stage_invariants():
    n, gates = 16, W.layered(16, 6, 9)
    p = qsim.Plan(n, gates, opt=qsim.OPT_STAGES | qsim.OPT_FUSE, C=12)
    for op in p.ops():
        if op["kind"] != "STAGE":
            continue
        local = set(op["local"])
        assert len(local) == 12 and set(range(6)) <= local
        for g in op["gates"]:
            m = g["payload"]
            if g["diagonal"]:
                continue
            # every qubit the operator is not block diagonal in must be local
            k = len(g["qubits"])
            for t, q in enumerate(g["qubits"]):
                r = np.arange(1 << k)
                off = ((r[:, None] ^ r[None, :]) >> t) & 1
                if np.any(np.abs(m[off == 1]) > 0):
                    assert q in local


# ---------------------------------------------------------------- diagonal detector (Sec. 4.5)
def figure4_circuit():
    """Reconstruction of the diagonal-detector example (the figure itself is
    not available): RZZ2, H3, RY4, RZZ5, CP6, RX7, RZZ8, CP9, a non-diagonal
    gate 10 on a qubit of the run, RZZ11 on that qubit."""
    return [
        Gate("H", (0,)), Gate("H", (1,)), Gate("H", (2,)), Gate("H", (3,)), Gate("H", (4,)),  # prefix
        Gate("RZZ", (0, 1), 0.3),      # 2
        Gate("H", (2,)),               # 3
        Gate("RY", (3,), 0.4),         # 4
        Gate("RZZ", (1, 2), 0.5),      # 5
        Gate("CPHASE", (2, 3), 0.6),   # 6
        Gate("RX", (4,), 0.7),         # 7  (barrier of the conventional fuser)
        Gate("RZZ", (0, 3), 0.8),      # 8
        Gate("CPHASE", (1, 3), 0.9),   # 9
        Gate("RX", (1,), 1.0),         # 10 (touches the run: deferred, marks qubit 1)
        Gate("RZZ", (1, 4), 1.1),      # 11 (touches a marked qubit: stops the run)
    ]


def conventional_diag_fusion(gates):
    """Fuses only runs of adjacent diagonal gates (stops at the first
    non-diagonal gate); returns the list of runs' qubit sets and sizes."""
    runs, cur = [], []
    for g in gates:
        if g.kind in W.DIAGONAL_KINDS:
            cur.append(g)
        else:
            if cur:
                runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    return [(sorted(set(q for g in r for q in g.qubits)), len(r)) for r in runs]


def test_diagonal_detector_figure4(oracle_mod):
    n = 5
    gates = figure4_circuit()
    p = qsim.Plan(n, gates, opt=qsim.OPT_DIAG)
    ops = p.ops()
    diags = [o for o in ops if o["kind"] == "DIAG"]
    # one 4-qubit fused diagonal from RZZ2, RZZ5, CP6, RZZ8, CP9 and RZZ11 alone
    assert [d["qubits"] for d in diags] == [[0, 1, 2, 3], [1, 4]]
    # gates after the prefix: H3, RY4, RX7, D4, RX10, RZZ11 -> 6 ops
    assert len([o for o in ops if o["kind"] in ("DENSE", "DIAG")]) == 5 + 6
    # conventional fusion: RZZ5+CP6 and RZZ8+CP9 are two 3-qubit runs
    runs = conventional_diag_fusion(gates[5:])
    assert ([1, 2, 3], 2) in runs and ([0, 1, 3], 2) in runs
    assert max(len(q) for q, _ in runs) == 3
    want = oracle_mod.run(n, gates)
    got = run_plan(ops, n, p.layout())
    assert np.max(np.abs(got - want)) < 1e-13


def test_diagonal_detector_respects_D(oracle_mod):
    n = 12
    gates = W.hadamard_diagonal_circuit(n, 200, seed=7)
    for D in (2, 4, 7, 12):
        p = qsim.Plan(n, gates, opt=qsim.OPT_DIAG, D=D)
        ops = p.ops()
        assert all(len(o["qubits"]) <= max(D, 2) for o in ops if o["kind"] == "DIAG")
        got = run_plan(ops, n, p.layout())
        assert np.max(np.abs(got - oracle_mod.run(n, gates))) < 1e-12


def test_diagonal_detector_visits_each_gate_once():
    """Sec. 4.5: every gate is placed exactly once, O(G)."""
    for n, g in ((20, W.diag_heavy(20, 500, 1)), (16, W.layered(16, 10, 2)), (10, W.random_mixed(10, 300, 3))):
        p = qsim.Plan(n, g, opt=qsim.OPT_DIAG)
        assert p.counters()["dd_visits"] == len(g)


# ---------------------------------------------------------------- merge booster (Sec. 4.4)
def worked_example_circuit():
    """8 qubits, 40 gates, with entanglement-free blocks of 6, 6, 7, 7 gates on
    the 2-qubit groups, 7 and 4 on the 4-qubit groups and 3 on all 8 (the
    per-block counts of the paper's example; the figure's circuit itself is
    not available)."""
    leaf = lambda a, b, extra: [Gate("H", (a,)), Gate("H", (b,)), Gate("CNOT", (a, b)), Gate("RZ", (a,), 0.3),
                                Gate("RX", (b,), 0.4), Gate("CZ", (a, b))] + extra
    g = leaf(0, 1, []) + leaf(2, 3, []) + leaf(4, 5, [Gate("RY", (4,), 0.5)]) + leaf(6, 7, [Gate("RY", (6,), 0.6)])
    g += [Gate("CNOT", (1, 2)), Gate("RX", (1,), 0.1), Gate("RX", (2,), 0.2), Gate("CZ", (0, 3)), Gate("H", (0,)),
          Gate("H", (3,)), Gate("CNOT", (0, 2))]
    g += [Gate("CNOT", (5, 6)), Gate("RX", (5,), 0.7), Gate("RY", (6,), 0.8), Gate("CZ", (4, 7))]
    g += [Gate("CNOT", (3, 4)), Gate("H", (3,)), Gate("CZ", (0, 7))]
    assert len(g) == 40
    return g


def test_booster_worked_example_counts(oracle_mod):
    """Sec. 4.4: 1,336 state accesses with the booster vs 40 x 2^8 = 10,240."""
    n = 8
    gates = worked_example_circuit()
    plain = qsim.Plan(n, gates, opt=0).ops()
    assert access_count(plain) == 40 * 2 ** 8 == 10240
    p = qsim.Plan(n, gates, opt=qsim.OPT_BOOST, B=4)
    ops = p.ops()
    assert access_count(ops) == (6 + 6 + 7 + 7) * 4 + (7 + 4) * 16 + 3 * 256 + 2 * 16 + 256 == 1336
    assert [o["buffer_qubits"] for o in ops if o["kind"] == "KRON"] == [4, 4, 8]
    assert np.max(np.abs(run_plan(ops, n, p.layout()) - oracle_mod.run(n, gates))) < 1e-13


def divider_leaves(n, B):
    """Leaf sizes of the plan's booster: sizes of the INIT'ed sub-states."""
    ops = qsim.Plan(n, [Gate("H", (0,))], opt=qsim.OPT_BOOST, B=B).ops()
    return [o["buffer_qubits"] for o in ops if o["kind"] == "INIT" and o["buffer"] != 0]


def test_divider_pins():
    for B in range(3, 8):
        assert divider_leaves(8, B) == [2, 2, 2, 2]  # ceil(8/B) = 2 or 3
    assert divider_leaves(30, 4) == [7, 8, 7, 8]
    assert divider_leaves(28, 4) == [7, 7, 7, 7]
    assert divider_leaves(5, 3) == [2, 1, 2]


def test_divider_32_qubits_two_16_halves():
    """Sec. 4.4: for 32 qubits the largest blocks are two 2^16 sub-states."""
    for B in range(2, 9):
        ops = qsim.Plan(32, [Gate("H", (0,))], opt=qsim.OPT_BOOST, B=B).ops()
        krons = [o for o in ops if o["kind"] == "KRON"]
        last = krons[-1]
        assert last["buffer"] == 0 and last["buffer_qubits"] == 32
        sizes = {o["buffer"]: o["buffer_qubits"] for o in ops if o["kind"] in ("INIT", "KRON")}
        assert sizes[last["src_lo"]] == 16 and sizes[last["src_hi"]] == 16


def test_booster_odd_queue_keeps_every_qubit(oracle_mod):
    """An unpaired trailing group is carried over (the literal listing would
    drop it): N=5, B=3 divides as [2, 1, 2]."""
    n = 5
    gates = W.random_mixed(n, 60, seed=4, max_k=2)
    p = qsim.Plan(n, gates, opt=qsim.OPT_BOOST, B=3)
    ops = p.ops()
    assert np.max(np.abs(run_plan(ops, n, p.layout()) - oracle_mod.run(n, gates))) < 1e-13


@pytest.mark.parametrize("n,B", [(n, B) for n in (4, 6, 9, 12, 13) for B in (2, 3, 4, 6)])
def test_booster_product_prefix(oracle_mod, n, B):
    gates = W.product_circuit(n, 3, seed=n) + W.layered(n, 2, seed=B)
    p = qsim.Plan(n, gates, opt=qsim.OPT_BOOST | qsim.OPT_STAGES | qsim.OPT_FUSE, B=B, C=min(10, n))
    ops = p.ops()
    assert np.max(np.abs(run_plan(ops, n, p.layout()) - oracle_mod.run(n, gates))) < 1e-12


def test_booster_linear_gate_accounting():
    """Sec. 4.4 complexity: the booster visits the gates of the circuit a
    bounded number of times per merge level (O(G) per level, log N levels)."""
    for n in (16, 24, 30):
        g = W.layered(n, 5, 1)
        p = qsim.Plan(n, g, opt=qsim.OPT_BOOST)
        c = p.counters()
        assert c["booster_gates"] <= len(g)
        assert c["booster_groups"] >= 2


def test_plan_time_small_fraction():
    """Sec. 4.2: the optimiser stays polynomial and cheap; the 30-qubit
    layered plan takes well under a second on the host."""
    n, g = W.config_circuit("layered30")
    p = qsim.Plan(n, g, opt=qsim.OPT_ALL)
    assert p.stats()["plan_ms"] < 1000


def test_invalid_gates_rejected():
    with pytest.raises(qsim.QsimError):
        qsim.Plan(3, [Gate("H", (3,))])
    with pytest.raises(qsim.QsimError):
        qsim.Plan(3, [Gate("CZ", (1, 1))])
    with pytest.raises(qsim.QsimError):
        qsim.Plan(3, [Gate("U", (0,), 0.0, np.array([[1, 1], [0, 1]], dtype=complex))])
    with pytest.raises(qsim.QsimError):
        qsim.Plan(3, [Gate("DIAG", (0,), 0.0, np.array([1, 2], dtype=complex))])


# ---------------------------------------------------------------- qubit reordering (Sec. 2.3)
def high_qubit_circuit(n, offset, layers_lo, layers_hi, seed):
    """Entangle every qubit, then work only on the top qubits (the always-local
    low bits are idle there, so moving hot qubits down pays)."""
    g = W.layered(n, layers_lo, seed)
    g += [Gate(x.kind, tuple(q + offset for q in x.qubits), x.theta, x.data)
          for x in W.layered(n - offset, layers_hi, seed + 1)]
    return g


def test_remap_emits_permutation_and_matches_oracle(oracle_mod):
    n = 14
    gates = high_qubit_circuit(n, 6, 2, 12, 5)
    # six fixed low qubits idle while the work sits on the top ones
    p = qsim.Plan(n, gates, opt=qsim.OPT_ALL, C=10, L=6)
    ops = p.ops()
    perms = [o for o in ops if o["kind"] == "PERM"]
    assert perms, "expected a qubit permutation"
    for o in perms:  # products of swaps of low (< 6) and high bits
        for src, dst in enumerate(o["perm"]):
            assert o["perm"][dst] == src
            if src != dst:
                assert (src < 6) != (dst < 6)
    assert p.layout() != list(range(n))
    want = oracle_mod.run(n, gates)
    assert np.max(np.abs(run_plan(ops, n, p.layout()) - want)) < 1e-12
    # fewer full passes than without reordering
    q = qsim.Plan(n, gates, opt=qsim.OPT_ALL & ~qsim.OPT_REMAP, C=10, L=6)
    assert p.stats()["full_passes"] < q.stats()["full_passes"]


def test_remap_free_relabel_at_start():
    """From |0...0> a relabelling costs nothing: no PERM op, layout changed."""
    n = 30
    gates = [Gate(x.kind, tuple(q + 10 for q in x.qubits), x.theta, x.data) for x in W.layered(20, 10, 3)]
    opt = qsim.OPT_STAGES | qsim.OPT_FUSE | qsim.OPT_REMAP
    p = qsim.Plan(n, gates, opt=opt, L=6)   # six fixed low qubits, all idle
    assert not [o for o in p.ops() if o["kind"] == "PERM"]
    assert p.layout() != list(range(n))
    q = qsim.Plan(n, gates, opt=qsim.OPT_STAGES | qsim.OPT_FUSE, L=6)
    assert p.stats()["full_passes"] < q.stats()["full_passes"]


def operator_path_circuit(n, seed):
    """Circuit whose stages need the stage kernel's rarer operator shapes:
    six-qubit diagonals (more than four selector bits), three- and four-qubit
    dense gates (whole register tile) and controlled gates on many qubits
    (block-diagonal operators with selectors)."""
    rng = np.random.default_rng(seed)
    gates = []
    for layer in range(3):
        for q in range(n):
            gates.append(Gate("U", (q,), data=W.haar_unitary(rng)))
        # six-qubit diagonals, mostly on high qubits (global or thread bits of
        # a stage, so most of their qubits select blocks), and a phase gate
        for _ in range(3):
            qs = [int(x) for x in rng.choice(np.arange(n // 4, n), 6, replace=False)]
            gates.append(Gate("DIAG", tuple(qs), data=np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << 6))))
        gates.append(Gate("CPHASE", (qs[0], qs[5]), theta=float(rng.uniform(0, 2 * np.pi))))
        for k in (3, 4):
            qk = tuple(int(x) for x in rng.choice(n, k, replace=False))
            gates.append(Gate("U", qk, data=W.haar_unitary(rng, 1 << k)))
        for _ in range(n):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append(Gate("CNOT", (a, b)))
            gates.append(Gate("CPHASE", (b, a), theta=float(rng.uniform(0, 2 * np.pi))))
    return gates


def test_operator_path_circuit_has_the_rare_shapes():
    """The circuit used by the GPU operator-path test produces stage-kernel
    operators with more than four selector bits (diagonal tables whose
    selector sources are read from memory), two-bit dense operators with
    selectors, and whole-register-tile dense operators."""
    n = 16
    opt = qsim.OPT_STAGES | qsim.OPT_FUSE | qsim.OPT_DIAG
    ops = qsim.Plan(n, operator_path_circuit(n, 3), opt=opt, C=12).ops()
    wide_sel = two_bit_sel = whole_tile = 0
    for o in ops:
        if o["kind"] != "STAGE":
            continue
        for k in o["kernel_ops"]:
            nsel = len(k["qubits"]) - k["n_register"]
            if k["diagonal"]:
                wide_sel += nsel > 4
            else:
                two_bit_sel += k["n_register"] == 2 and nsel > 0
                whole_tile += k["n_register"] == 4
    assert wide_sel > 0 and two_bit_sel > 0 and whole_tile > 0, (wide_sel, two_bit_sel, whole_tile)


def test_stage_partition_quality_layered30():
    """Regression guard for the stage partition: the 30-qubit layered circuit
    (2,680 gates) plans into at most 22 full-state passes with all passes on
    (the gate block search alone, taking local qubits in gate order, needs 30)."""
    n, gates = W.config_circuit("layered30")
    st = qsim.Plan(n, gates).stats()
    assert st["full_passes"] <= 22, st
    assert st["n_perm"] == 0


def test_premarshalled_circuit_plans_identically():
    """A `Circuit` (gates converted once) plans exactly like the gate list."""
    n, gates = 14, W.layered(14, 8, seed=3)
    a = qsim.Plan(n, gates).ops()
    circ = qsim.Circuit(gates)
    for _ in range(2):  # reusable
        b = qsim.Plan(n, circ).ops()
        assert [o["kind"] for o in a] == [o["kind"] for o in b]
        for x, y in zip(a, b):
            if x["kind"] == "STAGE":
                assert x["local"] == y["local"]
                assert len(x["kernel_ops"]) == len(y["kernel_ops"])
                for kx, ky in zip(x["kernel_ops"], y["kernel_ops"]):
                    assert np.array_equal(kx["payload"], ky["payload"])


def test_swap_gates_become_relabellings(oracle_mod):
    """With remapping on, a SWAP moves no data: the plan holds no op for it,
    later gates act on the exchanged qubits and the layout records where each
    logical qubit ended up (Sec. 2.3)."""
    n = 11
    gates = W.qft(n, 5) + W.random_mixed(n, 80, seed=6, max_k=3)
    n_swaps = sum(1 for g in gates if g.kind == "SWAP")
    assert n_swaps >= n // 2
    want = oracle_mod.run(n, gates)
    for opt in (qsim.OPT_ALL, qsim.OPT_REMAP | qsim.OPT_STAGES, qsim.OPT_STAGES, qsim.OPT_DIAG):
        p = qsim.Plan(n, gates, opt=opt, C=9)
        ops = p.ops()
        got = run_plan(ops, n, p.layout())
        assert np.max(np.abs(got - want)) < 1e-12, opt
        relabel = bool(opt & qsim.OPT_REMAP)
        assert (sorted(p.layout()) == list(range(n)))
        assert (p.layout() != list(range(n))) == relabel


def test_benchmark_family_plans_30q():
    """Plan sizes of the Sec. 5 benchmark families at 30 qubits (complex128):
    the all-pairs RZZ layer is one diagonal-only pass after the booster, the
    QFT's closing SWAPs cost nothing, and QAOA needs about three passes a level."""
    s = qsim.Plan(*W.config_circuit("rzz30")).stats()
    assert s["full_passes"] == 1 and s["n_kron"] == 1
    s = qsim.Plan(*W.config_circuit("qft30")).stats()
    assert s["full_passes"] <= 2 and s["n_perm"] == 0
    s = qsim.Plan(*W.config_circuit("qaoa30")).stats()
    assert s["full_passes"] <= 16 and s["n_perm"] == 0


def test_phase_diagonals_merge_into_wide_tables(oracle_mod):
    """Every diagonal of a register phase (narrow gates and detector outputs,
    on register, lane, wave or chunk qubits) folds into one table of up to 12
    selector qubits; the interpreted plan must still reproduce the oracle."""
    n = 16
    for gates in (W.qaoa_full(n, 2, 3), W.rzz_full(n, 4) + W.layered(n, 2, 5), W.qft(n, 6)):
        want = oracle_mod.run(n, gates)
        for dtype, C in (("c128", 10), ("c64", 11), ("c128", 12)):
            p = qsim.Plan(n, gates, dtype=dtype, C=C, opt=qsim.OPT_ALL & ~qsim.OPT_QUAD)
            ops = p.ops()
            widths = [len(k["qubits"]) for o in ops if o["kind"] == "STAGE"
                      for k in o["kernel_ops"] if k["diagonal"]]
            assert max(widths) >= 11
            for use_k in (True, False):
                got = run_plan(ops, n, p.layout(), use_kernel_ops=use_k)
                assert np.max(np.abs(got - want)) < 1e-12, (dtype, C, use_k)


@pytest.mark.parametrize("L", [1, 3, 4, 6])
def test_fixed_low_qubits_option(oracle_mod, L):
    """Every choice of always-local low qubits gives the oracle's state, and
    fewer fixed qubits never need more stage passes here."""
    n = 13
    gates = W.layered(n, 6, seed=L)
    want = oracle_mod.run(n, gates)
    p = qsim.Plan(n, gates, opt=qsim.OPT_ALL, C=10, L=L)
    ops = p.ops()
    for o in ops:
        if o["kind"] == "STAGE" and o["buffer"] == 0:
            assert set(range(L)) <= set(o["local"])
    assert np.max(np.abs(run_plan(ops, n, p.layout()) - want)) < 1e-12
    assert np.max(np.abs(run_plan(ops, n, p.layout(), use_kernel_ops=False) - want)) < 1e-12
    if L < 6:
        assert p.stats()["full_passes"] <= qsim.Plan(n, gates, opt=qsim.OPT_ALL, C=10, L=6).stats()["full_passes"]


# ---------------------------------------------------------------- host-memory offload plans
def _offload_cases(n):
    return [("layered", W.layered(n, 8, 21)), ("mixed", W.random_mixed(n, 160, seed=22, max_k=3)),
            ("qft", W.qft(n, 23)), ("hdiag", W.hadamard_diagonal_circuit(n, 120, 24)),
            ("qaoa", W.qaoa_full(n, 2, 25)),
            # controls and diagonals on the top qubits (outer bits of the windows)
            ("controls", [Gate("H", (q,)) for q in range(n)] +
             [Gate("CNOT", (n - 1 - (i % 3), i % (n - 3))) for i in range(3 * n)] +
             [Gate("CPHASE", (n - 1, i), theta=0.1 * (i + 1)) for i in range(n - 1)] +
             [Gate("RX", (n - 1,), theta=0.3), Gate("CZ", (0, n - 2))])]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_offload_plans_match_oracle(oracle_mod, dtype):
    """Host-memory offload: each pass fixes a contiguous range of outer
    qubits; the pass's stages (planned on the window) must reproduce the
    oracle's state, no stage may hold an outer qubit locally, and every
    dense operator's register qubits avoid the outer range."""
    n = 16
    Wq = 12 if dtype == "c128" else 13
    for name, gates in _offload_cases(n):
        want = oracle_mod.run(n, gates)
        p = qsim.Plan(n, gates, dtype=dtype, opt=qsim.OPT_ALL, offload_window=Wq)
        ops = p.ops()
        st = p.stats()
        assert p.layout() == list(range(n))
        assert ops[0]["kind"] == "WINDOW" and ops[0]["init"]
        i, passes = 0, 0
        while i < len(ops):
            w = ops[i]
            assert w["kind"] == "WINDOW", (name, i, w["kind"])
            assert w["outer_n"] == n - Wq
            outer = set(range(w["outer_lo"], w["outer_lo"] + w["outer_n"]))
            assert w["outer_lo"] >= (3 if dtype == "c128" else 4) and w["outer_lo"] + w["outer_n"] <= n
            for op in ops[i + 1:i + 1 + w["pass_ops"]]:
                assert op["kind"] in ("STAGE", "DENSE", "DIAG"), op["kind"]
                if op["kind"] == "STAGE":
                    assert not outer & set(op["local"]), (name, outer, op["local"])
                    for k in op["kernel_ops"]:
                        assert not outer & set(k["qubits"][:k["n_register"]])
                elif op["kind"] == "DENSE":
                    assert not outer & set(op["qubits"])
            i += 1 + w["pass_ops"]
            passes += 1
        assert st["offload_passes"] == passes and st["window_qubits"] == Wq
        amp = 16 if dtype == "c128" else 8
        assert st["pcie_bytes"] == (2 * passes - 1) * amp * 2 ** n
        got_k = run_plan(ops, n, p.layout())
        got_g = run_plan(ops, n, p.layout(), use_kernel_ops=False)
        assert np.max(np.abs(got_g - want)) < 1e-12, name
        assert np.max(np.abs(got_k - want)) < 1e-12, name


def test_offload_window_size_and_empty_circuit():
    n = 16
    p = qsim.Plan(n, [], opt=qsim.OPT_ALL, offload_window=12)
    ops = p.ops()
    assert [o["kind"] for o in ops] == ["WINDOW"] and ops[0]["init"] and ops[0]["pass_ops"] == 0
    # the largest window whose two copies fit the device bytes, at most n - 1
    assert qsim.Plan(n, [], opt=qsim.OPT_ALL, offload_window=15).stats()["window_qubits"] == 15
    assert qsim.Plan(n, [], opt=qsim.OPT_ALL, offload_window=16).stats()["window_qubits"] == 15


def brickwork(n, layers, seed):
    """Two-qubit Haar unitaries on neighbouring pairs, alternating offsets."""
    rng = np.random.default_rng(seed)
    gates = []
    for layer in range(layers):
        for a in range(layer % 2, n - 1, 2):
            gates.append(Gate("U", (a, a + 1), 0.0, W.haar_unitary(rng, 4)))
    return gates


@pytest.mark.parametrize("n", [11, 12])
def test_phase_cap_splits_the_stage(oracle_mod, n):
    """Every qubit local and a deep brickwork: a stage reaches the cap of 96
    register phases and the rest of the circuit moves to the next stage; the
    plan reproduces the oracle."""
    gates = brickwork(n, 150, 5)
    ops, got_k, got_g = plan_state(n, gates, opt=qsim.OPT_STAGES | qsim.OPT_FUSE)
    phases = [o["n_phases"] for o in ops if o["kind"] == "STAGE"]
    assert phases[:3] == [96, 96, 96] and len(phases) == 4
    want = oracle_mod.run(n, gates)
    assert np.max(np.abs(got_k - want)) < 1e-12
    assert np.max(np.abs(got_g - want)) < 1e-12


def test_quadratic_phase_operator_plans(oracle_mod):
    """Plans whose register phases turn one- and two-qubit diagonals into a
    quadratic-phase operator: the exported (term, angle) form, applied as
    e^{i phi(x)} by the interpreter, reproduces the oracle's state; without
    the option the same circuits keep diagonal tables."""
    for n, gates in ((16, W.rzz_full(16, 4)), (17, W.qft(17, 6))):
        want = oracle_mod.run(n, gates)
        for dtype in ("c128", "c64"):
            C = 12 if dtype == "c128" else 13
            p = qsim.Plan(n, gates, dtype=dtype, C=C)
            ops = p.ops()
            quads = [k for o in ops if o["kind"] == "STAGE" for k in o["kernel_ops"] if k.get("quad")]
            if dtype == "c128":
                assert quads, n
            for k in quads:
                codes = [c for c, _ in k["terms"]]
                assert codes[0] == -1 and len(set(codes)) == len(codes)
                assert all(c == -1 or (c // 64 <= c % 64 < n) for c in codes)
            assert np.max(np.abs(run_plan(ops, n, p.layout()) - want)) < 1e-12, (n, dtype)
            q = qsim.Plan(n, gates, dtype=dtype, C=C, opt=qsim.OPT_ALL & ~qsim.OPT_QUAD)
            assert not any(k.get("quad") for o in q.ops() if o["kind"] == "STAGE" for k in o["kernel_ops"])
