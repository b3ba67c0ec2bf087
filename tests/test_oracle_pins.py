"""Pins of the CPU oracle against facts fixed outside the oracle itself.

* Gate matrices: identities of the Pauli algebra and matrix exponentials of
  the generators (scipy.linalg.expm), not a retyped formula.
* Gate application and bit order (Sec. 2.2): the 2^N x 2^N lift built with
  numpy.kron exactly as the paper writes it for one qubit,
  U_j = I^{(N-j-1)} (x) U (x) I^{(j)}, and for adjacent two-qubit gates,
  plus an entry-by-entry lift for arbitrary placements.
* Closed forms: H^{(x)N}|0> uniform, GHZ, X masks, SWAP as the bit exchange of
  Eq. (swap gate) in Sec. 2.3.
* Invariants: norm preservation, C * C^-1 = identity.
* Reductions: marginals, norm and inner product against numpy.
* Benchmark families of Sec. 5 (fully-connected RZZ, QFT, QAOA): the QFT
  circuit against numpy's inverse FFT on random states, and the closed forms
  used at 30 qubits against the full oracle, special cases and a second
  derivation.
* Measurement (Sec. 2's projective model): collapse against the literal
  kron lift of the projector |i><i| on qubit j; sampling against closed
  forms (uniform, GHZ, basis states) and brute-force interval counting;
  Z-string expectations against the kron lift of Pauli Z and product-state
  closed forms.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.linalg import expm

from paper_2604_12256_amd import workloads as W
from paper_2604_12256_amd.workloads import Gate

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)  # |1><1|
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)  # |0><0|


def kron2(hi, lo):
    """Two-qubit operator with ``hi`` on matrix bit 1 and ``lo`` on bit 0."""
    return np.kron(hi, lo)


# ---------------------------------------------------------------- gate matrices
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, math.pi, 5.9])
def test_rotation_matrices_are_generator_exponentials(oracle_mod, theta):
    O = oracle_mod
    np.testing.assert_allclose(O.gate_matrix(Gate("RX", (0,), theta)), expm(-0.5j * theta * X), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix(Gate("RY", (0,), theta)), expm(-0.5j * theta * Y), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix(Gate("RZ", (0,), theta)), expm(-0.5j * theta * Z), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix(Gate("RZZ", (0, 1), theta)),
                               expm(-0.5j * theta * kron2(Z, Z)), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix(Gate("CPHASE", (0, 1), theta)),
                               expm(1j * theta * kron2(P1, P1)), atol=1e-15)


def test_fixed_gates_from_pauli_identities(oracle_mod):
    O = oracle_mod
    m = lambda k, q=(0,): O.gate_matrix(Gate(k, q))
    np.testing.assert_allclose(m("X"), X, atol=0)
    np.testing.assert_allclose(m("Y"), Y, atol=0)
    np.testing.assert_allclose(m("Z"), Z, atol=0)
    np.testing.assert_allclose(m("H"), (X + Z) / math.sqrt(2), atol=1e-16)
    np.testing.assert_allclose(m("SX") @ m("SX"), X, atol=1e-16)
    # SX = e^{i pi/4} RX(pi/2)
    np.testing.assert_allclose(m("SX"), np.exp(0.25j * math.pi) * expm(-0.25j * math.pi * X), atol=1e-15)
    np.testing.assert_allclose(m("S") @ m("S"), Z, atol=1e-16)
    np.testing.assert_allclose(m("T") @ m("T"), m("S"), atol=1e-15)
    # two-qubit: bit 0 <-> q[0], bit 1 <-> q[1]; CNOT(control=q[0], target=q[1])
    np.testing.assert_allclose(m("CZ", (0, 1)), expm(1j * math.pi * kron2(P1, P1)), atol=1e-15)
    np.testing.assert_allclose(m("CNOT", (0, 1)), kron2(I2, P0) + kron2(X, P1), atol=0)
    sw = m("SWAP", (0, 1))
    a, b = np.array([0.6, 0.8j]), np.array([0.28, 0.96])
    np.testing.assert_allclose(sw @ np.kron(a, b), np.kron(b, a), atol=1e-16)
    np.testing.assert_allclose(O.gate_matrix(Gate("CPHASE", (0, 1), math.pi)), m("CZ", (0, 1)), atol=1e-15)


def test_all_named_matrices_unitary(oracle_mod):
    for kind in sorted(W.ONE_QUBIT_KINDS):
        u = oracle_mod.gate_matrix(Gate(kind, (0,), 0.77))
        np.testing.assert_allclose(u.conj().T @ u, np.eye(2), atol=1e-15)
    for kind in sorted(W.TWO_QUBIT_KINDS):
        u = oracle_mod.gate_matrix(Gate(kind, (0, 1), 0.77))
        np.testing.assert_allclose(u.conj().T @ u, np.eye(4), atol=1e-15)


# ---------------------------------------------------------------- lifting / bit order
def lift_single_paper(n, j, u):
    """U_j = I^{(N-j-1)} (x) U (x) I^{(j)} (Sec. 2.2), literal numpy.kron."""
    return np.kron(np.kron(np.eye(1 << (n - j - 1)), u), np.eye(1 << j))


def lift_entrywise(n, qubits, m):
    """Entry (x, y) of the lift is M[r(x), r(y)] when x and y agree off the
    gate qubits, else 0; r(x) collects bit qubits[t] of x into bit t."""
    dim = 1 << n
    mask = 0
    for q in qubits:
        mask |= 1 << q
    out = np.zeros((dim, dim), dtype=np.complex128)
    for x in range(dim):
        rx = sum(((x >> q) & 1) << t for t, q in enumerate(qubits))
        for y in range(dim):
            if (x & ~mask) != (y & ~mask):
                continue
            ry = sum(((y >> q) & 1) << t for t, q in enumerate(qubits))
            out[x, y] = m[rx, ry]
    return out


def random_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("kind", sorted(W.ONE_QUBIT_KINDS) + ["U"])
def test_single_qubit_lift_matches_paper_kron(oracle_mod, kind):
    n = 5
    rng = np.random.default_rng(11)
    for j in range(n):
        data = W.haar_unitary(rng) if kind == "U" else None
        g = Gate(kind, (j,), 1.234, data)
        psi = random_state(n, 100 + j)
        want = lift_single_paper(n, j, oracle_mod.gate_matrix(g)) @ psi
        got = oracle_mod.apply(n, [g], psi)
        np.testing.assert_allclose(got, want, atol=1e-14, rtol=0)


@pytest.mark.parametrize("kind", sorted(W.TWO_QUBIT_KINDS))
def test_adjacent_two_qubit_lift_matches_paper_layout(oracle_mod, kind):
    """Sec. 2.2: V on qubits j > k, rows ordered |b_j b_k> = 00, 01, 10, 11;
    for an adjacent ascending pair (k, k+1) the lift is I (x) V (x) I."""
    n = 5
    for k in range(n - 1):
        g = Gate(kind, (k, k + 1), 0.913)
        v = oracle_mod.gate_matrix(g)
        lift = np.kron(np.kron(np.eye(1 << (n - k - 2)), v), np.eye(1 << k))
        psi = random_state(n, 7 + k)
        np.testing.assert_allclose(oracle_mod.apply(n, [g], psi), lift @ psi, atol=1e-14, rtol=0)


def test_every_placement_matches_entrywise_lift(oracle_mod):
    n = 4
    rng = np.random.default_rng(5)
    for k in (1, 2, 3):
        for qs in itertools.permutations(range(n), k):
            for kind in ("U", "DIAG"):
                if kind == "U":
                    data = W.haar_unitary(rng, 1 << k)
                else:
                    data = np.exp(1j * rng.uniform(0, 2 * math.pi, 1 << k))
                g = Gate(kind, tuple(qs), 0.0, data)
                m = oracle_mod.gate_matrix(g)
                psi = random_state(n, sum(qs) + 31 * k)
                np.testing.assert_allclose(oracle_mod.apply(n, [g], psi),
                                           lift_entrywise(n, qs, m) @ psi, atol=1e-14, rtol=0)
    for kind in sorted(W.TWO_QUBIT_KINDS):
        for qs in itertools.permutations(range(n), 2):
            g = Gate(kind, qs, 2.2)
            psi = random_state(n, 3)
            np.testing.assert_allclose(oracle_mod.apply(n, [g], psi),
                                       lift_entrywise(n, qs, oracle_mod.gate_matrix(g)) @ psi,
                                       atol=1e-14, rtol=0)


def test_five_and_six_qubit_gates(oracle_mod):
    n = 6
    rng = np.random.default_rng(9)
    for k in (5, 6):
        qs = tuple(int(x) for x in rng.permutation(n)[:k])
        g = Gate("U", qs, 0.0, W.haar_unitary(rng, 1 << k))
        psi = random_state(n, k)
        np.testing.assert_allclose(oracle_mod.apply(n, [g], psi),
                                   lift_entrywise(n, qs, g.data) @ psi, atol=1e-14, rtol=0)


def test_random_circuit_matches_kron_product(oracle_mod):
    n = 5
    gates = W.random_mixed(n, 60, seed=4, max_k=3)
    full = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        full = lift_entrywise(n, g.qubits, oracle_mod.gate_matrix(g)) @ full
    np.testing.assert_allclose(oracle_mod.run(n, gates), full[:, 0], atol=1e-13, rtol=0)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 3, 8, 12])
def test_hadamard_all_gives_uniform(oracle_mod, n):
    s = oracle_mod.run(n, [Gate("H", (q,)) for q in range(n)])
    np.testing.assert_allclose(s, np.full(1 << n, 2.0 ** (-n / 2)), atol=1e-15)


@pytest.mark.parametrize("n", [2, 5, 10])
def test_ghz(oracle_mod, n):
    gates = [Gate("H", (0,))] + [Gate("CNOT", (q, q + 1)) for q in range(n - 1)]
    s = oracle_mod.run(n, gates)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(s, want, atol=1e-15)


def test_x_mask_gives_basis_state(oracle_mod):
    n = 9
    for mask in (0, 1, 0b101010101, (1 << n) - 1, 0b100000000):
        gates = [Gate("X", (q,)) for q in range(n) if (mask >> q) & 1]
        s = oracle_mod.run(n, gates)
        want = np.zeros(1 << n, dtype=np.complex128)
        want[mask] = 1
        np.testing.assert_array_equal(s, want)


def test_swap_is_bit_exchange(oracle_mod):
    """Eq. (swap gate): amplitudes |..1_i..0_j..> and |..0_i..1_j..> trade
    places, every other amplitude stays."""
    n = 6
    psi = random_state(n, 77)
    for i, j in itertools.permutations(range(n), 2):
        got = oracle_mod.apply(n, [Gate("SWAP", (i, j))], psi)
        idx = np.arange(1 << n)
        bi, bj = (idx >> i) & 1, (idx >> j) & 1
        perm = idx ^ (((bi ^ bj) << i) | ((bi ^ bj) << j))
        np.testing.assert_array_equal(got, psi[perm])


# ---------------------------------------------------------------- invariants
def inverse_circuit(gates):
    inv = []
    for g in reversed(gates):
        if g.kind in ("RX", "RY", "RZ", "CPHASE", "RZZ"):
            inv.append(Gate(g.kind, g.qubits, -g.theta))
        elif g.kind in ("H", "X", "Y", "Z", "CZ", "CNOT", "SWAP"):
            inv.append(g)
        elif g.kind == "S":
            inv += [g, g, g]
        elif g.kind == "T":
            inv += [g] * 7
        elif g.kind == "SX":
            inv += [g, g, g]
        elif g.kind == "U":
            inv.append(Gate("U", g.qubits, 0.0, np.ascontiguousarray(g.data.conj().T)))
        elif g.kind == "DIAG":
            inv.append(Gate("DIAG", g.qubits, 0.0, np.ascontiguousarray(g.data.conj())))
        else:
            raise AssertionError(g.kind)
    return inv


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_circuit_times_inverse_is_identity(oracle_mod, seed):
    n = 10
    gates = W.random_mixed(n, 300, seed=seed, max_k=4)
    s = oracle_mod.run(n, gates + inverse_circuit(gates))
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = 1
    np.testing.assert_allclose(s, want, atol=1e-13)


def test_norm_preserved_layered(oracle_mod):
    n, gates = W.config_circuit("layered12")
    s = oracle_mod.run(n, gates)
    assert abs(oracle_mod.norm(s) - 1.0) < 1e-13
    assert abs(np.sum(np.abs(s) ** 2) - 1.0) < 1e-13


def test_generated_unitaries_are_unitary():
    rng = np.random.default_rng(0)
    for d in (2, 4, 8, 32):
        for _ in range(5):
            u = W.haar_unitary(rng, d)
            assert np.max(np.abs(u.conj().T @ u - np.eye(d))) < 1e-14


# ---------------------------------------------------------------- reductions
def test_marginal_norm_inner_against_numpy(oracle_mod):
    n = 11
    psi = oracle_mod.run(n, W.random_mixed(n, 80, seed=12, max_k=3))
    p = np.abs(psi) ** 2
    assert abs(oracle_mod.norm(psi) - np.sum(p)) < 1e-14
    phi = random_state(n, 5)
    np.testing.assert_allclose(oracle_mod.inner(psi, phi), np.vdot(psi, phi), atol=1e-14)
    tens = p.reshape([2] * n)  # axis a <-> qubit n-1-a
    for qs in ([0], [3], [10, 0], [2, 7, 5], list(range(n))):
        got = oracle_mod.marginal(psi, qs)
        keep = [n - 1 - q for q in qs]
        other = tuple(a for a in range(n) if a not in keep)
        m = tens.sum(axis=other)  # remaining axes in ascending axis order
        order = sorted(keep)
        # y bit t <-> qubit qs[t]; axis order sorted(keep) is descending qubit
        want = np.zeros(1 << len(qs))
        for y in range(1 << len(qs)):
            ix = tuple((y >> qs.index(n - 1 - a)) & 1 for a in order)
            want[y] = m[ix]
        np.testing.assert_allclose(got, want, atol=1e-15)
    assert oracle_mod.marginal(psi, [])[0] == pytest.approx(1.0, abs=1e-13)


def test_marginal_independent_of_thread_count(oracle_mod):
    """The oracle's marginals are bitwise the same for any OpenMP thread
    count (fixed parts combined in a fixed order)."""
    n = 14
    psi = oracle_mod.run(n, W.random_mixed(n, 60, seed=21, max_k=2))
    before = oracle_mod.num_threads()
    outs = []
    try:
        for t in (1, 3, 8):
            oracle_mod.set_threads(t)
            outs.append(oracle_mod.marginal(psi, [13, 0, 6, 9]))
    finally:
        oracle_mod.set_threads(before)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_infidelity(oracle_mod):
    a = random_state(6, 1)
    assert abs(oracle_mod.infidelity(a, a * np.exp(0.3j))) < 1e-14
    b = random_state(6, 2)
    want = 1 - abs(np.vdot(a, b)) ** 2
    assert abs(oracle_mod.infidelity(a, b) - want) < 1e-14


def test_invalid_circuits_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.run(3, [Gate("H", (3,))])
    with pytest.raises(ValueError):
        oracle_mod.run(3, [Gate("CZ", (1, 1))])


# ---------------------------------------------------------------- closed-form helpers
def test_closed_forms_against_full_oracle(oracle_mod):
    from oracle import closed_forms as CF
    n = 10
    idx = np.arange(1 << n, dtype=np.uint64)
    g = W.product_circuit(n, 6, seed=3)
    np.testing.assert_allclose(CF.product_state_amplitudes(n, g, idx), oracle_mod.run(n, g), atol=1e-14)
    g2 = W.hadamard_diagonal_circuit(n, 120, seed=4)
    np.testing.assert_allclose(CF.hadamard_diagonal_amplitudes(n, g2, idx), oracle_mod.run(n, g2), atol=1e-14)


# ---------------------------------------------------------------- benchmark families (Sec. 5)
def _qft_only(n, seed):
    g = W.qft(n, seed)
    return g[sum(1 for x in g if x.kind == "X"):] if g and g[0].kind == "X" else g


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_qft_circuit_is_inverse_dft(oracle_mod, n):
    """The QFT maps a to sqrt(2^n) * ifft(a) (numpy's convention
    ifft(a)[y] = 2^-n sum_x a_x exp(2 pi i x y / 2^n)), on random states."""
    gates = [g for g in _qft_only(n, 0) if g.kind != "X"]
    assert sum(1 for g in gates if g.kind == "H") == n
    for seed in range(3):
        psi = random_state(n, 40 + seed)
        got = oracle_mod.apply(n, gates, psi)
        np.testing.assert_allclose(got, math.sqrt(1 << n) * np.fft.ifft(psi), atol=1e-13)


def test_qft_closed_form_against_oracle(oracle_mod):
    from oracle import closed_forms as CF
    for n in range(1, 10):
        for seed in range(3):
            g = W.qft(n, seed)
            x0 = CF.qft_input(n, g)
            assert x0 == W.qft_input_index(n, seed)
            want = oracle_mod.run(n, g)
            got = CF.qft_amplitudes(n, x0, np.arange(1 << n, dtype=np.uint64))
            assert np.max(np.abs(got - want)) < 1e-13, (n, seed)


def test_rzz_full_against_diagonal_closed_form(oracle_mod):
    from oracle import closed_forms as CF
    for n in (2, 5, 9):
        g = W.rzz_full(n, seed=n)
        assert len(g) == n + n * (n - 1) // 2
        idx = np.arange(1 << n, dtype=np.uint64)
        np.testing.assert_allclose(CF.hadamard_diagonal_amplitudes(n, g, idx), oracle_mod.run(n, g), atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 6, 10])
def test_qaoa_symmetric_form_against_oracle(oracle_mod, n):
    from oracle import closed_forms as CF
    for levels, seed in ((1, 0), (3, n), (5, 9)):
        g = W.qaoa_full(n, levels, seed)
        want = oracle_mod.run(n, g)
        got = CF.qaoa_amplitudes(n, g, np.arange(1 << n, dtype=np.uint64))
        assert np.max(np.abs(got - want)) < 1e-13, (n, levels)


def _qaoa_circuit(n, gammas, betas):
    g = [Gate("H", (q,)) for q in range(n)]
    for gm, bt in zip(gammas, betas):
        g += [Gate("RZZ", (i, j), gm) for i in range(n) for j in range(i + 1, n)]
        g += [Gate("RX", (q,), bt) for q in range(n)]
    return g


def test_qaoa_symmetric_form_special_cases():
    """beta = 0 leaves H^n plus diagonals (the diagonal closed form); gamma = 0
    leaves |+>^n, an eigenvector of every RX(b) with eigenvalue exp(-i b/2)."""
    from oracle import closed_forms as CF
    n = 7
    idx = np.arange(1 << n, dtype=np.uint64)
    g = _qaoa_circuit(n, [0.4, 1.1], [0.0, 0.0])
    diag_only = [x for x in g if x.kind != "RX"]
    np.testing.assert_allclose(CF.qaoa_amplitudes(n, g, idx), CF.hadamard_diagonal_amplitudes(n, diag_only, idx),
                               atol=1e-15)
    betas = [0.3, 2.2, 1.0]
    g = _qaoa_circuit(n, [0.0, 0.0, 0.0], betas)
    want = 2.0 ** (-n / 2) * np.exp(-0.5j * n * sum(betas))
    np.testing.assert_allclose(CF.qaoa_amplitudes(n, g, idx), np.full(1 << n, want), atol=1e-15)


def test_qaoa_30_qubits_two_derivations():
    """The weight-class amplitudes at 30 qubits (the size they are used at)
    against a second derivation: the RX layer as exp(-i beta J_x) with J_x the
    collective spin operator, tridiagonal in the normalised Dicke basis
    (<D_{w+1}| J_x |D_w> = sqrt((w + 1)(n - w)) / 2), exponentiated by eigh."""
    from oracle import closed_forms as CF
    n = 30
    g = W.qaoa_full(n, 5, 9)
    w = np.arange(n + 1)
    binom = np.array([math.comb(n, k) for k in range(n + 1)], dtype=np.float64)
    off = 0.5 * np.sqrt((w[:-1] + 1.0) * (n - w[:-1]))
    ev, V = np.linalg.eigh(np.diag(off, 1) + np.diag(off, -1))
    gammas, betas = W.qaoa_angles(5, 9)
    d = np.full(n + 1, 2.0 ** (-n / 2.0), dtype=np.complex128) * np.sqrt(binom)
    for gm, bt in zip(gammas, betas):
        s = (n - 2 * w).astype(np.float64)
        d = d * np.exp(-0.5j * gm * (s * s - n) / 2.0)
        d = V @ (np.exp(-1j * bt * ev) * (V.T @ d))
    c = CF.qaoa_weights(n, g)
    assert np.max(np.abs(c - d / np.sqrt(binom))) < 1e-13
    assert abs(np.sum(binom * np.abs(c) ** 2) - 1.0) < 1e-11


def test_qaoa_form_rejects_other_circuits():
    from oracle import closed_forms as CF
    g = W.qaoa_full(5, 2, 1)
    with pytest.raises(ValueError):
        CF.qaoa_weights(5, g[:-1])
    bad = list(g)
    bad[7] = Gate("RZZ", bad[7].qubits, bad[7].theta + 0.1)
    with pytest.raises(ValueError):
        CF.qaoa_weights(5, bad)


# ---------------------------------------------------------------- measurement (Sec. 2)
def test_collapse_matches_paper_projector(oracle_mod):
    from oracle import measure as M
    n = 5
    proj = [np.array([[1, 0], [0, 0]], dtype=np.complex128), np.array([[0, 0], [0, 1]], dtype=np.complex128)]
    for seed in range(4):
        psi = random_state(n, 60 + seed)
        for j in range(n):
            for u in (0.05, 0.5, 0.95):
                m, p, out = M.measure(psi, j, u)
                lifted = [lift_single_paper(n, j, proj[i]) @ psi for i in (0, 1)]
                probs = [float(np.vdot(v, v).real) for v in lifted]
                assert m == (0 if u < probs[0] else 1)
                assert abs(p - probs[m]) < 1e-14
                np.testing.assert_allclose(out, lifted[m] / np.sqrt(probs[m]), atol=1e-14)


def test_collapse_closed_forms(oracle_mod):
    from oracle import measure as M
    n = 6
    ghz = np.zeros(1 << n, dtype=np.complex128)
    ghz[0] = ghz[-1] = 1 / math.sqrt(2)
    for q in range(n):
        m, p, out = M.measure(ghz, q, 0.3)
        assert (m, abs(p - 0.5) < 1e-15) == (0, True) and abs(out[0] - 1) < 1e-15
        m, p, out = M.measure(ghz, q, 0.7)
        assert m == 1 and abs(out[-1] - 1) < 1e-15
    # product state: qubit q's factor becomes the basis vector of the outcome
    from oracle import closed_forms as CF
    g = W.product_circuit(n, 3, seed=12)
    f = CF.product_state_factors(n, g)
    psi = oracle_mod.run(n, g)
    m, p, out = M.measure(psi, 2, 0.4)
    assert abs(p - abs(f[2][m]) ** 2) < 1e-14
    f2 = f.copy()
    f2[2] = 0
    f2[2][m] = f[2][m] / abs(f[2][m])
    idx = np.arange(1 << n, dtype=np.uint64)
    want = np.ones(1 << n, dtype=np.complex128)
    for q in range(n):
        want *= f2[q][((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64)]
    np.testing.assert_allclose(out, want, atol=1e-14)


def test_sampling_closed_forms():
    from oracle import measure as M
    n = 8
    uni = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    k = np.arange(1 << n)
    np.testing.assert_array_equal(M.sample(uni, (k + 0.5) / (1 << n)), k)
    np.testing.assert_array_equal(M.sample(uni, k / (1 << n)), k)
    ghz = np.zeros(1 << n, dtype=np.complex128)
    ghz[0] = ghz[-1] = 1 / math.sqrt(2)
    np.testing.assert_array_equal(M.sample(ghz, [0.0, 0.2, 0.4999, 0.5, 0.9]), [0, 0, 0, (1 << n) - 1, (1 << n) - 1])
    basis = np.zeros(1 << n, dtype=np.complex128)
    basis[77] = 1j
    np.testing.assert_array_equal(M.sample(basis, np.linspace(0, 0.999, 50)), np.full(50, 77))


def test_sampling_by_interval_counting():
    """On a sparse random state, every u lands on the index whose cumulative
    interval [c_{x-1}, c_x) holds u T (brute force per index), and never on a
    zero-probability index."""
    from oracle import measure as M
    rng = np.random.default_rng(3)
    n = 6
    psi = random_state(n, 70)
    psi[rng.random(1 << n) < 0.4] = 0
    p = np.abs(psi) ** 2
    u = (np.arange(4000) + 0.5) / 4000
    got = M.sample(psi, u)
    T = p.sum()
    for i, x in enumerate(got):
        lo = sum(p[:x])
        assert p[x] > 0 and lo <= u[i] * T + 1e-15 and u[i] * T < lo + p[x] + 1e-15


def test_expect_z_against_pauli_lift(oracle_mod):
    from oracle import measure as M
    n = 5
    Zm = np.diag([1.0, -1.0])
    for seed in range(3):
        psi = random_state(n, 80 + seed)
        masks = [0, 1, 0b10110, (1 << n) - 1, 0b01001]
        for m, val in zip(masks, M.expect_z(psi, masks)):
            op = np.eye(1)
            for q in range(n - 1, -1, -1):  # kron order: qubit n-1 is the leftmost factor (Sec. 2.2)
                op = np.kron(op, Zm if (m >> q) & 1 else np.eye(2))
            assert abs(val - np.vdot(psi, op @ psi).real) < 1e-13
    # product states: the expectation factorises
    from oracle import closed_forms as CF
    g = W.product_circuit(n, 3, seed=4)
    f = CF.product_state_factors(n, g)
    psi = oracle_mod.run(n, g)
    for m in (0b1, 0b10101, 0b11111):
        want = np.prod([abs(f[q][0]) ** 2 - abs(f[q][1]) ** 2 for q in range(n) if (m >> q) & 1])
        assert abs(M.expect_z(psi, [m])[0] - want) < 1e-13


def test_expect_diagonal_against_marginal(oracle_mod):
    from oracle import measure as M
    n = 7
    psi = random_state(n, 90)
    qs = [5, 1, 3]
    f = np.random.default_rng(1).standard_normal(8)
    assert abs(M.expect_diagonal(psi, qs, f) - float(np.dot(oracle_mod.marginal(psi, qs), f))) < 1e-14


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_transposed_operand(oracle_mod):
    """A transposed gate matrix (a plausible marshalling slip) must be caught
    by the lift comparison."""
    n = 3
    rng = np.random.default_rng(1)
    u = W.haar_unitary(rng)
    psi = random_state(n, 2)
    good = oracle_mod.apply(n, [Gate("U", (1,), 0.0, u)], psi)
    bad = oracle_mod.apply(n, [Gate("U", (1,), 0.0, np.ascontiguousarray(u.T))], psi)
    want = lift_single_paper(n, 1, u) @ psi
    assert np.max(np.abs(good - want)) < 1e-14
    assert np.max(np.abs(bad - want)) > 1e-3


def test_pins_catch_wrong_bit_order():
    """Reversing the qubit order of a non-symmetric two-qubit gate changes the
    result, so the layout pins above are sensitive to it."""
    from oracle import oracle as O
    n = 3
    psi = random_state(n, 9)
    a = O.apply(n, [Gate("CNOT", (0, 2))], psi)
    b = O.apply(n, [Gate("CNOT", (2, 0))], psi)
    assert np.max(np.abs(a - b)) > 1e-3
