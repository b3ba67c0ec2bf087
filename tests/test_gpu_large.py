"""States of more than 2^32 amplitudes on one GPU: 33 qubits in complex128
(128 GiB), 34 qubits in complex64 (128 GiB) and complex128 (256 GiB), and 35
qubits in complex64 (256 GiB), through the C ABI.

Expected values come from closed forms evaluated per sampled index:

* a circuit whose gates each stay inside one of several disjoint qubit
  blocks leaves a product of block states, so a_x is the product of the
  oracle's small block states at the bits of x in each block;
* H on every qubit followed by diagonal gates (phase product);
* the QFT of a basis state (exact integer phase x0 y mod 2^N);
* sampling from the uniform state (x = floor(u 2^N) inside a cell).

Each test holds one large state at a time and frees it before the next.
"""
import math
import sys

import numpy as np
import pytest

from paper_2604_12256_amd import qsim
from paper_2604_12256_amd import workloads as W
from paper_2604_12256_amd.workloads import Gate

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_free(bytes_needed, margin=8 << 30):
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < bytes_needed + margin:
        pytest.skip(f"needs {bytes_needed / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")


def release(sim):
    import torch
    sim.close()
    del sim
    torch.cuda.empty_cache()


def block_product_circuit(n, blocks, seed):
    """Random gates of every kind, each inside one block (dense 1..6-qubit,
    diagonal, SWAP, CNOT), plus the block states computed by the oracle."""
    rng = np.random.default_rng(seed)
    gates, per_block = [], []
    for qs in blocks:
        k = len(qs)
        local = [Gate("H", (q,)) for q in range(k)] + W.random_mixed(k, 12, seed=int(rng.integers(1 << 30)),
                                                                    max_k=min(k, 6))
        per_block.append((qs, local))
    # interleave the blocks' gate lists
    i = 0
    while any(i < len(l) for _, l in per_block):
        for qs, l in per_block:
            if i < len(l):
                g = l[i]
                gates.append(Gate(g.kind, tuple(qs[q] for q in g.qubits), g.theta, g.data))
        i += 1
    return gates, per_block


def block_product_amplitudes(oracle_mod, per_block, idx):
    """Qubits in no block stay |0>: amplitudes with any of them set are 0."""
    idx = np.asarray(idx, dtype=np.uint64)
    covered = 0
    for qs, _ in per_block:
        for q in qs:
            covered |= 1 << q
    out = ((idx & ~np.uint64(covered)) == 0).astype(np.complex128)
    for qs, local in per_block:
        psi = oracle_mod.run(len(qs), local)
        y = np.zeros(idx.shape, dtype=np.int64)
        for t, q in enumerate(qs):
            y |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << t
        out *= psi[y]
    return out


def covered_indices(per_block, count, seed):
    """Seeded indices whose set bits all lie on block qubits (the nonzero
    part of the state), plus the extremes of that set."""
    qs = sorted(q for b, _ in per_block for q in b)
    r = np.random.default_rng(seed).integers(0, 1 << len(qs), size=count, dtype=np.uint64)
    out = np.zeros(count, dtype=np.uint64)
    for t, q in enumerate(qs):
        out |= ((r >> np.uint64(t)) & np.uint64(1)) << np.uint64(q)
    full = np.uint64(sum(1 << q for q in qs))
    return np.concatenate([out, np.array([0, full], dtype=np.uint64)])


BLOCKS33 = [(0, 1, 2, 3, 4, 5), (6, 13, 20, 27), (31, 32), (7, 8, 9), (29, 30, 12, 14, 15)]


@pytest.mark.parametrize("opt", [0, qsim.OPT_ALL])
def test_33q_block_product(oracle_mod, opt):
    """Every full-pass kernel (plain path: dense k = 1..6, diagonals) and the
    optimised path (booster tensor product, stages) on 2^33 amplitudes."""
    n = 33
    need_free(16 << n)
    gates, per_block = block_product_circuit(n, BLOCKS33, seed=5)
    idx = np.concatenate([covered_indices(per_block, 1 << 16, 31), W.sample_indices(n, 4096, 32),
                          np.array([(1 << n) - 1, 1 << 32, (1 << 32) - 1], dtype=np.uint64)])
    say(f"33q block product opt={opt}: {len(gates)} gates")
    sim = qsim.Simulator(n, opt=opt)
    sim.load(gates)
    sim.run()
    got = sim.amplitudes(idx)
    err = np.max(np.abs(got - block_product_amplitudes(oracle_mod, per_block, idx)))
    assert err <= TOL128, err
    assert abs(sim.norm() - 1) < 1e-11
    release(sim)


def test_33q_diagonal_and_qft_closed_forms():
    from oracle import closed_forms as CF
    n = 33
    need_free(16 << n)
    gates = W.hadamard_diagonal_circuit(n, 300, seed=12)
    idx = W.sample_indices(n, 1 << 16, 13)
    say("33q hadamard-diagonal")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    assert np.max(np.abs(sim.amplitudes(idx) - CF.hadamard_diagonal_amplitudes(n, gates, idx))) <= TOL128
    say("33q QFT")
    gates = W.qft(n, 8)
    x0 = CF.qft_input(n, gates)
    sim.load(gates)
    sim.run()
    r = np.array([(x0 * int(y)) % (1 << n) for y in idx], dtype=np.float64)
    want = 2.0 ** (-n / 2) * np.exp(2j * math.pi * (r / float(1 << n)))
    assert np.max(np.abs(sim.amplitudes(idx) - want)) <= TOL128
    release(sim)


def test_33q_measurement():
    n = 33
    need_free(16 << n)
    say("33q uniform sampling and Z strings")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load([Gate("H", (q,)) for q in range(n)])
    sim.run()
    rng = np.random.default_rng(7)
    k = rng.integers(0, 1 << n, size=50000, dtype=np.uint64)
    np.testing.assert_array_equal(sim.sample((k.astype(np.float64) + 0.5) / float(1 << n)), k)
    np.testing.assert_allclose(sim.expect_z([0, 1, 1 << 32, (1 << n) - 1]), [1, 0, 0, 0], atol=1e-12)
    m, p = sim.measure(32, 0.75)
    assert m == 1 and abs(p - 0.5) < 1e-12
    assert abs(sim.norm() - 1) < 1e-11
    # marginals and Z strings over qubits above bit 31 after the collapse
    # (indices of 2^31 and above on both marginal paths)
    np.testing.assert_allclose(sim.probabilities([6, 32]), [0, 0, 0.5, 0.5], atol=1e-12)
    np.testing.assert_allclose(sim.probabilities([32, 31]), [0, 0.5, 0, 0.5], atol=1e-12)
    np.testing.assert_allclose(sim.probabilities([0, 32]), [0, 0, 0.5, 0.5], atol=1e-12)
    np.testing.assert_allclose(sim.expect_z([1 << 32, (1 << 32) | (1 << 31), 1 << 31]), [-1, 0, 0], atol=1e-12)
    amp = sim.amplitudes(np.array([0, 1 << 32, (1 << n) - 1], dtype=np.uint64))
    assert abs(amp[0]) == 0 and abs(amp[1] - 2.0 ** (-(n - 1) / 2)) < 1e-15
    release(sim)


def test_34q_complex64_block_product(oracle_mod):
    n = 34
    need_free(8 << n)
    blocks = [(0, 1, 2, 3), (33, 32, 5), (10, 20, 30), (6, 7)]
    gates, per_block = block_product_circuit(n, blocks, seed=9)
    idx = np.concatenate([covered_indices(per_block, 1 << 16, 33), W.sample_indices(n, 4096, 34)])
    say(f"34q complex64 block product: {len(gates)} gates")
    sim = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    got = sim.amplitudes(idx)
    want = block_product_amplitudes(oracle_mod, per_block, idx)
    assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(want)) + 1e-9
    release(sim)


def test_34q_complex128_diagonal_closed_form():
    """A 256 GiB complex128 state (most of the device): H on every qubit and
    the fully-connected RZZ layer, against the diagonal closed form."""
    from oracle import closed_forms as CF
    n = 34
    need_free(16 << n, margin=3 << 30)
    gates = W.rzz_full(n, 7)
    idx = W.sample_indices(n, 1 << 14, 35)
    say(f"34q complex128 fully-connected RZZ: {len(gates)} gates")
    sim = qsim.Simulator(n, opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    assert np.max(np.abs(sim.amplitudes(idx) - CF.hadamard_diagonal_amplitudes(n, gates, idx))) <= TOL128
    np.testing.assert_allclose(sim.expect_z([0, 1 << 33]), [1, 0], atol=1e-12)
    release(sim)


def test_35q_complex64_diagonal_closed_form():
    """The largest resident state: 35 qubits in complex64 (256 GiB). H on
    every qubit and the fully-connected RZZ layer against the diagonal closed
    form on sampled indices, then marginals and Z strings over the top qubit."""
    from oracle import closed_forms as CF
    n = 35
    need_free(8 << n, margin=3 << 30)
    gates = W.rzz_full(n, 7)
    idx = W.sample_indices(n, 1 << 14, 36)
    say(f"35q complex64 fully-connected RZZ: {len(gates)} gates")
    sim = qsim.Simulator(n, dtype="c64", opt=qsim.OPT_ALL)
    sim.load(gates)
    sim.run()
    want = CF.hadamard_diagonal_amplitudes(n, gates, idx)
    got = sim.amplitudes(idx)
    assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(want))
    assert abs(sim.norm() - 1) < 1e-5
    np.testing.assert_allclose(sim.probabilities([34, 0]), [0.25] * 4, atol=1e-6)
    np.testing.assert_allclose(sim.expect_z([0, 1 << 34, (1 << 34) | (1 << 31)]), [1, 0, 0], atol=1e-6)
    release(sim)
