"""Seeded synthetic circuit generators.

This module only draws random circuits; it holds none of the simulator's
arithmetic (no gate matrices for named gates, no state updates).  Both the
GPU path and the CPU oracle consume its output, each through its own
marshalling code.

A circuit is a list of :class:`Gate`.  ``kind`` is a gate name, ``qubits`` the
ordered qubit list (bit t of the gate's matrix index corresponds to
``qubits[t]``), ``theta`` the angle of a parametrised gate and ``data`` an
explicit complex matrix (kind ``"U"``: 2^k x 2^k, row-major) or diagonal
(kind ``"DIAG"``: 2^k entries).

Gate names: H X Y Z S T SX RX RY RZ CZ CNOT CPHASE RZZ SWAP U DIAG.
CNOT takes (control, target).

Workload recipes (all numpy PCG64 via ``numpy.random.default_rng``):

* ``layered``: per layer a Haar-random U(2) on every qubit, then CZ on
  floor(N/4) disjoint pairs (consecutive entries of a seeded permutation,
  covering half the qubits), then RZ(theta), theta ~ U[0, 2 pi), on every qubit.
* ``diag_heavy``: exactly 80 % diagonal gates drawn uniformly from
  {RZ, CZ, CPHASE, RZZ} and 20 % non-diagonal gates from {H, SX, U},
  interleaved by a seeded shuffle; qubits uniform (pairs distinct), angles
  ~ U[0, 2 pi).
* ``rzz_full``: H on every qubit, then RZZ(theta) on every pair i < j
  (i outer, j inner), theta ~ U[0, 2 pi): the gate-level benchmark of
  Sec. 5.2 (Table 1).
* ``qft``: X on the set bits of a seeded basis index x0, then the textbook
  quantum Fourier transform (H and controlled phases from the top qubit
  down, then the qubit-order reversal by SWAPs): the circuit-level QFT of
  Sec. 5.3.
* ``qaoa_full``: H on every qubit, then per level RZZ(gamma_l) on every pair
  i < j and RX(beta_l) on every qubit, gamma_l and beta_l ~ U[0, pi): the
  5-level fully-connected QAOA of Sec. 5.3 and the ablation of Table 3
  (unweighted complete graph).
* ``serving_stream``: Poisson arrivals of layered circuits with N uniform in
  {10..30}, depth uniform in [10, 60] and a fair coin between complex128 and
  complex64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

DIAGONAL_KINDS = frozenset({"Z", "S", "T", "RZ", "CZ", "CPHASE", "RZZ", "DIAG"})
ONE_QUBIT_KINDS = frozenset({"H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ"})
TWO_QUBIT_KINDS = frozenset({"CZ", "CNOT", "CPHASE", "RZZ", "SWAP"})
ALL_KINDS = ONE_QUBIT_KINDS | TWO_QUBIT_KINDS | {"U", "DIAG"}


@dataclass(frozen=True)
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    theta: float = 0.0
    data: Optional[np.ndarray] = field(default=None, compare=False)

    @property
    def k(self) -> int:
        return len(self.qubits)

    def __repr__(self) -> str:  # short form, matrices elided
        t = f",{self.theta:.4g}" if self.kind in ("RX", "RY", "RZ", "CPHASE", "RZZ") else ""
        return f"{self.kind}{list(self.qubits)}{t}"


def haar_unitary(rng: np.random.Generator, dim: int = 2) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Ginibre matrix with the phases
    of R's diagonal moved into Q (Mezzadri's construction)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return np.ascontiguousarray(q * ph[None, :], dtype=np.complex128)


def layered(n: int, layers: int, seed: int) -> List[Gate]:
    """Random layered circuit: U(2) on every qubit, CZ on floor(n/4) disjoint
    pairs, RZ on every qubit; ``n + n//4 + n`` gates per layer."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    npairs = n // 4
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("U", (q,), 0.0, haar_unitary(rng, 2)))
        perm = rng.permutation(n)
        for p in range(npairs):
            a, b = int(perm[2 * p]), int(perm[2 * p + 1])
            gates.append(Gate("CZ", (a, b)))
        thetas = rng.uniform(0.0, 2.0 * math.pi, size=n)
        for q in range(n):
            gates.append(Gate("RZ", (q,), float(thetas[q])))
    return gates


def diag_heavy(n: int, n_gates: int = 200, seed: int = 2, diag_frac: float = 0.8) -> List[Gate]:
    """Diagonal-heavy circuit: round(diag_frac*n_gates) diagonal gates and the
    rest non-diagonal, order fixed by a seeded shuffle."""
    rng = np.random.default_rng(seed)
    n_diag = int(round(diag_frac * n_gates))
    is_diag = np.array([True] * n_diag + [False] * (n_gates - n_diag))
    rng.shuffle(is_diag)
    diag_kinds = ("RZ", "CZ", "CPHASE", "RZZ")
    nondiag_kinds = ("H", "SX", "U")
    gates: List[Gate] = []
    for d in is_diag:
        kind = (diag_kinds if d else nondiag_kinds)[int(rng.integers(0, 4 if d else 3))]
        if kind in TWO_QUBIT_KINDS:
            a = int(rng.integers(0, n))
            b = int(rng.integers(0, n - 1))
            if b >= a:
                b += 1
            qs: Tuple[int, ...] = (a, b)
        else:
            qs = (int(rng.integers(0, n)),)
        theta = float(rng.uniform(0.0, 2.0 * math.pi)) if kind in ("RZ", "CPHASE", "RZZ") else 0.0
        data = haar_unitary(rng, 2) if kind == "U" else None
        gates.append(Gate(kind, qs, theta, data))
    return gates


def product_circuit(n: int, depth: int, seed: int) -> List[Gate]:
    """Only single-qubit gates (no entanglement): ``depth`` random gates per
    qubit drawn from {U, H, SX, RX, RY, RZ}, interleaved across qubits."""
    rng = np.random.default_rng(seed)
    kinds = ("U", "H", "SX", "RX", "RY", "RZ")
    gates: List[Gate] = []
    for _ in range(depth):
        for q in rng.permutation(n):
            kind = kinds[int(rng.integers(0, len(kinds)))]
            theta = float(rng.uniform(0.0, 2.0 * math.pi)) if kind in ("RX", "RY", "RZ") else 0.0
            data = haar_unitary(rng, 2) if kind == "U" else None
            gates.append(Gate(kind, (int(q),), theta, data))
    return gates


def hadamard_diagonal_circuit(n: int, n_diag: int, seed: int) -> List[Gate]:
    """H on every qubit followed only by diagonal gates (RZ, CZ, CPHASE, RZZ,
    Z, S, T) on random qubits."""
    rng = np.random.default_rng(seed)
    gates = [Gate("H", (q,)) for q in range(n)]
    kinds = ("RZ", "CZ", "CPHASE", "RZZ", "Z", "S", "T")
    for _ in range(n_diag):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind in TWO_QUBIT_KINDS:
            a = int(rng.integers(0, n))
            b = int(rng.integers(0, n - 1))
            if b >= a:
                b += 1
            qs: Tuple[int, ...] = (a, b)
        else:
            qs = (int(rng.integers(0, n)),)
        theta = float(rng.uniform(0.0, 2.0 * math.pi)) if kind in ("RZ", "CPHASE", "RZZ") else 0.0
        gates.append(Gate(kind, qs, theta))
    return gates


def random_mixed(n: int, n_gates: int, seed: int, max_k: int = 3,
                 kinds: Sequence[str] = ("H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ",
                                         "CZ", "CNOT", "CPHASE", "RZZ", "SWAP", "U", "DIAG")) -> List[Gate]:
    """Random circuit over every gate kind; ``U``/``DIAG`` act on 1..max_k
    qubits (Haar unitary / unit-modulus random phases)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(n_gates):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind in ("U", "DIAG"):
            k = int(rng.integers(1, min(max_k, n) + 1))
        elif kind in TWO_QUBIT_KINDS:
            k = 2
        else:
            k = 1
        if k > n:
            continue
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        theta = float(rng.uniform(0.0, 2.0 * math.pi)) if kind in ("RX", "RY", "RZ", "CPHASE", "RZZ") else 0.0
        data = None
        if kind == "U":
            data = haar_unitary(rng, 1 << k)
        elif kind == "DIAG":
            data = np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, size=1 << k)).astype(np.complex128)
        gates.append(Gate(kind, qs, theta, data))
    return gates


def rzz_full(n: int, seed: int = 7) -> List[Gate]:
    """H on every qubit, then RZZ on all n(n-1)/2 pairs with seeded angles."""
    rng = np.random.default_rng(seed)
    gates = [Gate("H", (q,)) for q in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            gates.append(Gate("RZZ", (i, j), float(rng.uniform(0.0, 2.0 * math.pi))))
    return gates


def qft_input_index(n: int, seed: int) -> int:
    """The seeded basis index x0 that ``qft`` prepares before the transform."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n, dtype=np.uint64))


def qft(n: int, seed: int = 8) -> List[Gate]:
    """X gates preparing |x0> (x0 = qft_input_index(n, seed)), then the QFT:
    for j = n-1 down to 0, H on j and CPHASE(pi / 2^(j-k)) on (k, j) for
    k = j-1 down to 0; finally SWAP(j, n-1-j) for j < n/2."""
    x0 = qft_input_index(n, seed)
    gates = [Gate("X", (q,)) for q in range(n) if (x0 >> q) & 1]
    for j in range(n - 1, -1, -1):
        gates.append(Gate("H", (j,)))
        for k in range(j - 1, -1, -1):
            gates.append(Gate("CPHASE", (k, j), math.pi / float(1 << (j - k))))
    for j in range(n // 2):
        gates.append(Gate("SWAP", (j, n - 1 - j)))
    return gates


def qaoa_angles(levels: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """(gammas, betas) of ``qaoa_full``, each ~ U[0, pi)."""
    rng = np.random.default_rng(seed)
    gammas = rng.uniform(0.0, math.pi, size=levels)
    betas = rng.uniform(0.0, math.pi, size=levels)
    return gammas, betas


def qaoa_full(n: int, levels: int = 5, seed: int = 9) -> List[Gate]:
    """QAOA on the complete graph: H on every qubit, then per level RZZ(gamma)
    on every pair and RX(beta) on every qubit; n + levels (n(n-1)/2 + n) gates."""
    gammas, betas = qaoa_angles(levels, seed)
    gates = [Gate("H", (q,)) for q in range(n)]
    for lv in range(levels):
        for i in range(n):
            for j in range(i + 1, n):
                gates.append(Gate("RZZ", (i, j), float(gammas[lv])))
        for q in range(n):
            gates.append(Gate("RX", (q,), float(betas[lv])))
    return gates


def layered_gate_count(n: int, layers: int) -> int:
    """Number of gates of layered(n, layers, seed)."""
    return layers * (n + n // 4 + n)


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    layers: int
    dtype: str        # "c128" or "c64"
    seed: int

    def circuit(self) -> List[Gate]:
        return layered(self.n, self.layers, self.seed)


def serving_stream(n_requests: int = 200, rate_per_s: float = 0.8, seed: int = 5,
                   n_min: int = 10, n_max: int = 30, l_min: int = 10, l_max: int = 60) -> List[Request]:
    """Poisson arrival stream of layered circuits (exponential inter-arrival
    times with mean 1/rate)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out: List[Request] = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(rng.integers(n_min, n_max + 1))
        layers = int(rng.integers(l_min, l_max + 1))
        dtype = "c128" if rng.integers(0, 2) == 0 else "c64"
        out.append(Request(i, t, n, layers, dtype, int(seed * 100003 + i)))
    return out


# The configurations the simulator is checked and measured on.
def config_circuit(name: str) -> Tuple[int, List[Gate]]:
    if name == "layered12":        # 12 qubits, 20 layers, seed 0 -> 540 gates
        return 12, layered(12, 20, 0)
    if name == "layered28":        # 28 qubits, 40 layers, seed 1 -> 2520 gates
        return 28, layered(28, 40, 1)
    if name == "layered30":        # 30 qubits, 40 layers, seed 1 -> 2680 gates
        return 30, layered(30, 40, 1)
    if name == "diag30":           # 30 qubits, 200 gates, 80 % diagonal, seed 2
        return 30, diag_heavy(30, 200, 2)
    if name == "diag24":           # same pattern at 24 qubits
        return 24, diag_heavy(24, 200, 2)
    if name == "layered32":        # 32 qubits, 40 layers, seed 4 -> 2880 gates
        return 32, layered(32, 40, 4)
    if name.startswith("qaoa"):     # 5-level fully-connected QAOA, seed 9
        n = int(name[4:])
        return n, qaoa_full(n, 5, 9)
    if name.startswith("qft"):      # QFT of a seeded basis state, seed 8
        n = int(name[3:])
        return n, qft(n, 8)
    if name.startswith("rzz"):      # H layer + RZZ on every pair, seed 7
        n = int(name[3:])
        return n, rzz_full(n, 7)
    raise KeyError(name)


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded uniform amplitude indices in [0, 2^n), uint64."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << n, size=count, dtype=np.uint64)
