"""Per-amplitude closed forms for the oracle -- TEST INFRASTRUCTURE ONLY.

Two circuit families have amplitudes that can be computed one index at a time,
so they give expected values at sizes where the full oracle state would not
fit or would take too long:

* a circuit of single-qubit gates only leaves a product state (no
  entanglement, the situation the merge booster exploits, Sec. 3 and
  Sec. 4.4): a_x = prod_q (U_q ... U_q |0>)[bit q of x];
* H on every qubit followed only by diagonal gates (Sec. 4.5: a diagonal gate
  multiplies amplitude i by lambda_i): a_x = 2^{-N/2} prod_d lambda_d(x);
* the quantum Fourier transform (the circuit-level benchmark of Sec. 5.3) of
  a basis state |x0>: a_y = 2^{-N/2} exp(2 pi i x0 y / 2^N);
* QAOA on the complete graph (Sec. 5.3, Table 3): H on every qubit, then
  levels of RZZ(gamma) on every pair and RX(beta) on every qubit.  Every
  gate layer is invariant under permutations of the qubits, so the amplitude
  of x depends only on its Hamming weight w, and the state is carried as
  N + 1 numbers c_w (parity unpinned by the paper itself: it prints no
  amplitudes; pinned against the full oracle at small N and by special cases).

Gate matrices come from the oracle's own gate library, except in the QAOA
form, whose layer actions are derived below from RZZ and RX's definitions.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

from . import oracle


def product_state_factors(n: int, gates: Sequence) -> np.ndarray:
    """[n, 2] complex: the single-qubit state of every qubit."""
    f = np.zeros((n, 2), dtype=np.complex128)
    f[:, 0] = 1.0
    for g in gates:
        if len(g.qubits) != 1:
            raise ValueError("product_state_factors: only single-qubit gates")
        q = g.qubits[0]
        f[q] = oracle.gate_matrix(g) @ f[q]
    return f


def product_state_amplitudes(n: int, gates: Sequence, idx: np.ndarray) -> np.ndarray:
    f = product_state_factors(n, gates)
    idx = np.asarray(idx, dtype=np.uint64)
    out = np.ones(idx.shape, dtype=np.complex128)
    for q in range(n):
        bit = ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
        out *= f[q][bit]
    return out


def hadamard_diagonal_amplitudes(n: int, gates: Sequence, idx: np.ndarray) -> np.ndarray:
    """Amplitudes of H^{(x)n} followed by diagonal gates only.  ``gates`` must
    start with H on every qubit; every later gate must be diagonal."""
    for q in range(n):
        g = gates[q]
        if g.kind != "H" or g.qubits != (q,):
            raise ValueError("hadamard_diagonal_amplitudes: expects H on qubit 0..n-1 first")
    idx = np.asarray(idx, dtype=np.uint64)
    out = np.full(idx.shape, 2.0 ** (-n / 2.0), dtype=np.complex128)
    for g in gates[n:]:
        m = oracle.gate_matrix(g)
        lam = np.diagonal(m).copy()
        off = m - np.diag(lam)
        if np.any(off != 0):
            raise ValueError(f"hadamard_diagonal_amplitudes: {g!r} is not diagonal")
        r = np.zeros(idx.shape, dtype=np.int64)
        for t, q in enumerate(g.qubits):
            r |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << t
        out *= lam[r]
    return out


def qft_input(n: int, gates: Sequence) -> int:
    """x0 of a QFT circuit: the leading X gates prepare |x0>."""
    x0 = 0
    for g in gates:
        if g.kind != "X":
            break
        x0 |= 1 << g.qubits[0]
    return x0


def qft_amplitudes(n: int, x0: int, idx: np.ndarray) -> np.ndarray:
    """2^{-n/2} exp(2 pi i x0 y / 2^n) at y = idx; the phase is reduced
    mod 2^n in exact integer arithmetic first."""
    if n > 32:
        raise ValueError("qft_amplitudes: n <= 32 keeps x0 * y inside 64 bits")
    y = np.asarray(idx, dtype=np.uint64)
    r = (np.uint64(x0) * y) & np.uint64((1 << n) - 1)
    ang = (2.0 * math.pi) * (r.astype(np.float64) / float(1 << n))
    return (2.0 ** (-n / 2.0)) * (np.cos(ang) + 1j * np.sin(ang))


def _qaoa_layers(n: int, gates: Sequence) -> Sequence[Tuple[float, float]]:
    """Splits H^n, then [all-pairs RZZ(gamma), all-qubit RX(beta)]* into
    (gamma, beta) per level; raises if the circuit is not of that form."""
    for q in range(n):
        if gates[q].kind != "H" or gates[q].qubits != (q,):
            raise ValueError("qaoa: expects H on qubit 0..n-1 first")
    npairs = n * (n - 1) // 2
    pos, levels = n, []
    while pos < len(gates):
        block = gates[pos:pos + npairs]
        rx = gates[pos + npairs:pos + npairs + n]
        if len(block) != npairs or len(rx) != n:
            raise ValueError("qaoa: incomplete level")
        if any(g.kind != "RZZ" for g in block) or \
                {tuple(sorted(g.qubits)) for g in block} != {(i, j) for i in range(n) for j in range(i + 1, n)}:
            raise ValueError("qaoa: a level must start with RZZ on every pair")
        if any(g.kind != "RX" for g in rx) or sorted(g.qubits[0] for g in rx) != list(range(n)):
            raise ValueError("qaoa: a level must end with RX on every qubit")
        gamma, beta = block[0].theta, rx[0].theta
        if any(g.theta != gamma for g in block) or any(g.theta != beta for g in rx):
            raise ValueError("qaoa: one angle per layer")
        levels.append((gamma, beta))
        pos += npairs + n
    return levels


def qaoa_weights(n: int, gates: Sequence) -> np.ndarray:
    """c_w, w = 0..n: the amplitude of every basis state of Hamming weight w.

    * H^n|0>: c_w = 2^{-n/2}.
    * RZZ(g) = exp(-i g/2 Z Z) on every pair multiplies a basis state by
      exp(-i g/2 sum_{i<j} z_i z_j), z = +1 for a 0 bit and -1 for a 1 bit;
      with S = n - 2w, sum_{i<j} z_i z_j = (S^2 - n) / 2.
    * RX(b) = [[c, -is], [-is, c]] (c = cos b/2, s = sin b/2) on every qubit:
      a state y that differs from x (weight w) in k of x's ones and m of its
      zeros has weight w - k + m and contributes c^{n-k-m} (-is)^{k+m} a_y;
      there are C(w, k) C(n - w, m) such y.
    """
    c = np.full(n + 1, 2.0 ** (-n / 2.0), dtype=np.complex128)
    w = np.arange(n + 1)
    for gamma, beta in _qaoa_layers(n, gates):
        S = (n - 2 * w).astype(np.float64)
        c = c * np.exp(-0.5j * gamma * (S * S - n) / 2.0)
        co, si = math.cos(beta / 2.0), math.sin(beta / 2.0)
        new = np.zeros(n + 1, dtype=np.complex128)
        for x in range(n + 1):
            acc = 0j
            for k in range(x + 1):
                for m in range(n - x + 1):
                    d = k + m
                    acc += (math.comb(x, k) * math.comb(n - x, m) * co ** (n - d) * (-1j * si) ** d
                            * c[x - k + m])
            new[x] = acc
        c = new
    return c


def qaoa_amplitudes(n: int, gates: Sequence, idx: np.ndarray) -> np.ndarray:
    c = qaoa_weights(n, gates)
    idx = np.asarray(idx, dtype=np.uint64)
    w = np.zeros(idx.shape, dtype=np.int64)
    for q in range(n):
        w += ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
    return c[w]
