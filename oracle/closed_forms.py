"""Per-amplitude closed forms for the oracle -- TEST INFRASTRUCTURE ONLY.

Two circuit families have amplitudes that can be computed one index at a time,
so they give expected values at sizes where the full oracle state would not
fit or would take too long:

* a circuit of single-qubit gates only leaves a product state (no
  entanglement, the situation the merge booster exploits, Sec. 3 and
  Sec. 4.4): a_x = prod_q (U_q ... U_q |0>)[bit q of x];
* H on every qubit followed only by diagonal gates (Sec. 4.5: a diagonal gate
  multiplies amplitude i by lambda_i): a_x = 2^{-N/2} prod_d lambda_d(x).

Gate matrices come from the oracle's own gate library.
"""
from __future__ import annotations

from typing import Sequence

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
