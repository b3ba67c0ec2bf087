"""Measurement on a state vector, by definition -- TEST INFRASTRUCTURE ONLY.

The paper's measurement background (Sec. 2) uses projective operators:
M_i^j keeps the amplitudes whose qubit j equals i and zeroes the others; the
probability of outcome i is <psi| M_i^j |psi>, and after the outcome the
state is M_i^j |psi> renormalised.  Shots are drawn by inverting the
cumulative distribution of |a_x|^2 in index order; random numbers are inputs
(uniforms in [0, 1)).  Z strings are the diagonal observables
Z_S |x> = (-1)^{|x & S|} |x>.

Plain numpy in FP64: sequential cumulative sums (numpy.cumsum), full sums by
numpy.  Used by the tests, never by the library.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def _probs(state: np.ndarray) -> np.ndarray:
    a = np.asarray(state, dtype=np.complex128)
    return a.real * a.real + a.imag * a.imag


def measure(state: np.ndarray, qubit: int, u: float) -> Tuple[int, float, np.ndarray]:
    """(outcome, probability, collapsed state): outcome 0 iff u < p0 / (p0 + p1)."""
    if not (0.0 <= u < 1.0):
        raise ValueError("u must lie in [0, 1)")
    p = _probs(state)
    x = np.arange(p.size, dtype=np.uint64)
    one = ((x >> np.uint64(qubit)) & np.uint64(1)).astype(bool)
    p1 = float(p[one].sum())
    p0 = float(p[~one].sum())
    total = p0 + p1
    m = 0 if u < p0 / total else 1
    keep = one if m == 1 else ~one
    pm = p1 if m == 1 else p0
    out = np.where(keep, np.asarray(state, dtype=np.complex128), 0.0) / np.sqrt(pm)
    return m, pm / total, out


def sample(state: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Smallest x with cumsum(|a|^2)[x] > u * total, for every u."""
    u = np.asarray(u, dtype=np.float64)
    if np.any(~((u >= 0.0) & (u < 1.0))):
        raise ValueError("every u must lie in [0, 1)")
    cdf = np.cumsum(_probs(state))
    x = np.searchsorted(cdf, u * cdf[-1], side="right")
    return np.minimum(x, cdf.size - 1).astype(np.uint64)


def cdf(state: np.ndarray) -> np.ndarray:
    """Inclusive cumulative distribution in index order (for validity checks)."""
    return np.cumsum(_probs(state))


def expect_z(state: np.ndarray, masks: Sequence[int]) -> np.ndarray:
    p = _probs(state)
    x = np.arange(p.size, dtype=np.uint64)
    out = []
    for m in masks:
        bits = x & np.uint64(m)
        par = np.zeros(p.size, dtype=np.uint64)
        while np.any(bits):
            par ^= bits & np.uint64(1)
            bits >>= np.uint64(1)
        out.append(float(np.sum(np.where(par == 1, -p, p))))
    return np.array(out)


def expect_diagonal(state: np.ndarray, qubits: Sequence[int], f: np.ndarray) -> float:
    p = _probs(state)
    x = np.arange(p.size, dtype=np.uint64)
    y = np.zeros(p.size, dtype=np.int64)
    for t, q in enumerate(qubits):
        y |= ((x >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << t
    return float(np.sum(p * np.asarray(f, dtype=np.float64)[y]))
