"""Python front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It marshals generator circuits into the oracle's own C
structs (``oracle.c``) and wraps the plain complex128 simulator and its
reductions.  Nothing here is shared with, or imported by, the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Oracle-private gate numbering (mirrors the enum in oracle.c).
_KIND = {
    "U": 0, "DIAG": 1, "H": 2, "X": 3, "Y": 4, "Z": 5, "S": 6, "T": 7, "SX": 8,
    "RX": 9, "RY": 10, "RZ": 11, "CZ": 12, "CNOT": 13, "CPHASE": 14, "RZZ": 15, "SWAP": 16,
}


class _OGGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nq", ctypes.c_int32), ("q", ctypes.c_int32 * 6),
                ("theta", ctypes.c_double), ("data", ctypes.c_void_p)]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, OpenMP, no FMA
    contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.og_gate_matrix.argtypes = [ctypes.POINTER(_OGGate), ctypes.c_void_p]
        lib.og_gate_matrix.restype = ctypes.c_int
        lib.og_apply.argtypes = [ctypes.c_int, ctypes.POINTER(_OGGate), ctypes.c_int64, ctypes.c_void_p]
        lib.og_apply.restype = ctypes.c_int
        lib.og_run.argtypes = [ctypes.c_int, ctypes.POINTER(_OGGate), ctypes.c_int64, ctypes.c_void_p]
        lib.og_run.restype = ctypes.c_int
        lib.og_norm.argtypes = [ctypes.c_int, ctypes.c_void_p]
        lib.og_norm.restype = ctypes.c_double
        lib.og_inner.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.og_inner.restype = None
        lib.og_marginal.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p]
        lib.og_marginal.restype = ctypes.c_int
        lib.og_num_threads.restype = ctypes.c_int
        lib.og_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


class _Marshalled:
    """Keeps the ctypes array and the matrix buffers alive together."""

    def __init__(self, gates: Sequence) -> None:
        self.keep = []
        arr = (_OGGate * max(1, len(gates)))()
        for i, g in enumerate(gates):
            s = arr[i]
            s.kind = _KIND[g.kind]
            s.nq = len(g.qubits)
            for t, q in enumerate(g.qubits):
                s.q[t] = int(q)
            s.theta = float(g.theta)
            if g.data is not None:
                buf = np.ascontiguousarray(np.asarray(g.data, dtype=np.complex128)).view(np.float64)
                self.keep.append(buf)
                s.data = buf.ctypes.data
            else:
                s.data = None
        self.arr = arr
        self.n = len(gates)


def gate_matrix(gate) -> np.ndarray:
    """The oracle's 2^k x 2^k matrix of one gate (row-major, bit t <-> q[t])."""
    m = _Marshalled([gate])
    k = len(gate.qubits)
    out = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    if _load().og_gate_matrix(ctypes.byref(m.arr[0]), out.ctypes.data) != 0:
        raise ValueError(f"oracle: bad gate {gate!r}")
    return out


def run(n: int, gates: Sequence) -> np.ndarray:
    """|0...0> followed by the circuit, gate by gate; complex128[2^n]."""
    state = np.empty(1 << n, dtype=np.complex128)
    m = _Marshalled(gates)
    if _load().og_run(n, m.arr, m.n, state.ctypes.data) != 0:
        raise ValueError("oracle: invalid circuit")
    return state


def apply(n: int, gates: Sequence, state: np.ndarray) -> np.ndarray:
    """Apply the circuit to a copy of ``state``."""
    out = np.array(state, dtype=np.complex128, copy=True)
    if out.shape != (1 << n,):
        raise ValueError("oracle: state has the wrong length")
    m = _Marshalled(gates)
    if _load().og_apply(n, m.arr, m.n, out.ctypes.data) != 0:
        raise ValueError("oracle: invalid circuit")
    return out


def apply_inplace(n: int, gates: Sequence, state: np.ndarray) -> None:
    """Apply the circuit to ``state`` itself (complex128, C-contiguous, 2^n)."""
    if state.dtype != np.complex128 or state.shape != (1 << n,) or not state.flags.c_contiguous:
        raise ValueError("oracle: state must be a contiguous complex128 array of 2^n entries")
    m = _Marshalled(gates)
    if _load().og_apply(n, m.arr, m.n, state.ctypes.data) != 0:
        raise ValueError("oracle: invalid circuit")


def norm(state: np.ndarray) -> float:
    """sum |a_i|^2 by pairwise summation."""
    state = np.ascontiguousarray(state, dtype=np.complex128)
    n = int(state.size).bit_length() - 1
    return float(_load().og_norm(n, state.ctypes.data))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a|b> = sum conj(a_i) b_i by pairwise summation."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = int(a.size).bit_length() - 1
    out = np.zeros(2, dtype=np.float64)
    _load().og_inner(n, a.ctypes.data, b.ctypes.data, out.ctypes.data)
    return complex(out[0], out[1])


def infidelity(a: np.ndarray, b: np.ndarray) -> float:
    """1 - |<a|b>|^2 / (<a|a><b|b>)."""
    ab = inner(a, b)
    return 1.0 - (abs(ab) ** 2) / (norm(a) * norm(b))


def marginal(state: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """P[y] with bit t of y <-> qubit qubits[t]."""
    state = np.ascontiguousarray(state, dtype=np.complex128)
    n = int(state.size).bit_length() - 1
    q = np.ascontiguousarray(np.asarray(qubits, dtype=np.int32))
    out = np.zeros(1 << len(qubits), dtype=np.float64)
    if _load().og_marginal(n, state.ctypes.data, q.ctypes.data, len(qubits), out.ctypes.data) != 0:
        raise ValueError("oracle: bad qubit list")
    return out


def num_threads() -> int:
    return int(_load().og_num_threads())


def set_threads(t: int) -> None:
    _load().og_set_threads(int(t))
