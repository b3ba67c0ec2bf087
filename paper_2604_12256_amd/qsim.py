"""Python binding of libqsim355 (ctypes; argument marshalling only).

Every step of the simulation runs in the HIP library.  PyTorch provides the
device memory of the state vector and the stream the library launches on.
The binding raises if the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqsim355.so")

# sim_gate_kind
KIND = {"U": 0, "MATRIX": 0, "DIAG": 1, "H": 2, "X": 3, "Y": 4, "Z": 5, "S": 6, "T": 7, "SX": 8,
        "RX": 9, "RY": 10, "RZ": 11, "CZ": 12, "CNOT": 13, "CPHASE": 14, "RZZ": 15, "SWAP": 16}
# sim_status
OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED = range(6)
STATUS = {0: "OK", 1: "INVAL", 2: "NOMEM", 3: "DEVICE", 4: "STATE", 5: "UNSUPPORTED"}
# optimisation flags
OPT_DIAG, OPT_FUSE, OPT_STAGES, OPT_BOOST, OPT_REMAP, OPT_QUAD = 1, 2, 4, 8, 16, 32
OPT_ALL = 63
# plan op kinds
OP_NAMES = {0: "INIT", 1: "KRON", 2: "DENSE", 3: "DIAG", 4: "STAGE", 5: "PERM", 6: "WINDOW"}
DTYPES = {"c128": 0, "c64": 1}


class SimGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("nq", ctypes.c_uint32), ("q", ctypes.c_uint32 * 6),
                ("theta", ctypes.c_double), ("data", ctypes.c_void_p)]


class SimOptions(ctypes.Structure):
    _fields_ = [("opt", ctypes.c_uint32), ("C", ctypes.c_uint32), ("F", ctypes.c_uint32),
                ("D", ctypes.c_uint32), ("B", ctypes.c_uint32), ("force_fuse_k", ctypes.c_uint32),
                ("L", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("dev_state", ctypes.c_void_p), ("dev_state_bytes", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("host_state", ctypes.c_void_p), ("host_state_bytes", ctypes.c_uint64)]


class SimRunStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("n_gates", "n_ops", "full_passes", "write_passes",
                                                "read_passes", "n_stages", "n_dense", "n_diag", "n_kron",
                                                "n_perm", "n_subruns")] + \
               [(f, ctypes.c_double) for f in ("plan_ms", "run_ms", "algorithmic_bytes", "flops", "est_ms")] + \
               [(f, ctypes.c_uint64) for f in ("offload_passes", "window_qubits")] + [("pcie_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class SimOpTiming(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("buffer", ctypes.c_uint32), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class SimPlanOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("buffer", ctypes.c_uint32), ("buffer_qubits", ctypes.c_uint32),
                ("src_lo", ctypes.c_uint32), ("src_hi", ctypes.c_uint32), ("nq", ctypes.c_uint32),
                ("qubits", ctypes.c_uint32 * 32), ("local_qubits", ctypes.c_uint32),
                ("n_phases", ctypes.c_uint32), ("payload_len", ctypes.c_uint64),
                ("first_gate", ctypes.c_uint64)]


class SimPlanGate(ctypes.Structure):
    _fields_ = [("diagonal", ctypes.c_uint32), ("nq", ctypes.c_uint32), ("qubits", ctypes.c_uint32 * 16),
                ("payload_len", ctypes.c_uint64), ("n_register", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class QsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library() -> ctypes.CDLL:
    """Loads libqsim355.so (import torch first so that one HIP runtime is
    shared with PyTorch)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libqsim355.so not built ({LIB_PATH}); run __graft_entry__.build()")
    import torch  # noqa: F401  (shares its HIP runtime with the library)
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "sim_create": (I, [U32, I, ctypes.POINTER(SimOptions), ctypes.POINTER(P)]),
        "sim_load_circuit": (I, [P, ctypes.POINTER(SimGate), U64]),
        "sim_run": (I, [P]),
        "sim_run_async": (I, [P]),
        "sim_amplitudes": (I, [P, P, U64, P]),
        "sim_probabilities": (I, [P, P, U32, P]),
        "sim_inner": (I, [P, P, P]),
        "sim_stats": (I, [P, ctypes.POINTER(SimRunStats)]),
        "sim_set_profiling": (I, [P, U32]),
        "sim_op_timings": (I, [P, ctypes.POINTER(SimOpTiming), U64, ctypes.POINTER(U64)]),
        "sim_last_error": (ctypes.c_char_p, [P]),
        "sim_device_bytes": (I, [P, ctypes.POINTER(U64)]),
        "sim_probabilities_noalloc": (I, [P, P, U32, P]),
        "sim_destroy": (I, [P]),
        "sim_run_batch": (I, [P, U32, P]),
        "sim_plan_build": (I, [U32, I, ctypes.POINTER(SimOptions), ctypes.POINTER(SimGate), U64,
                               ctypes.POINTER(P)]),
        "sim_plan_num_ops": (U64, [P]),
        "sim_plan_get_op": (I, [P, U64, ctypes.POINTER(SimPlanOp), P]),
        "sim_plan_stage_gate": (I, [P, U64, U64, ctypes.POINTER(SimPlanGate), P]),
        "sim_plan_layout": (I, [P, P]),
        "sim_plan_stage_kernel_op": (I, [P, U64, U64, ctypes.POINTER(SimPlanGate), P]),
        "sim_plan_stats": (I, [P, ctypes.POINTER(SimRunStats)]),
        "sim_plan_counters": (I, [P, P, P, P]),
        "sim_plan_destroy": (I, [P]),
        "sim_version": (ctypes.c_char_p, []),
        "sim_device_copy": (I, [P, P, U64, P]),
        "sim_measure": (I, [P, U32, ctypes.c_double, P, P]),
        "sim_sample": (I, [P, P, U64, P]),
        "sim_expect_z": (I, [P, P, U32, P]),
        "sim_expect_diagonal": (I, [P, P, U32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class _Gates:
    """ctypes sim_gate array plus the payload buffers it points to."""

    def __init__(self, gates: Sequence) -> None:
        self.keep = []
        self.n = len(gates)
        arr = (SimGate * max(1, self.n))()
        for i, g in enumerate(gates):
            s = arr[i]
            s.kind = KIND[g.kind]
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


class Circuit(_Gates):
    """A circuit already marshalled into the ABI's gate array: `load` it any
    number of times without converting the Python gates again."""

    def __init__(self, gates: Sequence) -> None:
        super().__init__(gates)


def _as_gates(gates) -> _Gates:
    return gates if isinstance(gates, _Gates) else _Gates(gates)


def _options(opt: int, C: int, F: int, D: int, B: int, force_fuse_k: int, state_ptr: int = 0,
             state_bytes: int = 0, stream: int = 0, L: int = 0, host_ptr: int = 0,
             host_bytes: int = 0) -> SimOptions:
    o = SimOptions()
    o.opt, o.C, o.F, o.D, o.B, o.force_fuse_k, o.L = opt, C, F, D, B, force_fuse_k, L
    o.dev_state = state_ptr or None
    o.dev_state_bytes = state_bytes
    o.stream = stream or None
    o.host_state = host_ptr or None
    o.host_state_bytes = host_bytes
    return o


class Simulator:
    """One state vector on the GPU and the circuit loaded into it.

    offload_window > 0 keeps the state in pinned host memory instead and
    gives the device two windows of 2^offload_window amplitudes (host-memory
    offload; the state may then be larger than the device memory)."""

    def __init__(self, n: int, dtype: str = "c128", opt: int = 0, C: int = 0, F: int = 0, D: int = 0,
                 B: int = 0, force_fuse_k: int = 0, state=None, stream=None, device: int = 0, L: int = 0,
                 offload_window: int = 0) -> None:
        import torch
        self._lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("qsim355 needs a GPU: torch.cuda.is_available() is False")
        self.n = int(n)
        self.dtype = dtype
        real = torch.float64 if dtype == "c128" else torch.float32
        self.host_state = None
        host_ptr = host_bytes = 0
        if offload_window:
            # pinned host memory for the state, two device windows
            self.host_state = torch.empty(2 << self.n, dtype=real, pin_memory=True)
            host_ptr = self.host_state.data_ptr()
            host_bytes = self.host_state.numel() * self.host_state.element_size()
            if state is None:
                state = torch.empty(2 * (2 << int(offload_window)), dtype=real, device=f"cuda:{device}")
        if state is None:
            state = torch.empty(2 << self.n, dtype=real, device=f"cuda:{device}")
        self.state = state
        self.stream = stream if stream is not None else torch.cuda.current_stream(state.device)
        o = _options(opt, C, F, D, B, force_fuse_k, state.data_ptr(), state.numel() * state.element_size(),
                     self.stream.cuda_stream, L, host_ptr, host_bytes)
        ctx = ctypes.c_void_p()
        st = self._lib.sim_create(self.n, DTYPES[dtype], ctypes.byref(o), ctypes.byref(ctx))
        if st != OK:
            raise QsimError(st, "sim_create failed")
        self._ctx = ctx
        self.n_gates = 0

    def _check(self, st: int) -> None:
        if st != OK:
            raise QsimError(st, self._lib.sim_last_error(self._ctx).decode())

    def load(self, gates) -> None:
        """Validates and plans a circuit: a sequence of gates or a `Circuit`."""
        m = _as_gates(gates)
        self._check(self._lib.sim_load_circuit(self._ctx, m.arr, m.n))
        self.n_gates = m.n

    def run(self) -> None:
        self._check(self._lib.sim_run(self._ctx))

    def run_async(self) -> None:
        self._check(self._lib.sim_run_async(self._ctx))

    def amplitudes(self, idx: Optional[np.ndarray] = None) -> np.ndarray:
        if idx is None:
            out = np.empty(1 << self.n, dtype=np.complex128)
            self._check(self._lib.sim_amplitudes(self._ctx, None, 1 << self.n, out.ctypes.data))
            return out
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
        out = np.empty(idx.size, dtype=np.complex128)
        self._check(self._lib.sim_amplitudes(self._ctx, idx.ctypes.data, idx.size, out.ctypes.data))
        return out

    def probabilities(self, qubits: Sequence[int]) -> np.ndarray:
        q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.uint32))
        out = np.empty(1 << len(q), dtype=np.float64)
        self._check(self._lib.sim_probabilities(self._ctx, q.ctypes.data if len(q) else None, len(q),
                                                out.ctypes.data))
        return out

    def probabilities_noalloc(self, qubits: Sequence[int]) -> np.ndarray:
        """As probabilities(), through the entry point that allocates no
        device memory (a static per-GPU scratch array)."""
        q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.uint32))
        out = np.empty(1 << len(q), dtype=np.float64)
        self._check(self._lib.sim_probabilities_noalloc(self._ctx, q.ctypes.data if len(q) else None, len(q),
                                                        out.ctypes.data))
        return out

    def norm(self) -> float:
        return float(self.probabilities([])[0])

    def inner(self, other: "Simulator") -> complex:
        out = np.empty(2, dtype=np.float64)
        self._check(self._lib.sim_inner(self._ctx, other._ctx, out.ctypes.data))
        return complex(out[0], out[1])

    def measure(self, qubit: int, u: float) -> Tuple[int, float]:
        """Projective measurement of one qubit with the caller's uniform u in
        [0, 1); the state collapses in place.  Returns (outcome, probability)."""
        m = ctypes.c_uint32()
        p = ctypes.c_double()
        self._check(self._lib.sim_measure(self._ctx, int(qubit), float(u), ctypes.byref(m), ctypes.byref(p)))
        return int(m.value), float(p.value)

    def sample(self, u: np.ndarray) -> np.ndarray:
        """Basis states for the uniforms u (inverse cumulative distribution in
        logical index order)."""
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).ravel()
        out = np.empty(u.size, dtype=np.uint64)
        if u.size:
            self._check(self._lib.sim_sample(self._ctx, u.ctypes.data, u.size, out.ctypes.data))
        return out

    def expect_z(self, masks: Sequence[int]) -> np.ndarray:
        """<psi| Z_S |psi> for every logical qubit mask S."""
        m = np.ascontiguousarray(np.asarray(list(masks), dtype=np.uint64))
        out = np.empty(m.size, dtype=np.float64)
        if m.size:
            self._check(self._lib.sim_expect_z(self._ctx, m.ctypes.data, m.size, out.ctypes.data))
        return out

    def expect_diagonal(self, qubits: Sequence[int], f: np.ndarray) -> float:
        """sum_y P(y) f[y] over the marginal of `qubits`."""
        q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.uint32))
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        if f.size != (1 << len(q)):
            raise ValueError("f must hold 2^len(qubits) values")
        out = ctypes.c_double()
        self._check(self._lib.sim_expect_diagonal(self._ctx, q.ctypes.data if len(q) else None, len(q),
                                                  f.ctypes.data, ctypes.byref(out)))
        return float(out.value)

    def stats(self) -> dict:
        s = SimRunStats()
        self._check(self._lib.sim_stats(self._ctx, ctypes.byref(s)))
        return s.as_dict()

    def set_profiling(self, enable: bool) -> None:
        self._check(self._lib.sim_set_profiling(self._ctx, 1 if enable else 0))

    def device_bytes(self) -> int:
        """Device memory the context holds beside the state buffer."""
        v = ctypes.c_uint64()
        self._check(self._lib.sim_device_bytes(self._ctx, ctypes.byref(v)))
        return int(v.value)

    def op_timings(self) -> List[dict]:
        n = ctypes.c_uint64()
        self._lib.sim_op_timings(self._ctx, None, 0, ctypes.byref(n))
        arr = (SimOpTiming * max(1, n.value))()
        self._check(self._lib.sim_op_timings(self._ctx, arr, n.value, ctypes.byref(n)))
        return [{"kind": OP_NAMES[a.kind], "buffer": a.buffer, "ms": a.ms, "flops": a.flops, "bytes": a.bytes}
                for a in arr[:n.value]]

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self._lib.sim_destroy(self._ctx)
            self._ctx = None
        self.state = None  # the device state buffer may be released once the context is gone
        self.host_state = None

    def __del__(self) -> None:
        try:
            self.close()
        except Exception:
            pass


def device_copy(dst, src, stream=None) -> None:
    """Plain device copy between two torch tensors (bandwidth reference)."""
    import torch
    lib = load_library()
    nbytes = min(dst.numel() * dst.element_size(), src.numel() * src.element_size()) // 16 * 16
    s = stream if stream is not None else torch.cuda.current_stream(dst.device)
    st = lib.sim_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    if st != OK:
        raise QsimError(st, "sim_device_copy failed")


def run_batch(sims: Sequence[Simulator], stream=None) -> None:
    """Runs several loaded circuits of one dtype together: small states in
    one launch per 128, larger resident states with their full-state stages
    launched together (one launch per stage step for up to 64 states).
    Does not wait: synchronise the stream before reading the states."""
    lib = load_library()
    arr = (ctypes.c_void_p * max(1, len(sims)))(*[s._ctx for s in sims])
    st = lib.sim_run_batch(arr, len(sims), stream.cuda_stream if stream is not None else None)
    if st != OK:
        raise QsimError(st, "sim_run_batch failed")


# ---------------------------------------------------------------- host-only plans
class Plan:
    """The execution plan the library builds for a circuit (no GPU needed)."""

    def __init__(self, n: int, gates: Sequence, dtype: str = "c128", opt: int = OPT_ALL, C: int = 0,
                 F: int = 0, D: int = 0, B: int = 0, force_fuse_k: int = 0, L: int = 0,
                 offload_window: int = 0) -> None:
        self._lib = load_library()
        self.n = n
        m = _as_gates(gates)
        if offload_window:
            # planning only: the host buffer is never touched (any non-NULL value)
            amp = 16 if dtype == "c128" else 8
            o = _options(opt, C, F, D, B, force_fuse_k, L=L, state_bytes=2 * amp << offload_window,
                         host_ptr=1, host_bytes=amp << n)
        else:
            o = _options(opt, C, F, D, B, force_fuse_k, L=L)
        p = ctypes.c_void_p()
        st = self._lib.sim_plan_build(n, DTYPES[dtype], ctypes.byref(o), m.arr, m.n, ctypes.byref(p))
        if st != OK:
            raise QsimError(st, "sim_plan_build failed")
        self._p = p

    def ops(self) -> List[dict]:
        out = []
        for i in range(self._lib.sim_plan_num_ops(self._p)):
            op = SimPlanOp()
            self._lib.sim_plan_get_op(self._p, i, ctypes.byref(op), None)
            payload = np.empty(max(1, op.payload_len), dtype=np.complex128)
            self._lib.sim_plan_get_op(self._p, i, ctypes.byref(op), payload.ctypes.data)
            d = {"kind": OP_NAMES[op.kind], "buffer": op.buffer, "buffer_qubits": op.buffer_qubits,
                 "src_lo": op.src_lo, "src_hi": op.src_hi}
            if d["kind"] in ("DENSE", "DIAG"):
                d["qubits"] = [op.qubits[t] for t in range(op.nq)]
                k = op.nq
                d["payload"] = payload[:op.payload_len].copy()
                if d["kind"] == "DENSE":
                    d["payload"] = d["payload"].reshape(1 << k, 1 << k)
            elif d["kind"] == "STAGE":
                d["local"] = [op.qubits[t] for t in range(op.local_qubits)]
                d["n_phases"] = op.n_phases
                gates = []
                for j in range(op.nq):
                    g = SimPlanGate()
                    self._lib.sim_plan_stage_gate(self._p, i, j, ctypes.byref(g), None)
                    pl = np.empty(max(1, g.payload_len), dtype=np.complex128)
                    self._lib.sim_plan_stage_gate(self._p, i, j, ctypes.byref(g), pl.ctypes.data)
                    qs = [g.qubits[t] for t in range(g.nq)]
                    mat = pl[:g.payload_len].copy()
                    if not g.diagonal:
                        mat = mat.reshape(1 << g.nq, 1 << g.nq)
                    gates.append({"diagonal": bool(g.diagonal), "qubits": qs, "payload": mat})
                d["gates"] = gates
                kops = []
                j = 0
                while True:
                    g = SimPlanGate()
                    if self._lib.sim_plan_stage_kernel_op(self._p, i, j, ctypes.byref(g), None) != OK:
                        break
                    pl = np.empty(max(1, g.payload_len), dtype=np.complex128)
                    self._lib.sim_plan_stage_kernel_op(self._p, i, j, ctypes.byref(g), pl.ctypes.data)
                    if g.diagonal == 2:
                        # quadratic phase: (code, angle) terms, code -1 the
                        # constant, 64 q + q linear in qubit q, 64 q + p a pair
                        terms = [(int(round(v.real)), float(v.imag)) for v in pl[:g.payload_len]]
                        kops.append({"diagonal": True, "quad": True, "qubits": [], "terms": terms,
                                     "payload": None, "n_register": 0})
                        j += 1
                        continue
                    qs = [g.qubits[t] for t in range(g.nq)]
                    mat = pl[:g.payload_len].copy()
                    if not g.diagonal:
                        mat = mat.reshape(1 << g.nq, 1 << g.nq)
                    kops.append({"diagonal": bool(g.diagonal), "qubits": qs, "payload": mat,
                                 "n_register": g.n_register})
                    j += 1
                d["kernel_ops"] = kops
            elif d["kind"] == "PERM":
                d["perm"] = [op.qubits[t] for t in range(op.nq)]
            elif d["kind"] == "WINDOW":
                d["outer_lo"], d["outer_n"], d["init"] = op.qubits[0], op.qubits[1], bool(op.qubits[2])
                d["pass_ops"] = op.nq
            out.append(d)
        return out

    def layout(self) -> List[int]:
        a = np.zeros(self.n, dtype=np.uint32)
        self._lib.sim_plan_layout(self._p, a.ctypes.data)
        return [int(x) for x in a]

    def stats(self) -> dict:
        s = SimRunStats()
        self._lib.sim_plan_stats(self._p, ctypes.byref(s))
        return s.as_dict()

    def counters(self) -> dict:
        a = (ctypes.c_uint64 * 3)()
        self._lib.sim_plan_counters(self._p, ctypes.byref(a, 0), ctypes.byref(a, 8), ctypes.byref(a, 16))
        return {"dd_visits": a[0], "booster_gates": a[1], "booster_groups": a[2]}

    def close(self) -> None:
        if getattr(self, "_p", None):
            self._lib.sim_plan_destroy(self._p)
            self._p = None

    def __del__(self) -> None:
        try:
            self.close()
        except Exception:
            pass
