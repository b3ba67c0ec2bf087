"""Reference interpreter of exported execution plans (numpy, CPU).

Applies the ops of a plan built by the library's host optimiser, so that the
optimiser's transformations (booster, diagonal detector, stages, register
phases, fusion) can be checked against the oracle without a GPU.  It is
written independently of the oracle: operators are applied by tensor
contraction over a [2]*n view of the state.
"""
import numpy as np


def apply_dense(psi, n, qubits, m):
    k = len(qubits)
    t = psi.reshape([2] * n)
    axes = [n - 1 - q for q in qubits]  # qubit q <-> axis n-1-q
    mt = m.reshape([2] * (2 * k))       # (r_{k-1} .. r_0, c_{k-1} .. c_0)
    out = np.tensordot(mt, t, axes=([k + (k - 1 - j) for j in range(k)], axes))
    out = np.moveaxis(out, [k - 1 - j for j in range(k)], axes)
    return np.ascontiguousarray(out).reshape(-1)


def apply_diag(psi, n, qubits, table):
    x = np.arange(1 << n, dtype=np.int64)
    y = np.zeros_like(x)
    for j, q in enumerate(qubits):
        y |= ((x >> q) & 1) << j
    return psi * table[y]


def apply_quad(psi, n, terms):
    """Phase exp(i phi(x)) with phi a quadratic form of the index bits, given
    as (code, angle) terms: code -1 the constant, 64 q + q the linear term of
    qubit q, 64 q + p (q < p) the term of the pair."""
    x = np.arange(1 << n, dtype=np.int64)
    phi = np.zeros(1 << n)
    for code, ang in terms:
        if code < 0:
            phi += ang
            continue
        q, p = divmod(code, 64)
        bits = (x >> q) & 1 if q == p else ((x >> q) & (x >> p)) & 1
        phi += ang * bits
    return psi * np.exp(1j * phi)


def run_plan(ops, n, layout, use_kernel_ops=True):
    bufs = {}
    for op in ops:
        b, nb = op["buffer"], op["buffer_qubits"]
        kind = op["kind"]
        if kind == "INIT":
            v = np.zeros(1 << nb, dtype=np.complex128)
            v[0] = 1
            bufs[b] = v
        elif kind == "WINDOW":
            # a host-memory offload pass: its ops are exported on the full
            # state's physical qubits, so they apply to the whole state
            if op["init"]:
                v = np.zeros(1 << nb, dtype=np.complex128)
                v[0] = 1
                bufs[b] = v
        elif kind == "KRON":
            bufs[b] = np.kron(bufs[op["src_hi"]], bufs[op["src_lo"]])
        elif kind == "DENSE":
            bufs[b] = apply_dense(bufs[b], nb, op["qubits"], op["payload"])
        elif kind == "DIAG":
            bufs[b] = apply_diag(bufs[b], nb, op["qubits"], op["payload"])
        elif kind == "STAGE":
            seq = op["kernel_ops"] if (use_kernel_ops and op["n_phases"] > 0) else op["gates"]
            for g in seq:
                if g.get("quad"):
                    bufs[b] = apply_quad(bufs[b], nb, g["terms"])
                elif g["diagonal"]:
                    bufs[b] = apply_diag(bufs[b], nb, g["qubits"], g["payload"])
                else:
                    bufs[b] = apply_dense(bufs[b], nb, g["qubits"], g["payload"])
        elif kind == "PERM":
            src = bufs[b]
            x = np.arange(1 << nb, dtype=np.int64)
            y = np.zeros_like(x)
            for p, d in enumerate(op["perm"]):
                y |= ((x >> p) & 1) << d
            out = np.empty_like(src)
            out[y] = src
            bufs[b] = out
        else:
            raise AssertionError(kind)
    phys = bufs[0]
    x = np.arange(1 << n, dtype=np.int64)
    y = np.zeros_like(x)
    for q in range(n):
        y |= ((x >> q) & 1) << layout[q]
    return phys[y]


def access_count(ops):
    """State-vector accesses of a plan in the counting model of the paper's
    worked example (Sec. 4.4): 2^m per gate applied to an m-qubit (sub-)state
    and 2^m per tensor product producing an m-qubit state; initialisation is
    not counted."""
    total = 0
    for op in ops:
        if op["kind"] in ("DENSE", "DIAG", "KRON"):
            total += 1 << op["buffer_qubits"]
        elif op["kind"] == "STAGE":
            total += len(op["gates"]) << op["buffer_qubits"]
    return total
