"""Writes the stored expected values under tests/golden/ by running the CPU
oracle (and nothing else) on the seeded workload circuits.

    python tests/golden/make_golden.py layered28 layered30 diag30
    python tests/golden/make_golden.py --sketch layered28 layered30 diag30

Each output file holds, for one circuit: the oracle's norm, two marginal
distributions and the amplitudes at seeded sample indices.  With --sketch
the file <name>_sketch.txt holds instead the seeded projections of the
whole state (tests/golden/sketch.py), after checking that the recomputed
state still reproduces the stored sample amplitudes bit for bit.  Values
are printed with 17 significant digits (exact binary64 round trip).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2604_12256_amd import workloads as W  # noqa: E402
from tests.golden.sketch import N_PROJ, sketch  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 4096
SAMPLE_SEED = 3


def write(name: str) -> None:
    n, gates = W.config_circuit(name)
    t0 = time.time()
    state = oracle.run(n, gates)
    dt = time.time() - t0
    idx = W.sample_indices(n, N_SAMPLES, SAMPLE_SEED)
    idx = np.concatenate([np.arange(16, dtype=np.uint64), idx, np.array([(1 << n) - 1], dtype=np.uint64)])
    amp = state[idx.astype(np.int64)]
    lo = list(range(4))
    hi = list(range(n - 4, n))
    m_lo = oracle.marginal(state, lo)
    m_hi = oracle.marginal(state, hi)
    nrm = oracle.norm(state)
    path = os.path.join(HERE, f"{name}.txt")
    with open(path, "w") as f:
        f.write(f"# oracle output for workload {name}: n={n} gates={len(gates)}\n")
        f.write(f"# written by tests/golden/make_golden.py (CPU oracle only), {oracle.num_threads()} threads, "
                f"{dt:.0f} s\n")
        f.write(f"# sample indices: 0..15, workloads.sample_indices(n, {N_SAMPLES}, {SAMPLE_SEED}), 2^n-1\n")
        f.write(f"norm {nrm:.17g}\n")
        f.write("marginal_lo " + " ".join(str(q) for q in lo) + " : " + " ".join(f"{v:.17g}" for v in m_lo) + "\n")
        f.write("marginal_hi " + " ".join(str(q) for q in hi) + " : " + " ".join(f"{v:.17g}" for v in m_hi) + "\n")
        for i, a in zip(idx, amp):
            f.write(f"{int(i)} {a.real:.17g} {a.imag:.17g}\n")
    print(f"{name}: n={n} gates={len(gates)} oracle {dt:.1f} s -> {path}", flush=True)
    del state


def write_sketch(name: str) -> None:
    n, gates = W.config_circuit(name)
    t0 = time.time()
    state = oracle.run(n, gates)
    dt = time.time() - t0
    stored = read(name)
    same = np.array_equal(state[stored["idx"].astype(np.int64)], stored["amp"])
    if not same:
        raise SystemExit(f"{name}: the recomputed oracle state differs from the stored samples")
    s = sketch(state)
    path = os.path.join(HERE, f"{name}_sketch.txt")
    with open(path, "w") as f:
        f.write(f"# oracle output for workload {name}: n={n} gates={len(gates)}\n")
        f.write(f"# written by tests/golden/make_golden.py --sketch (CPU oracle only), {oracle.num_threads()} "
                f"threads, {dt:.0f} s; the state reproduces the stored samples of {name}.txt bit for bit\n")
        f.write(f"# {N_PROJ} projections s_k = sum_x w_k(x) a_x of tests/golden/sketch.py\n")
        for k, v in enumerate(s):
            f.write(f"sketch {k} {v.real:.17g} {v.imag:.17g}\n")
    print(f"{name}: n={n} gates={len(gates)} oracle {dt:.1f} s -> {path}", flush=True)
    del state


def read_sketch(name: str):
    """The stored projections of <name>_sketch.txt, or None when absent."""
    path = os.path.join(HERE, f"{name}_sketch.txt")
    if not os.path.exists(path):
        return None
    vals = []
    with open(path) as f:
        for line in f:
            if line.startswith("sketch"):
                parts = line.split()
                vals.append(complex(float(parts[2]), float(parts[3])))
    return np.array(vals, dtype=np.complex128)


def read(name: str):
    """Parse a golden file: dict(norm, marginals {tuple(qubits): array}, idx, amp)."""
    path = os.path.join(HERE, f"{name}.txt")
    out = {"marginals": {}}
    idx, amp = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "norm":
                out["norm"] = float(parts[1])
            elif parts[0].startswith("marginal"):
                colon = parts.index(":")
                qs = tuple(int(x) for x in parts[1:colon])
                out["marginals"][qs] = np.array([float(x) for x in parts[colon + 1:]])
            else:
                idx.append(int(parts[0]))
                amp.append(complex(float(parts[1]), float(parts[2])))
    out["idx"] = np.array(idx, dtype=np.uint64)
    out["amp"] = np.array(amp, dtype=np.complex128)
    return out


if __name__ == "__main__":
    oracle.build(force=False)
    names = [a for a in sys.argv[1:] if not a.startswith("--")]
    for name in names:
        if "--sketch" in sys.argv:
            write_sketch(name)
        else:
            write(name)
