"""Seeded random projections ("sketches") of a whole state vector, used to
compare states too large to store against the oracle's.

    s_k = sum_x w_k(x) a_x,   w_k(x) in {1, i, -1, -i},

with the four weights of index x taken from consecutive 2-bit fields of one
64-bit counter-based hash of x: SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) of x XOR a fixed
key.  An error delta in any single amplitude moves every s_k by |delta|;
errors spread over the state move it like a random walk, by the root of
their summed squares.  Test infrastructure only: it draws nothing the
simulator computes and holds none of its arithmetic.
"""
import numpy as np

N_PROJ = 4
_KEY = np.uint64(0x5DEECE66D1234567)
_BLOCK = 1 << 22


def _splitmix64(z: np.ndarray) -> np.ndarray:
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sketch(state: np.ndarray) -> np.ndarray:
    """The N_PROJ projections of a complex vector indexed 0..len-1."""
    a = np.asarray(state)
    # the top byte of the hash holds the four 2-bit weight fields: sum the
    # amplitudes per byte value once, then fold the 256 bins per projection
    bins = np.zeros(256, dtype=np.complex128)
    with np.errstate(over="ignore"):
        for start in range(0, a.size, _BLOCK):
            blk = a[start:start + _BLOCK].astype(np.complex128, copy=False)
            x = np.arange(start, start + blk.size, dtype=np.uint64)
            c = (_splitmix64(x ^ _KEY) >> np.uint64(56)).astype(np.intp)
            bins += np.bincount(c, weights=blk.real, minlength=256)
            bins += 1j * np.bincount(c, weights=blk.imag, minlength=256)
    phase = np.array([1, 1j, -1, -1j], dtype=np.complex128)
    v = np.arange(256)
    return np.array([np.dot(phase[(v >> (6 - 2 * k)) & 3], bins) for k in range(N_PROJ)])
