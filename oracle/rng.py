"""Counter-based SplitMix64 Rademacher probes (oracle side).

SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each output is the state passed through the MurmurHash3
finaliser variant mix64 (shift 30, multiply 0xBF58476D1CE4E5B9, shift 27,
multiply 0x94D049BB133111EB, shift 31).

Counter form used by this project: the k-th output (k = 0, 1, ...) of the
stream seeded with ``seed`` is mix64(seed + (k + 1) * golden) modulo 2^64.
Probe column c of a block of N-vectors uses counters k = c * N + i,
i = 0..N-1, and the entry is -1 when bit 63 of the output is set, +1 otherwise.

This is written independently of the GPU generator; a GPU test checks that
both produce the same stream.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number ``counters`` of the SplitMix64 stream seeded by ``seed``."""
    with np.errstate(over="ignore"):
        k = counters.astype(np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def rademacher(seed: int, col0: int, ncols: int, N: int) -> np.ndarray:
    """N x ncols matrix of +-1 (FP64); column j uses counters (col0+j)*N + i."""
    out = np.empty((N, ncols), dtype=np.float64)
    i = np.arange(N, dtype=np.uint64)
    for j in range(ncols):
        z = splitmix64(seed, np.uint64(col0 + j) * np.uint64(N) + i)
        out[:, j] = np.where((z >> np.uint64(63)) != 0, -1.0, 1.0)
    return out
