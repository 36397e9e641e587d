"""Counter-based standard normals for the prescribed-current noise (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/qds.py).  The HIP path implements the same
published generator independently.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; constants as in Vigna's public reference code).  The
k-th output (k >= 1) of a stream seeded with ``seed`` is mix(seed + k * GAMMA)
mod 2^64, so any output can be computed directly from its index.  A normal
variate is formed by the Box-Muller transform (Box & Muller 1958) from outputs
2c+1 and 2c+2 of the counter c = (step << 32) | (lab column << 12) | row.
"""
import math

import numpy as np
import torch

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, k: np.ndarray) -> np.ndarray:
    """k-th output (k >= 1) of the SplitMix64 stream seeded with ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed) + k * GAMMA)


def counter(step: int, col: np.ndarray, row: np.ndarray) -> np.ndarray:
    col = np.asarray(col, dtype=np.uint64)
    row = np.asarray(row, dtype=np.uint64)
    return (np.uint64(step) << np.uint64(32)) | (col << np.uint64(12)) | row


def normal(seed: int, ctr: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        k1 = np.uint64(2) * ctr + np.uint64(1)
        k2 = np.uint64(2) * ctr + np.uint64(2)
    z1 = splitmix64_at(seed, k1)
    z2 = splitmix64_at(seed, k2)
    u1 = ((z1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (z2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def normal_field(seed: int, step: int, nx: int, nrows: int, w: int) -> torch.Tensor:
    """[nrows, nx] standard normals for H cells i (lab column i + w), rows j."""
    col = np.arange(nx, dtype=np.uint64)[None, :] + np.uint64(w)
    row = np.arange(nrows, dtype=np.uint64)[:, None]
    return torch.from_numpy(normal(seed, counter(step, col, row)))
