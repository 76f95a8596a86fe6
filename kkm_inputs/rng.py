"""Counter-based random draws consumed by the method, from published definitions.

Generator
---------
SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the odd constant
0x9E3779B97F4A7C15 and each output is the state passed through the 64-bit
finaliser ``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31``.

Streams
-------
Every use gets its own stream whose initial state is derived from
``(seed, purpose, batch)`` by two rounds of the finaliser:
``key = mix(seed + G*(1+purpose)); key = mix(key + G*(1+batch))`` (mod 2^64).

Derived draws
-------------
* bounded integers in [0, n): D. Lemire, "Fast random integer generation in an
  interval", ACM TOMACS 2019 (multiply-shift with rejection);
* uniform doubles in [0, 1): ``(r >> 11) * 2**-53``;
* a landmark set: the first l positions of a partial Fisher-Yates shuffle of
  [0, n), sorted ascending.

The HIP library carries its own C++ implementation of the same definitions
(used when the caller passes no explicit draws); the two are checked against
each other by the CPU tests.
"""
from __future__ import annotations

import math
import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB

PURPOSE_LANDMARKS = 0
PURPOSE_INIT_LABELS = 1
PURPOSE_KMEANSPP = 2
PURPOSE_SUBSAMPLE = 3


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * MUL1) & MASK64
    z = ((z ^ (z >> 27)) * MUL2) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, state: int):
        self.state = state & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + GOLDEN) & MASK64
        return mix64(self.state)

    def bounded(self, n: int) -> int:
        """Uniform integer in [0, n), Lemire's nearly-divisionless method."""
        if n <= 0:
            raise ValueError("bounded(n) needs n >= 1")
        x = self.next_u64()
        m = x * n
        low = m & MASK64
        if low < n:
            threshold = ((1 << 64) - n) % n
            while low < threshold:
                x = self.next_u64()
                m = x * n
                low = m & MASK64
        return m >> 64

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def stream(seed: int, purpose: int, batch: int = 0) -> SplitMix64:
    key = mix64((seed + GOLDEN * (1 + purpose)) & MASK64)
    key = mix64((key + GOLDEN * (1 + batch)) & MASK64)
    return SplitMix64(key)


def landmark_count(n: int, s: float) -> int:
    """Number of landmarks in a batch of n samples at sparsity s (s = |L| B / N).

    Rounded half up and clamped to [1, n]."""
    return int(min(n, max(1, math.floor(s * n + 0.5))))


def draw_landmarks(seed: int, batch: int, n: int, s: float) -> np.ndarray:
    """Batch-local landmark indices, uniform without replacement, ascending."""
    ell = landmark_count(n, s)
    if ell == n:
        return np.arange(n, dtype=np.int64)
    g = stream(seed, PURPOSE_LANDMARKS, batch)
    idx = list(range(n))
    for k in range(ell):
        r = k + g.bounded(n - k)
        idx[k], idx[r] = idx[r], idx[k]
    return np.sort(np.asarray(idx[:ell], dtype=np.int64))


def batch_index_sets(N: int, B: int, sampling: str = "stride") -> list[np.ndarray]:
    """Global sample indices of each mini-batch.

    stride: batch i = {i, i+B, i+2B, ...}; block: contiguous runs whose sizes
    differ by at most one, the longer runs first."""
    if sampling == "stride":
        return [np.arange(i, N, B, dtype=np.int64) for i in range(B)]
    if sampling == "block":
        q, r = divmod(N, B)
        out, start = [], 0
        for i in range(B):
            n = q + (1 if i < r else 0)
            out.append(np.arange(start, start + n, dtype=np.int64))
            start += n
        return out
    raise ValueError(sampling)


def draw_all_landmarks(seed: int, N: int, B: int, s: float, sampling: str = "stride") -> list[np.ndarray]:
    return [draw_landmarks(seed, i, len(ix), s) for i, ix in enumerate(batch_index_sets(N, B, sampling))]


def draw_kmpp_uniforms(seed: int, C: int) -> np.ndarray:
    """C uniforms in [0,1): the first picks the first medoid, the others drive D^2 sampling."""
    g = stream(seed, PURPOSE_KMEANSPP, 0)
    return np.array([g.uniform() for _ in range(C)], dtype=np.float64)


def draw_init_labels(seed: int, n: int, C: int) -> np.ndarray:
    """Random initial labels for the n samples of batch 0, in batch order."""
    g = stream(seed, PURPOSE_INIT_LABELS, 0)
    return np.array([g.bounded(C) for _ in range(n)], dtype=np.int32)


def draw_subsample(seed: int, N: int, k: int) -> np.ndarray:
    """k distinct indices of [0, N), ascending (evaluation subsamples)."""
    k = min(k, N)
    g = stream(seed, PURPOSE_SUBSAMPLE, 0)
    chosen: dict[int, int] = {}
    out = np.empty(k, dtype=np.int64)
    for j in range(k):
        r = j + g.bounded(N - j)
        vj, vr = chosen.get(j, j), chosen.get(r, r)
        chosen[j], chosen[r] = vr, vj
        out[j] = vr
    return np.sort(out)
