"""Sample draw for the oracle (test infrastructure only).

The paper draws k nodes uniformly at random, as a set (Sec. 2; Alg. 1 input
step).  Both sides of a parity test must see the same sample, so the draw is
fixed by a published generator that each side implements on its own:

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the output mix
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
  z ^= z >> 31.
* Bounded integers in [0, s) by Lemire's multiply-shift with rejection
  ("Fast random integer generation in an interval", ACM TOMACS 2019), 64-bit
  draws, 128-bit products.
* Sample without replacement by a partial Fisher-Yates shuffle of 0..n-1: for
  i = 0..k-1, j = i + bounded(n - i), swap positions i and j, emit position i.
  The emitted order is the sample index order c_0, c_1, ...

This is the oracle's own implementation; the GPU library has a separate one.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, s: int) -> int:
        """Uniform integer in [0, s)."""
        assert 1 <= s <= MASK64
        m = self.next() * s
        low = m & MASK64
        if low < s:
            t = ((1 << 64) - s) % s
            while low < t:
                m = self.next() * s
                low = m & MASK64
        return m >> 64


def draw_samples(n: int, k: int, seed: int) -> list[int]:
    """k distinct node ids in [0, n), in draw order."""
    if not (1 <= k <= n):
        raise ValueError("need 1 <= k <= n")
    rng = SplitMix64(seed)
    moved: dict[int, int] = {}
    out = []
    for i in range(k):
        j = i + rng.below(n - i)
        a_i = moved.get(i, i)
        a_j = moved.get(j, j)
        moved[i] = a_j
        moved[j] = a_i
        out.append(a_j)
    return out
