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


def draw_weighted(beta, k: int, seed: int):
    """Node-weighted sample of Sec. 5: exactly k nodes (all nodes with
    beta > 0 when there are at most k of them), node v included with
    probability min(1, beta(v)/tau), where tau solves
    sum_v min(1, beta(v)/tau) = k (VarOpt's threshold).  Integer weights,
    exact integer arithmetic throughout:

    * threshold: nodes with beta > 0, heaviest first (ties by id); the number
      L of heavy nodes is the first L with beta_(L+1) * (k - L) < R_L, R_L the
      weight of all but the L heaviest; tau = R_L / (k - L) = R / m;
    * the heavy nodes are taken; the light ones get masses beta(v) * m, out of
      Q = R per unit, summing to m * Q, and pass in a random order (the full
      Fisher-Yates permutation of draw_samples(n, n, seed)) through ordered
      pivotal sampling (Deville & Tille's splitting method): the current
      pivot with mass a meets the next node with mass b; if a + b <= Q, one
      of the two gets a + b (the pivot with probability a/(a+b)) and the
      other is dropped; else one of the two is taken with mass Q (the pivot
      with probability (Q-b)/(2Q-a-b)) and the other keeps a + b - Q; a
      pivot that reaches Q is taken;
    * each decision with probability num/den draws x = next() from the same
      generator (after the permutation's draws) and is "yes" iff
      x * den < num * 2^64.
    Returns (sample ids in increasing order, per-sample light flags, R, m);
    when every positive node is taken, R = 0, m = 1 and none is light."""
    n = len(beta)
    pos = [v for v in range(n) if beta[v] > 0]
    if len(pos) <= k:
        return sorted(pos), [False] * len(pos), 0, 1
    heavy_first = sorted(pos, key=lambda v: (-beta[v], v))
    R = sum(beta[v] for v in pos)
    L = 0
    while not (beta[heavy_first[L]] * (k - L) < R):
        R -= beta[heavy_first[L]]
        L += 1
    m = k - L
    heavy = set(heavy_first[:L])
    rng = SplitMix64(seed)
    perm = list(range(n))
    for i in range(n):  # the same draws as draw_samples(n, n, seed)
        j = i + rng.below(n - i)
        perm[i], perm[j] = perm[j], perm[i]
    Q = R

    def yes(num, den):
        return rng.next() * den < (num << 64)

    taken = set(heavy)
    cur, ca = None, 0
    for v in perm:
        if beta[v] == 0 or v in heavy:
            continue
        b = beta[v] * m
        if cur is None:
            cur, ca = v, b
            continue
        s = ca + b
        if s <= Q:
            if not yes(ca, s):
                cur = v
            ca = s
            if ca == Q:
                taken.add(cur)
                cur, ca = None, 0
        else:
            if yes(Q - b, 2 * Q - s):
                taken.add(cur)
                cur = v
            else:
                taken.add(v)
            ca = s - Q
    assert cur is None, "pivotal sampling left a fractional mass"
    sample = sorted(taken)
    assert len(sample) == k
    return sample, [v not in heavy for v in sample], R, m
