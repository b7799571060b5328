"""k-means initialisation.  Test infrastructure only.

The paper takes landmarks as k-means centroids of the range list (Section III)
but does not say how k-means is started.  Reading used here: the initial
centroids are the guide values at r distinct pixels drawn by a partial
Fisher-Yates shuffle of the pixel indices [0, N), driven by SplitMix64
(G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).

SplitMix64 state update and output, all arithmetic modulo 2^64:
    s <- s + 0x9E3779B97F4A7C15
    z <- s
    z <- (z xor (z >> 30)) * 0xBF58476D1CE4E5B9
    z <- (z xor (z >> 27)) * 0x94D049BB133111EB
    return z xor (z >> 31)

Draw of r distinct indices: for i = 0 .. r-1, j = i + (next() mod (N - i)),
swap entries i and j of the (virtual) identity array, take entry i.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.s = int(seed) & _M64

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)


def distinct_indices(n, r, seed):
    """r distinct integers from [0, n), in draw order."""
    if not (1 <= r <= n):
        raise ValueError("need 1 <= r <= n")
    g = SplitMix64(seed)
    swapped = {}
    out = np.empty(r, np.int64)
    for i in range(r):
        j = i + g.next() % (n - i)
        ai = swapped.get(i, i)
        aj = swapped.get(j, j)
        swapped[i], swapped[j] = aj, ai
        out[i] = aj
    return out
