"""Subset counts by two row sums over a set of columns: a dynamic programme
in numpy, shared by tests that check a residue class's 1-D hit count at
sizes beyond brute force.  It holds none of the solver's or the oracle's
arithmetic."""
import numpy as np


def half_counts(a1, a2):
    """N[s1, s2] = #{subsets T of the columns : sum a1[T] = s1, sum a2[T] = s2}."""
    a1, a2 = np.asarray(a1, dtype=np.int64), np.asarray(a2, dtype=np.int64)
    S1, S2 = int(a1.sum()), int(a2.sum())
    N = np.zeros((S1 + 1, S2 + 1), dtype=np.int64)
    N[0, 0] = 1
    for x, y in zip(a1.tolist(), a2.tolist()):
        N[x:, y:] += N[:S1 + 1 - x, :S2 + 1 - y].copy()
    return N
