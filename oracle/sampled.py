"""Algorithm 1 of Sec. 4.1.1 (the sampled forward for unweighted graphs),
distances only, written out step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a set of sources and a distinguished set S that contains them (the
random sample is an input, drawn by the caller):
  step 2  from every x in S, a k-limited breadth-first search: d'(x, v) is
          d(x, v) when v is within k hops of x, and infinite otherwise;
  step 3  the weighted graph H on S with edge weights d'(x, y);
  step 4  all-pairs shortest distances D_H in H (Floyd-Warshall);
  step 5  d(s, v) = min over x in S of D_H(s, x) + d'(x, v).
Every value is the length of a real walk, so the result never falls below the
true distance; it equals it when every shortest s-v path meets S at least
once in every k consecutive hops, which a random S of size about
sqrt(n) log n achieves with high probability for k = sqrt(n).  Step 6 (the
number of shortest paths as the number of minimising vertices) does not
count paths and is not computed.
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << np.int64(40)


def limited_bfs(g, x: int, k: int) -> np.ndarray:
    """Step 2: hop distances from x up to k hops (int64, INF beyond)."""
    d = np.full(g.n, INF, dtype=np.int64)
    d[x] = 0
    front = np.array([x], dtype=np.int64)
    for level in range(1, k + 1):
        if front.size == 0:
            break
        nb = np.concatenate([g.col[g.row_ptr[v]:g.row_ptr[v + 1]] for v in front])
        nb = np.unique(nb)
        nb = nb[d[nb] == INF]
        d[nb] = level
        front = nb
    return d


def floyd_warshall(H: np.ndarray) -> np.ndarray:
    """Step 4: all-pairs shortest distances of a weighted graph given by its
    (symmetric, INF-padded) weight matrix with zero diagonal."""
    D = H.copy()
    for k in range(D.shape[0]):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return np.minimum(D, INF)


def sampled_distances(g, sources, sample, k: int) -> np.ndarray:
    """Distances d(s, v) for every s in `sources` by Algorithm 1 with the
    distinguished set S = sources + sample (order kept, duplicates dropped)
    and search limit k.  Returns int64 [len(sources)][n], -1 where the walk
    found none."""
    if g.weight is not None:
        raise ValueError("Algorithm 1's limited search is for unweighted graphs")
    S = list(dict.fromkeys([int(s) for s in sources] + [int(x) for x in sample]))
    Dp = np.stack([limited_bfs(g, x, k) for x in S]) if S else np.zeros((0, g.n), np.int64)   # step 2
    H = Dp[:, S]                                                   # step 3
    np.fill_diagonal(H, 0)
    DH = floyd_warshall(H)                                         # step 4
    out = np.empty((len(sources), g.n), dtype=np.int64)
    for i, s in enumerate(sources):                                # step 5
        r = S.index(int(s))
        best = np.min(DH[r][:, None] + Dp, axis=0)
        out[i] = np.where(best >= INF, -1, best)
    return out
