"""The sampled forward of Sec. 4.1.1 (Algorithm 1, unweighted graphs),
distances only.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method, in this module's terms, for a set of sources and a distinguished
vertex set S that contains them (the random sample is an input, drawn by the
caller):
  * hop-limited searches: from every x in S a breadth-first search that stops
    after k hops gives d'(x, v), the distance when v is within k hops of x and
    infinite otherwise (limited_bfs);
  * a small weighted graph H on the vertices of S, the weight of x-y being
    d'(x, y), and its all-pairs distances D_H (floyd_warshall);
  * for every source s: d(s, v) = min over x in S of D_H(s, x) + d'(x, v)
    (sampled_distances).
Every value is the length of a real walk, so the result never falls below the
true distance; it equals it when every shortest s-v path meets S at least
once in every k consecutive hops, which a random S of size about
sqrt(n) log n achieves with high probability for k = sqrt(n).  The algorithm
also reads a path count off the number of minimising x; that is not a count
of shortest paths, and it is not computed here.
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << np.int64(40)


def limited_bfs(g, x: int, k: int) -> np.ndarray:
    """Hop distances from x up to k hops (int64, INF beyond): the limited
    search of Sec. 4.1.1."""
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
    """All-pairs shortest distances of the graph on the distinguished set,
    given by its (symmetric, INF-padded) weight matrix with zero diagonal."""
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
    # hop-limited distances from every distinguished vertex
    Dp = np.stack([limited_bfs(g, x, k) for x in S]) if S else np.zeros((0, g.n), np.int64)
    # the graph on S and its all-pairs distances
    H = Dp[:, S]
    np.fill_diagonal(H, 0)
    DH = floyd_warshall(H)
    # each source's distance: the best way through a distinguished vertex
    out = np.empty((len(sources), g.n), dtype=np.int64)
    for i, s in enumerate(sources):
        r = S.index(int(s))
        best = np.min(DH[r][:, None] + Dp, axis=0)
        out[i] = np.where(best >= INF, -1, best)
    return out
