"""Seeded synthetic graphs in symmetric CSR form.

Every generator returns a :class:`Graph`: an undirected simple graph stored as a
symmetric CSR (both arcs of every edge, rows sorted by column, no self-loops or
duplicates), optionally with a positive integer weight per arc that is equal on
both arcs of an edge.  This module only builds inputs; it holds none of the
betweenness arithmetic and is shared by the oracle side and the GPU side.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from .rng import BASE_SEED, Stream, substream


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    weight: Optional[np.ndarray] = None  # uint32[nnz] or None (unit weights)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    @property
    def m(self) -> int:
        """Undirected edge count (arcs / 2)."""
        return int(self.col.size // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edges(self):
        """Undirected edges (u < v) and their weights (or None)."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        keep = rows < self.col
        w = None if self.weight is None else self.weight[keep]
        return rows[keep], self.col[keep].astype(np.int64), w

    def relabel(self, perm: np.ndarray) -> "Graph":
        """Graph with vertex v renamed perm[v]."""
        u, v, w = self.edges()
        perm = np.asarray(perm, dtype=np.int64)
        return from_edges(self.n, perm[u], perm[v], w, name=self.name + "-relabelled")


def from_edges(n: int, u, v, weight=None, name: str = "", meta=None) -> Graph:
    """Symmetric, deduplicated CSR from an undirected edge list.

    Self-loops are dropped.  Duplicate edges are merged; with weights, the
    first occurrence (in input order) of an undirected edge keeps its weight.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size != v.size:
        raise ValueError("u and v differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    a, b = np.minimum(u, v), np.maximum(u, v)
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    first.sort()
    a, b = a[first], b[first]
    w = None
    if weight is not None:
        w = np.asarray(weight, dtype=np.uint32).ravel()[keep][first]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(rows, minlength=n))
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("too many arcs for an int32 CSR")
    wa = None
    if w is not None:
        wa = np.concatenate([w, w])[order].astype(np.uint32)
    return Graph(n, row_ptr.astype(np.int32), cols.astype(np.int32), wa, name, dict(meta or {}))


def largest_component(g: Graph) -> Graph:
    """Induced subgraph on the largest connected component, ids compacted in order.

    Among equally large components the one holding the smallest vertex id wins.
    """
    if g.n == 0:
        return g
    mat = csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, label = connected_components(mat, directed=False)
    sizes = np.bincount(label, minlength=ncomp)
    best = sizes.max()
    cand = np.flatnonzero(sizes == best)
    first_vertex = np.array([np.flatnonzero(label == c)[0] for c in cand])
    lab = cand[np.argmin(first_vertex)]
    keepv = label == lab
    newid = -np.ones(g.n, dtype=np.int64)
    newid[keepv] = np.arange(int(keepv.sum()))
    u, v, w = g.edges()
    ke = keepv[u]
    meta = dict(g.meta)
    meta["components_before_lcc"] = int(ncomp)
    meta["n_before_lcc"] = int(g.n)
    return from_edges(int(keepv.sum()), newid[u[ke]], newid[v[ke]], None if w is None else w[ke],
                      name=g.name, meta=meta)


def with_uniform_weights(g: Graph, seed: int, lo: int = 1, hi: int = 255) -> Graph:
    """Integer weights uniform in [lo, hi] per undirected edge, equal on both arcs."""
    u, v, _ = g.edges()
    s = Stream(substream(seed, 0x77))
    w = s.bounded(np.full(u.size, hi - lo + 1)) + lo
    out = from_edges(g.n, u, v, w, name=g.name + f"-w{lo}..{hi}", meta=g.meta)
    return out


def with_constant_weight(g: Graph, c: int) -> Graph:
    u, v, _ = g.edges()
    return from_edges(g.n, u, v, np.full(u.size, c), name=g.name + f"-w{c}", meta=g.meta)


# ----------------------------------------------------------------------------
# Random families
# ----------------------------------------------------------------------------

def _pair_from_index(k: np.ndarray):
    """Inverse of k = v(v-1)/2 + w for 0 <= w < v."""
    k = k.astype(np.int64)
    v = np.floor((1.0 + np.sqrt(1.0 + 8.0 * k.astype(np.float64))) / 2.0).astype(np.int64)
    # integer corrections for floating-point rounding
    for _ in range(3):
        too_big = v * (v - 1) // 2 > k
        v = np.where(too_big, v - 1, v)
        too_small = (v + 1) * v // 2 <= k
        v = np.where(too_small, v + 1, v)
    w = k - v * (v - 1) // 2
    return v, w


def erdos_renyi_edges(n: int, p: float, seed: int):
    """G(n, p) edge list by geometric skipping (Batagelj and Brandes, PRE 2005).

    Candidate pairs (v, w), w < v, are enumerated in the order
    k = v(v-1)/2 + w; the gap to the next chosen pair is geometric with
    parameter p, drawn as floor(log(1 - r) / log(1 - p)).
    """
    total = n * (n - 1) // 2
    if total == 0 or p <= 0.0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if p >= 1.0:
        k = np.arange(total, dtype=np.int64)
        return _pair_from_index(k)
    s = Stream(substream(seed, 0xE4))
    lq = np.log1p(-p)
    chunks = []
    pos = -1
    block = max(1024, int(total * p * 1.1) + 1024)
    while True:
        r = s.doubles(block)
        skip = np.floor(np.log1p(-r) / lq).astype(np.int64) + 1
        ks = pos + np.cumsum(skip)
        inside = ks < total
        chunks.append(ks[inside])
        if not inside.all():
            break
        pos = int(ks[-1])
    k = np.concatenate(chunks)
    return _pair_from_index(k)


def random_recursive_tree_edges(n: int, seed: int):
    """Random recursive spanning tree on a random permutation pi:
    for i = 1..n-1, edge (pi[i], pi[j]) with j uniform in [0, i)."""
    if n <= 1:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    s = Stream(substream(seed, 0x7E))
    pi = s.permutation(n)
    j = s.bounded(np.arange(1, n))
    return pi[1:], pi[j]


def er_plus_tree(n: int, avg_degree: float, seed: int, name: str = "") -> Graph:
    """G(n, p = avg_degree/(n-1)) united with a random recursive spanning tree."""
    p = avg_degree / (n - 1)
    a, b = erdos_renyi_edges(n, p, seed)
    c, d = random_recursive_tree_edges(n, seed)
    return from_edges(n, np.concatenate([a, c]), np.concatenate([b, d]),
                      name=name or f"er{n}-d{avg_degree:g}+tree")


def erdos_renyi(n: int, avg_degree: float, seed: int, lcc: bool = True, name: str = "") -> Graph:
    p = avg_degree / (n - 1)
    a, b = erdos_renyi_edges(n, p, seed)
    g = from_edges(n, a, b, name=name or f"er{n}-d{avg_degree:g}")
    return largest_component(g) if lcc else g


def rmat_edges(scale: int, edgefactor: int, seed: int, a=0.57, b=0.19, c=0.19):
    """R-MAT edge draws: each of edgefactor * 2^scale edges picks one of four
    quadrants per bit level with probabilities (a, b, c, 1-a-b-c)."""
    ne = edgefactor << scale
    src = np.zeros(ne, dtype=np.int64)
    dst = np.zeros(ne, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lev in range(scale):
        u = Stream(substream(seed, 0x4D, lev)).doubles(ne)
        row_bit = (u >= ab).astype(np.int64)
        col_bit = (((u >= a) & (u < ab)) | (u >= abc)).astype(np.int64)
        src |= row_bit << lev
        dst |= col_bit << lev
    perm = Stream(substream(seed, 0x9E)).permutation(1 << scale)
    return perm[src], perm[dst]


def rmat(scale: int, edgefactor: int, seed: int, lcc: bool = True, name: str = "") -> Graph:
    """Symmetrised, deduplicated, loop-free R-MAT graph (largest component by default)."""
    s, d = rmat_edges(scale, edgefactor, seed)
    g = from_edges(1 << scale, s, d, name=name or f"rmat{scale}-ef{edgefactor}")
    return largest_component(g) if lcc else g


def watts_strogatz(n: int, k: int, p: float, seed: int, name: str = "") -> Graph:
    """Watts-Strogatz small world: ring lattice joining each vertex to its k/2
    nearest neighbours on each side, then each lattice edge (i, i+j), taken
    i-major for j = 1..k/2, is rewired with probability p to (i, x) where x is
    uniform over vertices that are neither i nor already adjacent to i."""
    half = k // 2
    i = np.repeat(np.arange(n, dtype=np.int64), half)
    t = (i + np.tile(np.arange(1, half + 1, dtype=np.int64), n)) % n
    lo, hi = np.minimum(i, t), np.maximum(i, t)
    edges = set((lo * n + hi).tolist())
    deg = np.bincount(np.concatenate([lo, hi]), minlength=n) if n else np.zeros(0, np.int64)
    deg = deg.tolist()
    s = Stream(substream(seed, 0x3A))
    coins = np.flatnonzero(s.doubles(n * half) < p)
    cand = s.bounded(np.full(max(4 * coins.size, 16), max(n, 1))).tolist()
    ci = 0
    for idx in coins.tolist():
        a, b = int(i[idx]), int(t[idx])
        key = min(a, b) * n + max(a, b)
        if key not in edges or deg[a] >= n - 1:
            continue
        while True:
            if ci == len(cand):
                cand = s.bounded(np.full(len(cand), n)).tolist()
                ci = 0
            x = cand[ci]
            ci += 1
            if x != a and (min(a, x) * n + max(a, x)) not in edges:
                break
        edges.discard(key)
        deg[b] -= 1
        edges.add(min(a, x) * n + max(a, x))
        deg[x] += 1
    keys = np.fromiter(edges, dtype=np.int64, count=len(edges))
    return from_edges(n, keys // max(n, 1), keys % max(n, 1), name=name or f"ws{n}-k{k}-p{p:g}")


def sample_sources(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct vertices, uniform without replacement, sorted ascending."""
    if count > n:
        raise ValueError("sample larger than the vertex set")
    perm = Stream(substream(seed, 0x5A)).permutation(n)
    return np.sort(perm[:count]).astype(np.int32)


# ----------------------------------------------------------------------------
# Deterministic families (closed-form test graphs)
# ----------------------------------------------------------------------------

def path(n: int) -> Graph:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, name=f"path{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, name=f"cycle{n}")


def star(n: int) -> Graph:
    """K_{1,n-1} with centre 0."""
    i = np.arange(1, n)
    return from_edges(n, np.zeros(n - 1, np.int64), i, name=f"star{n}")


def complete(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return from_edges(n, iu[0], iu[1], name=f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    """K_{a,b}: side A = 0..a-1, side B = a..a+b-1."""
    uu, vv = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, uu.ravel(), vv.ravel(), name=f"K{a},{b}")


def grid(rows: int, cols: int) -> Graph:
    """rows x cols lattice; vertex (x, y) has id x * cols + y."""
    ids = np.arange(rows * cols).reshape(rows, cols)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(rows * cols, u, v, name=f"grid{rows}x{cols}")


def random_tree(n: int, seed: int) -> Graph:
    a, b = random_recursive_tree_edges(n, seed)
    return from_edges(n, a, b, name=f"tree{n}")


def disjoint_union(*gs: Graph) -> Graph:
    us, vs, ws = [], [], []
    off = 0
    weighted = any(g.weight is not None for g in gs)
    for g in gs:
        u, v, w = g.edges()
        us.append(u + off)
        vs.append(v + off)
        if weighted:
            ws.append(np.ones(u.size, np.uint32) if w is None else w)
        off += g.n
    w = np.concatenate(ws) if weighted else None
    return from_edges(off, np.concatenate(us), np.concatenate(vs), w,
                      name="+".join(g.name for g in gs))


def kkp_undirected(k: int) -> Graph:
    """Undirected, weighted version of the tripartite lower-bound construction:
    layers u_0..u_{k-1}, v_0..v_{k-1}, w_0..w_{k-1}; every u_i joins every v_j
    and every v_j joins every w_l; edges at v_0 weigh 1, all others weigh 3.
    Ids: u_i = i, v_j = k + j, w_l = 2k + l."""
    us, vs, ws = [], [], []
    for i in range(k):
        for j in range(k):
            us.append(i)
            vs.append(k + j)
            ws.append(1 if j == 0 else 3)
    for j in range(k):
        for l in range(k):
            us.append(k + j)
            vs.append(2 * k + l)
            ws.append(1 if j == 0 else 3)
    return from_edges(3 * k, us, vs, ws, name=f"kkp{k}")


def graph_from_bits(n: int, bits: int) -> Graph:
    """The labelled graph on n vertices whose i-th pair (in triu order) is an
    edge iff bit i of ``bits`` is set."""
    iu = np.triu_indices(n, 1)
    sel = np.array([(bits >> i) & 1 for i in range(iu[0].size)], dtype=bool)
    return from_edges(n, iu[0][sel], iu[1][sel], name=f"g{n}:{bits}")


def random_graph(n: int, p: float, seed: int, weights: Optional[int] = None) -> Graph:
    """Small G(n, p) (possibly disconnected), optional weights in [1, weights]."""
    a, b = erdos_renyi_edges(n, p, seed)
    g = from_edges(n, a, b, name=f"gnp{n}-{p:g}-{seed}")
    if weights is not None:
        g = with_uniform_weights(g, seed, 1, weights)
    return g


# ----------------------------------------------------------------------------
# The benchmark workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    "er1024": "ER n=1024, average degree 8, plus a random spanning tree; all 1024 sources",
    "rmat16": "RMAT scale 16, edgefactor 16, (a,b,c,d)=(.57,.19,.19,.05), largest component; all sources",
    "er16384": "ER n=16384, average degree 256, largest component; all sources",
    "ws4096": "4096 Watts-Strogatz graphs, n ~ U{64..4096}, k=6, p=0.1; all sources of every graph",
    "rmat20w": "RMAT scale 20, largest component, weights U{1..255}; 4096 sampled sources",
    "er16384w4": "ER n=16384, average degree 256, largest component, weights U{1..4}; all sources",
}


def workload_seed(index: int) -> int:
    return BASE_SEED + index


def er1024() -> Graph:
    return er_plus_tree(1024, 8.0, workload_seed(0), name="er1024")


def rmat16() -> Graph:
    return rmat(16, 16, workload_seed(1), name="rmat16")


def er16384() -> Graph:
    return erdos_renyi(16384, 256.0, workload_seed(2), name="er16384")


def er16384w4() -> Graph:
    """The er16384 graph with weights U{1..4} per undirected edge."""
    g = with_uniform_weights(er16384(), workload_seed(5), 1, 4)
    g.name = "er16384w4"
    return g


def ws_batch(count: int = 4096, nmin: int = 64, nmax: int = 4096, seed: Optional[int] = None):
    """``count`` Watts-Strogatz graphs with n uniform in [nmin, nmax]."""
    seed = workload_seed(3) if seed is None else seed
    sizes = Stream(substream(seed, 0x51)).bounded(np.full(count, nmax - nmin + 1)) + nmin
    return [watts_strogatz(int(sz), 6, 0.1, substream(seed, 0x60, g), name=f"ws{g}")
            for g, sz in enumerate(sizes)]


def rmat20w():
    """(graph, sources): RMAT-20 largest component with weights U{1..255},
    plus 4096 sorted sources sampled without replacement."""
    seed = workload_seed(4)
    g = rmat(20, 16, seed, name="rmat20")
    g = with_uniform_weights(g, seed, 1, 255)
    return g, sample_sources(g.n, 4096, seed)


def rmat16_sampled(count: int = 1024):
    """(graph, sources, sample) for the sampled forward of Sec. 4.1.1 on
    RMAT-16: ``count`` sources and a uniform sample of ceil(sqrt(n) ln n)
    vertices, both without replacement, drawn independently."""
    g = rmat16()
    seed = workload_seed(6)
    size = int(np.ceil(np.sqrt(g.n) * np.log(g.n)))
    return g, sample_sources(g.n, count, seed), sample_sources(g.n, size, seed + 1)
