"""Pins of the oracle's edge betweenness (each arc carries its edge's value,
ordered pairs, no halving): brute-force path enumeration from the definition,
closed forms, and identities with vertex betweenness."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import cross


def edge_of_arcs(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return list(zip(np.minimum(rows, g.col).tolist(), np.maximum(rows, g.col).tolist()))


def test_symmetric_and_nonnegative():
    g = gg.er_plus_tree(60, 4.0, 5)
    _, eb = oracle.edge_bc(g)
    arcs = edge_of_arcs(g)
    by_edge = {}
    for e, val in zip(arcs, eb):
        by_edge.setdefault(e, []).append(val)
    assert all(len(v) == 2 and v[0] == v[1] for v in by_edge.values())
    assert np.all(eb >= 1.0)  # every edge carries at least its own endpoints' pairs


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_brute_force_every_small_graph(n):
    """Every labelled graph on n vertices (n <= 5), disconnected ones included."""
    for mask in range(1 << (n * (n - 1) // 2)):
        g = gg.graph_from_bits(n, mask)
        _, eb = oracle.edge_bc(g)
        want = cross.brute_force_edges(g)
        for e, val in zip(edge_of_arcs(g), eb):
            w = float(want.get(e, 0))
            assert abs(val - w) <= 1e-12 * max(1.0, w), (n, mask, e)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_random_weighted(seed):
    g = gg.random_graph(7, 0.5, seed, weights=4)
    _, eb = oracle.edge_bc(g)
    want = cross.brute_force_edges(g)
    for e, val in zip(edge_of_arcs(g), eb):
        w = float(want.get(e, 0))  # a heavy edge may lie on no shortest path
        assert abs(val - w) <= 1e-12 * max(1.0, w)


@pytest.mark.parametrize("N", [2, 5, 9, 30])
def test_path_closed_form(N):
    """P_N: edge (i, i+1) separates i+1 vertices from N-1-i: 2 (i+1)(N-1-i)."""
    g = gg.path(N)
    _, eb = oracle.edge_bc(g)
    for e, val in zip(edge_of_arcs(g), eb):
        i = e[0]
        assert val == 2 * (i + 1) * (N - 1 - i)


@pytest.mark.parametrize("seed", range(4))
def test_tree_closed_form(seed):
    """Tree: an edge splitting the vertices into A and B carries 2 |A| |B|."""
    g = gg.random_tree(80, seed)
    _, eb = oracle.edge_bc(g)
    adj = [[] for _ in range(g.n)]
    for a, b in edge_of_arcs(g):
        adj[a].append(b)
    for (a, b), val in zip(edge_of_arcs(g), eb):
        # size of the side of b when the edge is removed
        side, stack = {b}, [b]
        while stack:
            v = stack.pop()
            lo, hi = g.row_ptr[v], g.row_ptr[v + 1]
            for x in g.col[lo:hi]:
                x = int(x)
                if {v, x} == {a, b} or x in side:
                    continue
                side.add(x)
                stack.append(x)
        k = len(side)
        assert val == 2 * k * (g.n - k)


@pytest.mark.parametrize("r", [1, 2, 5, 12])
def test_odd_cycle_closed_form(r):
    """C_{2r+1}: every edge carries r(r+1) (sum over ordered pairs of their
    distance, N r(r+1), spread evenly over N edges)."""
    g = gg.cycle(2 * r + 1)
    _, eb = oracle.edge_bc(g)
    assert np.all(eb == r * (r + 1))


def test_complete_graph():
    _, eb = oracle.edge_bc(gg.complete(9))
    assert np.all(eb == 2.0)


@pytest.mark.parametrize("weighted", [False, True])
def test_vertex_identity(weighted):
    """Sum of EB over the edges at v = 2 BC(v) + 2 (|reach(v)| - 1): a pair
    with v as an endpoint crosses one edge at v, a pair through v two."""
    g = gg.disjoint_union(gg.er_plus_tree(70, 5.0, 9), gg.path(6))
    if weighted:
        g = gg.with_uniform_weights(g, 9, 1, 7)
    bc, eb = oracle.edge_bc(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    at_v = np.bincount(rows, weights=eb, minlength=g.n)
    reach = np.array([np.count_nonzero(oracle.sssp_u64(g, v)[0] >= 0) for v in range(g.n)])
    assert np.allclose(at_v, 2 * bc + 2 * (reach - 1), rtol=1e-12, atol=1e-9)


def test_total_is_sum_of_distances():
    """Unit weights: the sum over edges of EB is the sum over ordered reachable
    pairs of d(s,t) (each shortest path has d(s,t) edges)."""
    g = gg.er_plus_tree(90, 4.0, 3)
    _, eb = oracle.edge_bc(g)
    total = sum(int(np.sum(oracle.sssp_u64(g, s)[0].clip(min=0))) for s in range(g.n))
    assert abs(eb.sum() / 2 - total) <= 1e-9 * total


def test_sources_add_up():
    """EB over a multiset of sources is the sum of the single-source values."""
    g = gg.er_plus_tree(40, 4.0, 2)
    src = np.array([3, 7, 7, 20], np.int32)
    _, eb = oracle.edge_bc(g, src)
    parts = sum(oracle.edge_bc(g, np.array([s], np.int32))[1] for s in src)
    assert np.allclose(eb, parts, rtol=1e-13, atol=0)
