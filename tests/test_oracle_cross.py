"""The Brandes oracle against independent cross-oracles (CPU only):
brute-force path enumeration from the definitions, Floyd-Warshall counts with
Algorithm 2, and the dense algebraic method in exact arithmetic."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import cross


def _rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0))) if y.size else 0.0


def _check_brute(g):
    dist, count, bf = cross.brute_force(g)
    bc = oracle.bc(g)
    assert _rel_err(bc, [float(x) for x in bf]) <= 1e-13
    for s in range(g.n):
        d, sigma, _ = oracle.sssp(g, s)
        for t in range(g.n):
            if dist[s][t] is None:
                assert d[t] == -1 and sigma[t] == 0
            else:
                assert d[t] == dist[s][t]
                assert sigma[t] == count[s][t]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_brute_force_every_labelled_graph(n):
    """All 2^(n(n-1)/2) labelled graphs on n <= 5 vertices, disconnected ones included."""
    pairs = n * (n - 1) // 2
    for bits in range(1 << pairs):
        _check_brute(gg.graph_from_bits(n, bits))


def test_brute_force_sampled_six_vertex_graphs():
    s = gg.Stream(606)
    for bits in s.bounded(np.full(300, 1 << 15)):
        _check_brute(gg.graph_from_bits(6, int(bits)))


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random_unweighted(seed):
    n = 6 + seed % 3
    _check_brute(gg.random_graph(n, 0.3 + 0.05 * (seed % 5), seed))


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random_weighted(seed):
    n = 5 + seed % 4
    _check_brute(gg.random_graph(n, 0.35 + 0.05 * (seed % 5), 100 + seed, weights=1 + seed % 6))


def test_brute_force_tripartite():
    _check_brute(gg.kkp_undirected(2))
    _check_brute(gg.kkp_undirected(3))


@pytest.mark.parametrize("seed,n,p,w", [(1, 60, 0.08, None), (2, 150, 0.03, None), (3, 200, 0.02, None),
                                        (4, 80, 0.06, 5), (5, 120, 0.04, 255), (6, 90, 0.05, 2)])
def test_algorithm2_random(seed, n, p, w):
    g = gg.random_graph(n, p, seed, weights=w)
    D, L = cross.allpairs_counts(g)
    assert _rel_err(oracle.bc(g), cross.algorithm2(D, L)) <= 1e-12
    for s in range(0, n, 7):
        d, sigma, _ = oracle.sssp(g, s)
        reach = D[s] < cross.INF
        np.testing.assert_array_equal(d[reach], D[s][reach])
        assert np.all(d[~reach] == -1)
        assert [int(x) for x in sigma] == [int(x) for x in L[s]]


def test_algorithm2_exact_small():
    g = gg.random_graph(14, 0.3, 77)
    D, L = cross.allpairs_counts(g, exact=True)
    ex = cross.algorithm2(D, L, exact=True)
    assert _rel_err(oracle.bc(g), [float(x) for x in ex]) <= 1e-14


def test_algorithm2_er1024_workload():
    """The whole 1024-vertex workload against Floyd-Warshall + Algorithm 2."""
    g = gg.er1024()
    D, L = cross.allpairs_counts(g)
    assert _rel_err(oracle.bc(g), cross.algorithm2(D, L)) <= 1e-12


@pytest.mark.parametrize("seed,n,p", [(1, 10, 0.3), (2, 14, 0.2), (3, 16, 0.25), (4, 12, 0.15)])
def test_algebraic_method_exact(seed, n, p):
    g = gg.random_graph(n, p, seed)
    D, Lam, Delta, bc = cross.algebraic(g)
    assert _rel_err(oracle.bc(g), [float(x) for x in bc]) <= 1e-13
    for s in range(n):
        d, sigma, delta = oracle.sssp(g, s)
        np.testing.assert_array_equal(d, D[s])
        assert [int(x) for x in sigma] == [int(x) for x in Lam[s]]
        np.testing.assert_allclose(delta, [float(x) for x in Delta[s]], rtol=1e-13, atol=1e-13)


def test_algebraic_method_grid():
    g = gg.grid(4, 4)
    _, _, _, bc = cross.algebraic(g)
    assert _rel_err(oracle.bc(g), [float(x) for x in bc]) <= 1e-14


@pytest.mark.parametrize("seed,n,p,wmax", [(11, 7, 0.45, 3), (12, 8, 0.4, 5), (13, 6, 0.6, 8), (14, 8, 0.35, 2)])
def test_algebraic_weighted_equals_brute_force(seed, n, p, wmax):
    """The per-weight-class reading of Sec. 3.2 against the definitions
    (every simple path enumerated, exact rationals)."""
    g = gg.random_graph(n, p, seed, weights=wmax)
    D, Lam, Delta, bc = cross.algebraic_weighted(g)
    dist, count, bf = cross.brute_force(g)
    assert bc == bf
    for s_ in range(n):
        for t in range(n):
            want = -1 if dist[s_][t] is None else dist[s_][t]
            assert D[s_, t] == want
            assert int(Lam[s_, t]) == count[s_][t]


@pytest.mark.parametrize("seed,n,p,wmax", [(21, 30, 0.15, 4), (22, 40, 0.1, 8), (23, 25, 0.2, 1)])
def test_algebraic_weighted_matches_oracle(seed, n, p, wmax):
    """Per source: distances and counts exactly, dependencies to rounding;
    M = 1 reduces to the method of Sec. 3.1."""
    g = gg.random_graph(n, p, seed, weights=wmax)
    D, Lam, Delta, bc = cross.algebraic_weighted(g)
    assert _rel_err(oracle.bc(g), [float(x) for x in bc]) <= 1e-13
    for s_ in range(n):
        d, sigma, delta = oracle.sssp(g, s_)
        np.testing.assert_array_equal(d, D[s_])
        assert [int(x) for x in sigma] == [int(x) for x in Lam[s_]]
        np.testing.assert_allclose(delta, [float(x) for x in Delta[s_]], rtol=1e-13, atol=1e-13)
    if wmax == 1:
        assert bc == cross.algebraic(gg.random_graph(n, p, seed))[3]


def test_algebraic_weighted_gap_levels():
    """Weights leave empty distance levels between non-empty ones (a path of
    weight-5 edges): the forward stops only after M empty levels."""
    g = gg.with_constant_weight(gg.path(6), 5)
    D, Lam, _, bc = cross.algebraic_weighted(g)
    assert D[0, 5] == 25 and int(Lam[0, 5]) == 1
    assert _rel_err(oracle.bc(g), [float(x) for x in bc]) <= 1e-14
