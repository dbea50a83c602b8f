"""Pins of the oracle against closed forms, invariants and the paper's printed
values.  CPU only.  Conventions: BC over ordered pairs, no halving (Sec. 1.1);
unordered values are BC/2."""
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return rows


# --------------------------------------------------------------- paper values

def test_paper_path_values():
    """Sec. 5, problem 2: P_{4k+1} has 0, 4k-1, 2(4k-2), ..., 4k^2 (unordered)."""
    for row in _read_golden("path_p4k1.txt"):
        n, vals = row[0], np.array(row[1:], dtype=np.float64)
        bc = oracle.bc(gg.path(n))
        np.testing.assert_array_equal(bc / 2.0, vals)


def test_paper_cycle_value_k1():
    """Sec. 5, problem 2: the k^2 value agrees with the definition at k = 1 only."""
    for n, val in _read_golden("cycle_c5.txt"):
        np.testing.assert_array_equal(oracle.bc(gg.cycle(n)) / 2.0, np.full(n, float(val)))


def test_lemma_3_3_farthest_pairs_have_zero_dependency():
    """Lemma 3.3: d(i,j) = Diam(G) implies delta_i*(j) = 0."""
    for g in [gg.grid(4, 5), gg.er_plus_tree(60, 3.0, 11), gg.cycle(9), gg.random_tree(40, 2)]:
        dists = [oracle.sssp(g, s)[0] for s in range(g.n)]
        diam = max(int(d.max()) for d in dists)
        hits = 0
        for s in range(g.n):
            d, _, delta = oracle.sssp(g, s)
            far = d == diam
            hits += int(far.sum())
            assert np.all(delta[far] == 0.0)
        assert hits > 0


# ----------------------------------------------------------------- distances

def test_distance_closed_forms():
    n = 11
    for s in range(n):
        d, _, _ = oracle.sssp(gg.path(n), s)
        np.testing.assert_array_equal(d, np.abs(np.arange(n) - s))
        d, _, _ = oracle.sssp(gg.cycle(n), s)
        k = np.abs(np.arange(n) - s)
        np.testing.assert_array_equal(d, np.minimum(k, n - k))
    r, c = 5, 7
    for s in range(r * c):
        d, _, _ = oracle.sssp(gg.grid(r, c), s)
        x, y = np.divmod(np.arange(r * c), c)
        np.testing.assert_array_equal(d, np.abs(x - s // c) + np.abs(y - s % c))
    d, _, _ = oracle.sssp(gg.complete(9), 4)
    assert d[4] == 0 and np.all(np.delete(d, 4) == 1)
    d, _, _ = oracle.sssp(gg.star(9), 3)
    assert d[3] == 0 and d[0] == 1 and np.all(np.delete(d, [0, 3]) == 2)


def test_distance_symmetry():
    g = gg.random_graph(40, 0.12, 5)
    D = np.array([oracle.sssp(g, s)[0] for s in range(g.n)])
    np.testing.assert_array_equal(D, D.T)
    gw = gg.random_graph(40, 0.12, 6, weights=9)
    Dw = np.array([oracle.sssp(gw, s)[0] for s in range(gw.n)])
    np.testing.assert_array_equal(Dw, Dw.T)


# --------------------------------------------------------------- path counts

@pytest.mark.parametrize("r,c", [(5, 6), (20, 20)])
def test_grid_path_counts_binomial(r, c):
    g = gg.grid(r, c)
    x, y = np.divmod(np.arange(r * c), c)
    for s in [0, c - 1, (r // 2) * c + c // 2, r * c - 1]:
        _, sigma, _ = oracle.sssp(g, s)
        dx, dy = np.abs(x - s // c), np.abs(y - s % c)
        want = [math.comb(int(a + b), int(a)) for a, b in zip(dx, dy)]
        assert list(sigma) == want


def test_grid_35_counts_exceed_u64_exactly():
    """C(68,34) > 2^64: the oracle keeps it exact and reports the excess."""
    g = gg.grid(35, 35)
    _, sigma, _ = oracle.sssp(g, 0)
    assert sigma[35 * 35 - 1] == math.comb(68, 34)
    assert sigma[35 * 35 - 1] > 2 ** 64 - 1
    _, above = oracle.bc(g, sources=[0], return_flags=True)
    assert above
    _, above34 = oracle.bc(gg.grid(34, 34), sources=[0], return_flags=True)
    assert not above34  # C(66,33) < 2^64


def test_complete_bipartite_counts():
    a, b = 4, 6
    g = gg.complete_bipartite(a, b)
    for s in range(a + b):
        _, sigma, _ = oracle.sssp(g, s)
        same = np.arange(a) if s < a else np.arange(a, a + b)
        other = b if s < a else a
        for t in same:
            assert sigma[t] == (1 if t == s else other)


def test_even_cycle_antipodal_and_tree_counts():
    n = 12
    for s in range(n):
        _, sigma, _ = oracle.sssp(gg.cycle(n), s)
        want = [2 if (t - s) % n == n // 2 else 1 for t in range(n)]
        assert list(sigma) == want
    t = gg.random_tree(50, 9)
    for s in range(0, 50, 7):
        _, sigma, _ = oracle.sssp(t, s)
        assert all(x == 1 for x in sigma)


def test_count_symmetry():
    g = gg.er_plus_tree(80, 6.0, 21)
    S = [oracle.sssp(g, s)[1] for s in range(g.n)]
    for s in range(g.n):
        for t in range(g.n):
            assert S[s][t] == S[t][s]


def test_walk_count_identity():
    """lambda_ij = (A^{d(i,j)})_ij: a shortest path is a walk of length d(i,j)
    and every walk of that length is a shortest path (Sec. 3.1.1)."""
    g = gg.er_plus_tree(30, 3.0, 8)
    A = np.zeros((g.n, g.n), dtype=object)
    A[:, :] = 0
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for r, c in zip(rows, g.col):
        A[r, c] = 1
    powers = [np.identity(g.n, dtype=object)]
    for _ in range(g.n):
        powers.append(powers[-1].dot(A))
    for s in range(g.n):
        d, sigma, _ = oracle.sssp(g, s)
        for t in range(g.n):
            assert sigma[t] == powers[d[t]][s, t]


# -------------------------------------------------------------- dependencies

@pytest.mark.parametrize("g", [gg.er_plus_tree(120, 4.0, 3), gg.grid(7, 9), gg.rmat(9, 8, 5)],
                         ids=["er120", "grid7x9", "rmat9"])
def test_dependency_invariants(g):
    for s in range(0, g.n, max(1, g.n // 17)):
        d, sigma, delta = oracle.sssp(g, s)
        reach = d >= 0
        # delta_s*(v) >= 0
        assert np.all(delta >= 0.0)
        # sum over v != s of delta_s*(v) = sum over reachable t != s of (d(s,t) - 1)
        lhs = delta[reach].sum() - delta[s]
        rhs = float((d[reach] - 1).sum() + 1)  # t = s contributes -1 in the sum; add it back
        assert lhs == pytest.approx(rhs, rel=1e-12)
        # the recurrence gives delta_s*(s) = |reach(s)| - 1
        assert delta[s] == pytest.approx(reach.sum() - 1, rel=1e-12)
        # no successor => zero dependency
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        succ = np.zeros(g.n, bool)
        dag = (d[rows] >= 0) & (d[g.col] == d[rows] + 1)
        succ[rows[dag]] = True
        assert np.all(delta[reach & ~succ] == 0.0)


# ----------------------------------------------------------------- BC values

@pytest.mark.parametrize("n", [1, 2, 3, 8, 33])
def test_bc_path(n):
    i = np.arange(n)
    np.testing.assert_array_equal(oracle.bc(gg.path(n)), 2.0 * i * (n - 1 - i))


@pytest.mark.parametrize("n", [2, 3, 10, 101])
def test_bc_star(n):
    bc = oracle.bc(gg.star(n))
    assert bc[0] == (n - 1) * (n - 2)
    assert np.all(bc[1:] == 0.0)


def test_bc_complete():
    assert np.all(oracle.bc(gg.complete(17)) == 0.0)


@pytest.mark.parametrize("a,b", [(1, 5), (3, 4), (5, 7)])
def test_bc_complete_bipartite(a, b):
    bc = oracle.bc(gg.complete_bipartite(a, b))
    np.testing.assert_allclose(bc[:a], b * (b - 1) / a, rtol=1e-14)
    np.testing.assert_allclose(bc[a:], a * (a - 1) / b, rtol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9, 10, 31, 32])
def test_bc_cycle(n):
    r = n // 2
    want = r * (r - 1) if n % 2 else (r - 1) ** 2
    np.testing.assert_allclose(oracle.bc(gg.cycle(n)), float(want), rtol=1e-13)


def test_bc_tree_formula():
    t = gg.random_tree(64, 17)
    bc = oracle.bc(t)
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    for v in range(t.n):
        keep = np.ones(t.n, bool)
        keep[v] = False
        rows = np.repeat(np.arange(t.n), np.diff(t.row_ptr))
        e = keep[rows] & keep[t.col]
        m = csr_matrix((np.ones(int(e.sum())), (rows[e], t.col[e])), shape=(t.n, t.n))
        _, lab = connected_components(m, directed=False)
        sizes = np.bincount(lab[keep])
        assert bc[v] == (t.n - 1) ** 2 - int((sizes.astype(np.int64) ** 2).sum())


@pytest.mark.parametrize("g", [gg.er_plus_tree(200, 5.0, 1), gg.rmat(10, 8, 3), gg.watts_strogatz(150, 6, 0.1, 2)],
                         ids=["er200", "rmat10", "ws150"])
def test_bc_total_equals_sum_of_distances_minus_one(g):
    """Sum_v BC(v) = sum over ordered reachable pairs s != t of (d(s,t) - 1)."""
    bc = oracle.bc(g)
    tot = 0
    for s in range(g.n):
        d = oracle.sssp(g, s)[0]
        r = (d > 0)
        tot += int((d[r] - 1).sum())
    assert bc.sum() == pytest.approx(float(tot), rel=1e-12)


def test_bc_relabel_invariance():
    g = gg.er_plus_tree(150, 5.0, 7)
    perm = gg.Stream(99).permutation(g.n)
    h = g.relabel(perm)
    np.testing.assert_allclose(oracle.bc(h)[perm], oracle.bc(g), rtol=1e-12, atol=1e-12)


def test_bc_disconnected_union_is_per_component():
    parts = [gg.path(7), gg.cycle(8), gg.star(6), gg.complete(4)]
    u = gg.disjoint_union(*parts)
    np.testing.assert_allclose(oracle.bc(u), np.concatenate([oracle.bc(p) for p in parts]), rtol=1e-14)


def test_bc_source_subset_is_partial_sum():
    g = gg.er_plus_tree(100, 4.0, 4)
    a, b = np.arange(0, 40), np.arange(40, 100)
    np.testing.assert_allclose(oracle.bc(g, a) + oracle.bc(g, b), oracle.bc(g), rtol=1e-12)
    # a source listed twice counts twice
    np.testing.assert_allclose(oracle.bc(g, [5, 5]), 2 * oracle.bc(g, [5]), rtol=0)


def test_threads_do_not_change_the_sum():
    g = gg.rmat(10, 8, 6)
    np.testing.assert_allclose(oracle.bc(g, threads=4), oracle.bc(g, threads=1), rtol=1e-13)


# -------------------------------------------------------------- weighted BC

def test_weighted_constant_weight_equals_unweighted():
    g = gg.er_plus_tree(90, 4.0, 12)
    base = oracle.bc(g)
    for c in (1, 3, 255):
        np.testing.assert_allclose(oracle.bc(gg.with_constant_weight(g, c)), base, rtol=1e-13)


def test_weighted_scaling_invariance():
    g = gg.with_uniform_weights(gg.er_plus_tree(90, 4.0, 13), 13, 1, 9)
    h = gg.from_edges(g.n, *g.edges()[:2], g.edges()[2] * 7)
    np.testing.assert_allclose(oracle.bc(h), oracle.bc(g), rtol=1e-13)


@pytest.mark.parametrize("k", [2, 3, 4, 6])
def test_weighted_tripartite_construction(k):
    """Undirected form of the Sec. 2 construction: BC(v_0) = 2k^2 + 2k(k-1)."""
    g = gg.kkp_undirected(k)
    bc = oracle.bc(g)
    assert bc[k] == pytest.approx(2 * k * k + 2 * k * (k - 1), rel=1e-13)
