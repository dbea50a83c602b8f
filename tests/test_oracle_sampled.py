"""Pins of the oracle's Algorithm 1 (Sec. 4.1.1, distances): the cases where
it must reduce to exact BFS distances, the upper-bound property that holds
for any sample, the hitting condition of its correctness argument, and
exactness with high probability at the sizes the section prescribes (checked
for fixed seeds)."""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import sampled


def exact(g, sources):
    return np.stack([oracle.sssp(g, int(s))[0] for s in sources])


@pytest.mark.parametrize("name", ["grid", "er", "union", "tree"])
def test_every_vertex_distinguished_is_exact(name):
    """S = V with k = 1: H is the graph itself, so its all-pairs closure alone
    gives the exact distances."""
    g = {"grid": lambda: gg.grid(6, 7), "er": lambda: gg.er_plus_tree(60, 3.0, 2),
         "union": lambda: gg.disjoint_union(gg.path(8), gg.cycle(9)), "tree": lambda: gg.random_tree(50, 4)}[name]()
    src = np.arange(0, g.n, 5)
    got = sampled.sampled_distances(g, src, np.arange(g.n), k=1)
    assert np.array_equal(got, exact(g, src))


def test_limit_past_the_diameter_is_exact():
    """With k at least the diameter, x = s alone gives every distance."""
    g = gg.er_plus_tree(80, 3.0, 5)
    src = np.array([0, 7, 41, 79])
    got = sampled.sampled_distances(g, src, gg.sample_sources(g.n, 3, 9), k=g.n)
    assert np.array_equal(got, exact(g, src))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_never_below_the_true_distance(seed):
    """Every value is a real walk: at least the distance, and -1 only where
    the walk search found nothing (always for unreachable targets)."""
    g = gg.disjoint_union(gg.er_plus_tree(70, 2.5, seed), gg.path(12))
    src = gg.sample_sources(g.n, 6, seed)
    got = sampled.sampled_distances(g, src, gg.sample_sources(g.n, 5, seed + 10), k=2)
    want = exact(g, src)
    assert np.all(got[want < 0] == -1)
    found = got >= 0
    assert np.all(got[found] >= want[found])


def test_hitting_condition():
    """On a path, a distinguished vertex every k hops makes every distance
    exact; a source alone finds nothing beyond k hops."""
    g = gg.path(21)
    got = sampled.sampled_distances(g, [0], np.arange(0, 21, 3), k=3)
    assert np.array_equal(got[0], np.arange(21))
    alone = sampled.sampled_distances(g, [0], [], k=3)[0]
    assert np.array_equal(alone[:4], np.arange(4)) and np.all(alone[4:] == -1)


@pytest.mark.parametrize("graph", ["grid40", "path2000", "ws1500"])
def test_exact_with_high_probability(graph):
    """k = ceil(sqrt(n)) and |S| = ceil(sqrt(n) ln n), as Sec. 4.1.1 sets
    them, on graphs whose diameter exceeds k (so the source's own limited
    search cannot reach every vertex): exact for these seeds."""
    g = {"grid40": lambda: gg.grid(40, 40), "path2000": lambda: gg.path(2000),
         "ws1500": lambda: gg.watts_strogatz(1500, 4, 0.01, 3)}[graph]()
    k = math.ceil(math.sqrt(g.n))
    size = math.ceil(math.sqrt(g.n) * math.log(g.n))
    src = gg.sample_sources(g.n, 8, 33)
    want = exact(g, src)
    assert want.max() > k
    alone = sampled.sampled_distances(g, src, [], k=k)
    assert not np.array_equal(alone, want)
    got = sampled.sampled_distances(g, src, gg.sample_sources(g.n, size, 34), k=k)
    assert np.array_equal(got, want)


def test_weighted_graphs_refused():
    with pytest.raises(ValueError):
        sampled.sampled_distances(gg.with_constant_weight(gg.path(5), 2), [0], [], k=2)
