"""GPU parity of Algorithm 1 (Sec. 4.1.1, the sampled forward, distances).

Every value must equal the oracle's bit for bit on the same sources, sample
and search limit. At the sizes the section prescribes, the result must equal
the exact distances for these seeds.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import sampled

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def exact(g, sources):
    return np.stack([oracle.sssp(g, int(s))[0] for s in sources])


def cases():
    return {
        # name: (graph, sources, sample, k)
        "grid_all_k1": (gg.grid(6, 7), np.arange(0, 42, 5), np.arange(42), 1),
        "er60_k2": (gg.er_plus_tree(60, 3.0, 2), np.array([0, 9, 33]), gg.sample_sources(60, 7, 4), 2),
        "union_unreachable": (gg.disjoint_union(gg.er_plus_tree(70, 2.5, 1), gg.path(12)),
                              gg.sample_sources(82, 6, 1), gg.sample_sources(82, 5, 11), 2),
        "path_every3": (gg.path(21), np.array([0]), np.arange(0, 21, 3), 3),
        "path_alone": (gg.path(21), np.array([0, 20]), np.array([], np.int64), 3),
        "tree50": (gg.random_tree(50, 4), np.array([3, 3, 17]), np.array([17, 5, 40]), 2),
        # three words of limited searches, the last ragged; repeats in both lists
        "er700_words": (gg.er_plus_tree(700, 3.0, 6), np.array([5, 5, 600, 699, 0]),
                        gg.sample_sources(700, 150, 7), 3),
        # n with a ragged last block; k past the diameter
        "ws1000_deep": (gg.watts_strogatz(1000, 4, 0.05, 9), np.array([1, 999]), gg.sample_sources(1000, 40, 5), 60),
        # H is a chain of 600 vertices over ten pivot blocks: distances of up to 600 hops in H
        "path1200_chain": (gg.path(1200), np.array([0, 1199, 601]), np.arange(0, 1200, 2), 2),
        "rmat10": (gg.rmat(10, 8, 3), gg.sample_sources(gg.rmat(10, 8, 3).n, 9, 2),
                   gg.sample_sources(gg.rmat(10, 8, 3).n, 70, 3), 2),
    }


@pytest.mark.parametrize("name", sorted(cases()))
def test_sampled_matches_oracle(gpu_lib, name):
    g, src, smp, k = cases()[name]
    say("sampled", name, g.n, len(src), len(smp), k)
    want = sampled.sampled_distances(g, src, smp, k=k)
    with gpu_lib.BC(g) as ctx:
        got = ctx.sampled_distances(src, smp, limit=k)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("graph", ["grid40", "path2000", "ws1500"])
def test_sampled_exact_at_prescribed_sizes(gpu_lib, graph):
    """k = ceil(sqrt(n)) by default and |S| = ceil(sqrt(n) ln n): exact for
    these seeds, on graphs whose diameter exceeds k."""
    g = {"grid40": lambda: gg.grid(40, 40), "path2000": lambda: gg.path(2000),
         "ws1500": lambda: gg.watts_strogatz(1500, 4, 0.01, 3)}[graph]()
    size = math.ceil(math.sqrt(g.n) * math.log(g.n))
    src = gg.sample_sources(g.n, 8, 33)
    smp = gg.sample_sources(g.n, size, 34)
    say("sampled_whp", graph, g.n, size)
    with gpu_lib.BC(g) as ctx:
        got = ctx.sampled_distances(src, smp)
        alone = ctx.sampled_distances(src, [])
    want = exact(g, src)
    assert np.array_equal(got, want)
    assert np.array_equal(alone, sampled.sampled_distances(g, src, [], k=math.ceil(math.sqrt(g.n))))
    assert not np.array_equal(alone, want)


def test_sampled_rmat16_exact(gpu_lib):
    """The RMAT-16 workload, |S| = ceil(sqrt(n) ln n): k = ceil(sqrt(n)) is
    past the diameter, so every distance is exact."""
    g = gg.rmat16()
    src = gg.sample_sources(g.n, 12, 5)
    smp = gg.sample_sources(g.n, math.ceil(math.sqrt(g.n) * math.log(g.n)), 6)
    say("sampled_rmat16", g.n, len(smp))
    with gpu_lib.BC(g, form="plain") as ctx:
        got = ctx.sampled_distances(src, smp)
    assert np.array_equal(got, exact(g, src))


def test_sampled_largest_set(gpu_lib):
    """|S| at its maximum (4096, every vertex of a 4096-vertex graph) with
    k = 1: H is the graph itself, so the result is the exact distances.  One
    more distinguished vertex is refused."""
    g = gg.watts_strogatz(4096, 6, 0.05, 12)
    src = np.array([0, 1, 2048, 4095, 777], np.int32)
    say("sampled_max", g.n)
    with gpu_lib.BC(g) as ctx:
        got = ctx.sampled_distances(src, np.arange(g.n), limit=1)
    assert np.array_equal(got, exact(g, src))
    big = gg.watts_strogatz(4097, 6, 0.05, 12)
    with gpu_lib.BC(big) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.sampled_distances(src, np.arange(big.n), limit=1)
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED


def test_sampled_errors_and_empty(gpu_lib):
    g = gg.er_plus_tree(100, 3.0, 3)
    with gpu_lib.BC(g) as ctx:
        assert ctx.sampled_distances([], [1, 2]).shape == (0, g.n)
        for src, smp, k in (([100], [], 2), ([0], [-1], 2), ([0], [], 65535)):
            with pytest.raises(gpu_lib.BCError) as e:
                ctx.sampled_distances(src, smp, limit=k)
            assert e.value.status == gpu_lib.BC_ERR_INVALID_ARG
        # still usable after the refusals
        assert np.array_equal(ctx.sampled_distances([4], [], limit=200), exact(g, [4]))
    with gpu_lib.BC(gg.with_constant_weight(g, 2)) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.sampled_distances([0], [], limit=2)
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED
    with gpu_lib.BC([gg.path(10), gg.cycle(7)]) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.sampled_distances([0], [], limit=2)
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED


@pytest.mark.parametrize("repeats", [False, True])
def test_sampled_device_output(gpu_lib, repeats):
    """Rows written into a device tensor: straight from the final kernel when
    no source repeats, through a row gather when some do."""
    import torch
    g = gg.er_plus_tree(900, 4.0, 21)
    src = np.array([7, 300, 899, 7, 5] if repeats else [7, 300, 899, 5], np.int32)
    smp = gg.sample_sources(g.n, 90, 22)
    want = sampled.sampled_distances(g, src, smp, k=3)
    say("sampled_device", repeats)
    with gpu_lib.BC(g) as ctx:
        out = torch.full((src.size, g.n), -7, dtype=torch.int32, device="cuda:0")
        assert ctx.sampled_distances(src, smp, limit=3, out=out) is out
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
        with pytest.raises(ValueError):
            ctx.sampled_distances(src, smp, limit=3, out=out[:, :10])


def test_sampled_wide_values_take_32_bit_path(gpu_lib):
    """The final minimum runs in 16-bit arithmetic only while every finite
    D_H entry is at most 65534 - k.  With k = 65534 any positive entry is over
    that bound, so the 32-bit product runs; both routes give the exact
    distances here (k is past the diameter either way)."""
    g = gg.er_plus_tree(600, 3.0, 41)
    src = gg.sample_sources(g.n, 5, 42)
    smp = gg.sample_sources(g.n, 40, 43)
    want = exact(g, src)
    say("sampled_wide", g.n)
    with gpu_lib.BC(g) as ctx:
        wide = ctx.sampled_distances(src, smp, limit=65534)
        narrow = ctx.sampled_distances(src, smp, limit=64)
    assert np.array_equal(wide, want) and np.array_equal(narrow, want)
    assert np.array_equal(wide, sampled.sampled_distances(g, src, smp, k=65534))
