"""GPU tests of the end of a search: a batch whose sources have reached every
vertex of their connected components has an empty next level, so the
algebraic form skips the products that would find that out, and the weighted
sweep stops at the phase that settles the last vertex of the source's
component.

The skipped work is observable: the forward products' k-tile counter of a
batch on a path graph counts one product per level but the last two (the
last level is found by the products from the one before it, and the products
from the last level are skipped).  Results must not change: distances and
counts bit-exact, dependencies and BC within the usual tolerances, also with
sources in components of different sizes, isolated sources and ragged
batches.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import oracle_threads

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def dense_ktiles_per_plane(n, batch):
    npad = max(256, (n + 255) // 256 * 256)
    return (npad // 32) * (npad // 128) * (batch // 128)


@pytest.mark.parametrize("host_driven", [1, 0])
def test_path_forward_skips_the_last_products(gpu_lib, host_driven):
    """One source at the end of a 40-vertex path: levels 0 .. 39, products
    for levels 1 -> 2 .. 38 -> 39 only (38 one-limb planes)."""
    g = gg.path(40)
    say("path40", host_driven)
    with gpu_lib.BC(g, form="algebraic", batch=256, vertex_order="input", host_driven=host_driven) as ctx:
        ctx.reset()
        ctx.run(np.array([0], np.int32))
        info = ctx.info()
        got = ctx.read()
    assert info.mfma_ktiles_dense_fwd == 38 * dense_ktiles_per_plane(g.n, 256)
    assert rel_err(got, oracle.bc(g, np.array([0], np.int32))) <= TOL


def test_small_component_runs_no_forward_product(gpu_lib):
    """Sources in a complete graph of 20 vertices beside a long path: level 1
    holds the whole component, so no forward product runs at all."""
    g = gg.disjoint_union(gg.path(60), gg.complete(20))
    src = np.arange(60, 80, dtype=np.int32)
    say("k20 beside path60")
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        dist, sigma, delta = ctx.sssp(src)
        ctx.reset()
        ctx.run(src)
        info = ctx.info()
        got = ctx.read()
    assert info.mfma_ktiles_dense_fwd == 0
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {s}"
        assert rel_err(delta[i], dl) <= TOL
    assert rel_err(got, oracle.bc(g, src)) <= TOL


def mixed_graph():
    """Components of different sizes and depths, and an isolated vertex."""
    return gg.disjoint_union(gg.er_plus_tree(700, 6.0, 21), gg.path(90), gg.star(30), gg.grid(9, 11),
                             gg.complete(1), gg.cycle(17))


@pytest.mark.parametrize("form,batch", [("algebraic", 256), ("algebraic", 512), ("hybrid", 256), ("sparse", 128)])
def test_mixed_components_bit_exact(gpu_lib, form, batch):
    """Sources spread over every component (the isolated vertex included, some
    repeated), a ragged last batch, replayed and host-driven runs."""
    g = mixed_graph()
    rng = gg.Stream(22)
    src = np.concatenate([np.arange(0, g.n, 7), rng.bounded(np.full(150, g.n)), [g.n - 18, g.n - 18]]).astype(np.int32)
    want = oracle.bc(g, src, threads=oracle_threads())
    say("mixed", form, batch, src.size)
    for hd in (0, 1):
        with gpu_lib.BC(g, form=form, batch=batch, host_driven=hd) as ctx:
            ctx.run(src)
            got = ctx.read()
            dist, sigma, delta = ctx.sssp(src[:min(batch, src.size)])
        assert rel_err(got, want) <= TOL, (form, hd)
        for i in range(0, min(batch, src.size), 5):
            d, sg, dl = oracle.sssp_u64(g, int(src[i]))
            assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {src[i]}"
            assert rel_err(delta[i], dl) <= TOL


def test_weighted_mixed_components(gpu_lib):
    """The weighted sweep (plain form) and the weighted algebraic form on
    components of different sizes with weights 1..8: results as the oracle's
    (the sweep stops once the source's component is settled)."""
    base = mixed_graph()
    g = gg.with_uniform_weights(base, 23, 1, 8)
    src = np.concatenate([np.arange(0, g.n, 9), [g.n - 18]]).astype(np.int32)
    want = oracle.bc(g, src, threads=oracle_threads())
    for form in ("plain", "algebraic"):
        say("weighted mixed", form)
        with gpu_lib.BC(g, form=form, batch=256 if form == "algebraic" else 0) as ctx:
            ctx.run(src)
            got = ctx.read()
            dist, sigma, delta = ctx.sssp(src[:64])
        assert rel_err(got, want) <= (1e-12 if form == "plain" else TOL), form
        for i in range(0, 64, 4):
            d, sg, dl = oracle.sssp_u64(g, int(src[i]))
            assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"{form} source {src[i]}"
            assert rel_err(delta[i], dl) <= (1e-12 if form == "plain" else TOL)
