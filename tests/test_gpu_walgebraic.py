"""GPU parity of the algebraic form on integer weights 1..M (Sec. 3.2):
per-weight-class products with levels taken as distances.

Distances and path counts must equal the oracle's bit for bit; dependencies
and BC stay within the FP32-state tolerance of the batched forms.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def graphs():
    return {
        "gnp40w8": gg.random_graph(40, 0.15, 5, weights=8),
        "er500w8": gg.with_uniform_weights(gg.er_plus_tree(500, 6.0, 8), 8, 1, 8),
        "grid15x17w3": gg.with_constant_weight(gg.grid(15, 17), 3),
        "path40w5": gg.with_constant_weight(gg.path(40), 5),
        "unionw": gg.disjoint_union(gg.with_uniform_weights(gg.path(30), 2, 1, 4),
                                    gg.random_graph(50, 0.1, 9, weights=7)),
        "rmat11w8": gg.with_uniform_weights(gg.rmat(11, 16, 4), 4, 1, 8),
        "er1024w2": gg.with_uniform_weights(gg.er1024(), 6, 1, 2),
        "ws300w1": gg.with_constant_weight(gg.watts_strogatz(300, 6, 0.1, 7), 1),
        "star50w7": gg.with_constant_weight(gg.star(50), 7),
        "k65w": gg.with_uniform_weights(gg.complete(65), 3, 1, 8),
    }


@pytest.mark.parametrize("batch", [256, 512])
@pytest.mark.parametrize("name", sorted(graphs()))
def test_weighted_algebraic_bc(gpu_lib, name, batch):
    g = graphs()[name]
    say("walg_bc", name, g.n, g.m, batch)
    with gpu_lib.BC(g, form="algebraic", batch=batch) as ctx:
        info = ctx.info()
        assert info.form == gpu_lib.BC_FORM_ALGEBRAIC and info.weighted == 1
        ctx.run()
        got = ctx.read()
        assert ctx.info().mfma_planes > 0
    assert rel_err(got, oracle.bc(g)) <= TOL


@pytest.mark.parametrize("name", ["gnp40w8", "er500w8", "path40w5", "unionw", "rmat11w8", "k65w"])
def test_weighted_algebraic_sssp_bit_exact(gpu_lib, name):
    g = graphs()[name]
    say("walg_sssp", name, g.n)
    rng = gg.Stream(41)
    src = np.concatenate([np.arange(min(4, g.n)), rng.bounded(np.full(60, g.n))]).astype(np.int32)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        dist, sigma, delta = ctx.sssp(src)
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d), f"dist source {s}"
        assert np.array_equal(sigma[i], sg), f"sigma source {s}"
        assert rel_err(delta[i], dl) <= TOL, f"delta source {s}"


def test_weighted_algebraic_multiset_and_accumulate(gpu_lib):
    g = gg.with_uniform_weights(gg.er_plus_tree(700, 5.0, 31), 31, 1, 6)
    src = np.concatenate([gg.Stream(3).bounded(np.full(300, g.n)), np.arange(10), np.arange(10)]).astype(np.int32)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        ctx.run(src[:150])
        ctx.run(src[150:])
        got = ctx.read()
    assert rel_err(got, oracle.bc(g, src)) <= TOL


def test_weighted_algebraic_wide_counts(gpu_lib):
    """Grid 20 x 20 with every weight 2: counts above 2^32 in several limbs,
    levels every other distance."""
    g = gg.with_constant_weight(gg.grid(20, 20), 2)
    src = np.array([0, 19, 380, 399, 210], np.int32)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        dist, sigma, _ = ctx.sssp(src)
        ctx.run()
        got = ctx.read()
    for i, s in enumerate(src):
        d, sg, _ = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
    assert sigma.max() > 2 ** 32
    assert rel_err(got, oracle.bc(g)) <= TOL


def test_weighted_algebraic_overflow_reported(gpu_lib):
    g = gg.with_constant_weight(gg.grid(35, 35), 2)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        ctx.run()
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.read()
        assert e.value.status == gpu_lib.BC_ERR_OVERFLOW


def test_weighted_algebraic_all_pairs(gpu_lib):
    """Algorithm 2 over distances and counts from the weighted products."""
    g = gg.with_uniform_weights(gg.er_plus_tree(400, 6.0, 17), 17, 1, 8)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        got = ctx.all_pairs()
    assert rel_err(got, oracle.bc(g)) <= 1e-12


def test_weighted_algebraic_matches_plain_form(gpu_lib):
    """Both weighted forms on one graph: the bucketed per-source sweep (FP64)
    and the per-class products agree to the FP32-state tolerance."""
    g = gg.with_uniform_weights(gg.rmat(12, 16, 19), 19, 1, 8)
    src = gg.Stream(8).bounded(np.full(512, g.n)).astype(np.int32)
    with gpu_lib.BC(g, form="plain") as p, gpu_lib.BC(g, form="algebraic", batch=512) as a:
        p.run(src)
        a.run(src)
        want, got = p.read(), a.read()
    assert rel_err(got, want) <= TOL
    assert rel_err(want, oracle.bc(g, src, threads=8)) <= 1e-12
