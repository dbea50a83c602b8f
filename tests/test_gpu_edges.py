"""Edge betweenness on the GPU (contexts created with edges=True) against the
oracle's per-arc values: each DAG arc's Theorem 1.1 term summed over sources
and over both directions of its edge.  Same error metric and tolerances as
BC: 1e-12 for the plain FP64 form, 1e-5 where c(v) is stored in FP32."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-12, "sparse": 1e-5, "hybrid": 1e-5}


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def graphs():
    return {"path33": gg.path(33), "star50": gg.star(50), "cycle31": gg.cycle(31), "complete40": gg.complete(40),
            "grid20": gg.grid(20, 20), "er1024": gg.er1024(), "ws300": gg.watts_strogatz(300, 6, 0.1, 7),
            "union": gg.disjoint_union(gg.path(40), gg.er_plus_tree(200, 5.0, 3), gg.star(7)), "path1": gg.path(1)}


@pytest.mark.parametrize("form", ["plain", "sparse", "hybrid"])
@pytest.mark.parametrize("name", ["path33", "star50", "cycle31", "complete40", "grid20", "er1024", "ws300", "union",
                                  "path1"])
def test_edges_all_sources(gpu_lib, form, name):
    g = graphs()[name]
    say("edges", form, name)
    want_bc, want_eb = oracle.edge_bc(g)
    with gpu_lib.BC(g, form=form, edges=True) as ctx:
        ctx.run()
        got_bc, got_eb = ctx.read(), ctx.read_edges()
    assert rel_err(got_bc, want_bc) <= TOL[form]
    assert rel_err(got_eb, want_eb) <= TOL[form]


@pytest.mark.parametrize("form", ["plain", "sparse"])
@pytest.mark.parametrize("order", ["degree", "input"])
def test_edges_sampled_multiset_and_reset(gpu_lib, form, order):
    """A multiset of sources over a ragged batch, in either internal
    numbering; reset clears the edge sums."""
    g = gg.er_plus_tree(700, 6.0, 17)
    src = np.concatenate([np.arange(0, 700, 3), [5, 5, 9]]).astype(np.int32)
    _, want = oracle.edge_bc(g, src)
    with gpu_lib.BC(g, form=form, edges=True, vertex_order=order) as ctx:
        ctx.run(src[:100])
        ctx.run(src[100:])
        assert rel_err(ctx.read_edges(), want) <= TOL[form]
        ctx.reset()
        assert not np.any(ctx.read_edges())
        ctx.run(src)
        assert rel_err(ctx.read_edges(), want) <= TOL[form]


@pytest.mark.parametrize("log2", [0, 6])
def test_edges_weighted(gpu_lib, log2):
    """Weighted graphs: the DAG arcs recorded by the forward carry the terms;
    a tiny ring (log2 = 6) sends sources through the full-size re-run."""
    g = gg.with_uniform_weights(gg.er_plus_tree(600, 6.0, 23), 23, 1, 9)
    src = np.arange(0, g.n, 2, dtype=np.int32)
    want_bc, want_eb = oracle.edge_bc(g, src)
    with gpu_lib.BC(g, edges=True, arena_log2=log2) as ctx:
        ctx.run(src)
        assert rel_err(ctx.read(), want_bc) <= 1e-12
        assert rel_err(ctx.read_edges(), want_eb) <= 1e-12


def test_edges_hybrid_forward_products(gpu_lib, tmp_path):
    """The hybrid form with forward levels by products still gives exact edge
    terms (the backward runs by pulls when edges are on)."""
    g = gg.er1024()
    path = str(tmp_path / "tune.txt")
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path):
        pass
    key = [ln for ln in open(path).read().splitlines() if ln][-1].split("\t")[0]
    with open(path, "a") as f:
        f.write(f"{key}\t256 0.0 0.0\n")
    _, want = oracle.edge_bc(g)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path, edges=True) as ctx:
        ctx.run()
        got = ctx.read_edges()
        assert ctx.info().mfma_planes > 0
    assert rel_err(got, want) <= 1e-5


def test_edges_rmat16_sampled(gpu_lib):
    g = gg.rmat16()
    say("edges rmat16", g.n, g.m)
    src = gg.Stream(41).bounded(np.full(300, g.n)).astype(np.int32)
    _, want = oracle.edge_bc(g, src, threads=8)
    with gpu_lib.BC(g, form="sparse", batch=256, edges=True) as ctx:
        ctx.run(src)
        got = ctx.read_edges()
    assert rel_err(got, want) <= 1e-5


def test_read_edges_needs_edges(gpu_lib):
    with gpu_lib.BC(gg.path(5), form="sparse") as ctx:
        ctx.run()
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.read_edges()
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED


@pytest.mark.parametrize("form", ["sparse", "hybrid"])
def test_edges_after_tuning(gpu_lib, form):
    """A context that tunes its batch width (batch 0, n >= 2048, no cache
    entry) runs calibration batches before any caller work; their per-arc
    terms must not stay in the edge sums, as their dependencies do not stay
    in BC."""
    g = gg.er_plus_tree(3000, 6.0, 2101)
    say("edges after tuning", form, g.n, g.m)
    want_bc, want_eb = oracle.edge_bc(g, threads=16)
    with gpu_lib.BC(g, form=form, batch=0, edges=True) as ctx:
        assert ctx.info().tune_source == 1, "the context should have measured its batch width"
        assert not np.any(ctx.read_edges()), "edge sums after create must be zero"
        ctx.run()
        got_bc, got_eb = ctx.read(), ctx.read_edges()
    assert rel_err(got_bc, want_bc) <= TOL[form]
    assert rel_err(got_eb, want_eb) <= TOL[form]
