"""Replayed batches: bc_run records one source batch's launches into a HIP
graph and replays it per batch; the level-synchronous search of Sec. 4 is
kept, one launch per level, levels past a batch's depth exiting at once.  A
batch that goes deeper than the recorded levels, or whose path counts need
64-bit storage, is handed back and re-run host-driven when the context is
next used.  Whatever the path, BC must equal the oracle's (Sec. 1.1) within
the FP32-state tolerance, and equal the host-driven path's."""
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
    return {"er1024": gg.er1024(), "grid20": gg.grid(20, 20), "ws600": gg.watts_strogatz(600, 6, 0.1, 9),
            "union": gg.disjoint_union(gg.star(300), gg.path(300), gg.er_plus_tree(400, 5.0, 4))}


@pytest.mark.parametrize("form", ["sparse", "hybrid", "algebraic"])
@pytest.mark.parametrize("name", ["er1024", "grid20", "ws600", "union"])
def test_replay_equals_oracle_and_host_driven(gpu_lib, form, name):
    g = graphs()[name]
    batch = 64 if form == "sparse" else 256
    say("replay", form, name, batch)
    want = oracle.bc(g)
    with gpu_lib.BC(g, form=form, batch=batch) as ctx:
        ctx.run()
        got = ctx.read()
        assert ctx.info().sources_run == g.n
    with gpu_lib.BC(g, form=form, batch=batch, host_driven=True) as ctx:
        ctx.run()
        host = ctx.read()
    assert rel_err(got, want) <= TOL
    assert rel_err(host, want) <= TOL
    assert rel_err(got, host) <= TOL


@pytest.mark.parametrize("form", ["sparse", "hybrid"])
def test_deeper_batches_handed_back(gpu_lib, form):
    """The first batch (run host-driven) comes from a star, 3 levels deep;
    the later batches from a 500-vertex path go far deeper than the recorded
    levels, so every replay hands its batch back; the host re-runs them and
    the next run records the new depth."""
    g = gg.disjoint_union(gg.star(200), gg.path(500))
    src = np.concatenate([np.arange(0, 64), np.arange(200, 700)]).astype(np.int32)
    want = oracle.bc(g, src)
    with gpu_lib.BC(g, form=form, batch=64 if form == "sparse" else 256) as ctx:
        ctx.run(src)
        got = ctx.read()
        assert ctx.info().max_levels >= 300
        ctx.reset()
        ctx.run(src)  # recorded again with the deeper level count
        again = ctx.read()
    assert rel_err(got, want) <= TOL
    assert rel_err(again, want) <= TOL


def test_wide_counts_handed_back(gpu_lib):
    """Grid 20 x 20 beside a 100-vertex path.  The first batch (host-driven)
    takes 63 sources from the grid's central 10 x 10 block, whose counts stay
    below C(28, 14) < 2^32, and one end of the path, which makes the recorded
    depth 100, past any grid distance.  The other grid vertices, corners
    included, have counts up to C(38, 19) > 2^32: the replays that meet them
    hand their batches back for 64-bit counts alone."""
    g = gg.disjoint_union(gg.grid(20, 20), gg.path(100))
    centre = [x * 20 + y for x in range(5, 15) for y in range(5, 15)][:63]
    rest = [v for v in range(400) if v not in set(centre)]
    src = np.array(centre + [400] + rest, np.int32)
    want = oracle.bc(g, src)
    with gpu_lib.BC(g, form="sparse", batch=64) as ctx:
        ctx.run(src)
        got = ctx.read()
        d, sigma, _ = ctx.sssp(np.array([0], np.int32))
    assert rel_err(got, want) <= TOL
    assert int(sigma[0][399]) == 35345263800


@pytest.mark.parametrize("timing", [1, 3])
def test_replay_with_timing(gpu_lib, timing):
    """With timing on, the timed batches (one in k) run host-driven with
    events around every launch and the others replay; the timers scale the
    host-driven batches' totals to all batches.  Results are unchanged."""
    g = gg.er1024()
    with gpu_lib.BC(g, form="sparse", batch=64, timing=timing) as ctx:
        ctx.run()
        ctx.run()
        got = ctx.read()
        ms, launches = ctx.timing("bwd_pull")
        fms, flaunches = ctx.timing("fwd_pull")
    assert rel_err(got, 2.0 * oracle.bc(g)) <= TOL
    assert launches >= 2 * 15 and flaunches >= 2 * 15
    assert ms > 0.0 and fms > 0.0


def test_runs_reads_and_dumps_interleaved(gpu_lib):
    """Several runs before a read, a per-source dump and a reset between runs:
    each call settles the replays of the run before it."""
    g = gg.er_plus_tree(900, 6.0, 2106)
    a = np.arange(0, 900, 2, dtype=np.int32)
    b = np.arange(1, 900, 2, dtype=np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256) as ctx:
        ctx.run(a)
        ctx.run(b)
        d, sg, _ = ctx.sssp(np.array([5, 6], np.int32))
        ctx.run(a)
        got = ctx.read()
        ctx.run(b)
        ctx.reset()
        ctx.run(b)
        only_b = ctx.read()
    assert rel_err(got, oracle.bc(g, np.concatenate([a, b, a]))) <= TOL
    assert rel_err(only_b, oracle.bc(g, b)) <= TOL
    for i, s in enumerate([5, 6]):
        od, osg, _ = oracle.sssp_u64(g, s)
        assert np.array_equal(d[i], od) and np.array_equal(sg[i], osg)


@pytest.mark.parametrize("form", ["sparse", "hybrid"])
def test_replay_edges(gpu_lib, form):
    """Edge betweenness through replayed batches (level 0 runs too)."""
    g = gg.er1024()
    want_bc, want_eb = oracle.edge_bc(g)
    with gpu_lib.BC(g, form=form, batch=64 if form == "sparse" else 256, edges=True) as ctx:
        ctx.run()
        assert rel_err(ctx.read(), want_bc) <= TOL
        assert rel_err(ctx.read_edges(), want_eb) <= TOL
