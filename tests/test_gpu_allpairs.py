"""GPU parity of Algorithm 2 (Sec. 4.2.1): BC over every ordered pair from the
all-pairs distance matrix D and path-count matrix Lambda, summed on the
device as lambda_sv * lambda_vt / lambda_st over the pairs with
d(s,t) = d(s,v) + d(v,t).

Each form's own forward kernels fill D and Lambda; the triple sum is FP64
whatever the form, so every case is held to the FP64 tolerance against the
oracle's all-source Brandes BC, and small graphs also against the oracle's
own Algorithm 2 on Floyd-Warshall counts.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import cross

pytestmark = pytest.mark.gpu

TOL = 1e-12
FORMS = ["plain", "sparse", "algebraic", "hybrid"]


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def unweighted():
    return [gg.path(1), gg.path(2), gg.from_edges(5, [], [], name="isolated5"), gg.path(33), gg.star(50),
            gg.cycle(31), gg.complete(64), gg.complete(65), gg.complete_bipartite(5, 7), gg.random_tree(100, 3),
            gg.disjoint_union(gg.path(7), gg.cycle(8), gg.star(6), gg.complete(4)), gg.grid(20, 20),
            gg.er1024(), gg.watts_strogatz(300, 6, 0.1, 7)]


@pytest.mark.parametrize("gi", range(len(unweighted())))
@pytest.mark.parametrize("form", FORMS)
def test_all_pairs_equals_brandes(gpu_lib, form, gi):
    g = unweighted()[gi]
    say("all_pairs", form, g.name, g.n, g.m)
    want = oracle.bc(g)
    with gpu_lib.BC(g, form=form) as ctx:
        got = ctx.all_pairs()
        # the running BC is not touched
        assert np.array_equal(ctx.read(), np.zeros(g.n))
        assert ctx.info().sources_run == 0
    assert got.shape == (g.n,)
    assert rel_err(got, want) <= TOL


@pytest.mark.parametrize("name", ["grid7x9", "union", "ws60", "kab"])
def test_all_pairs_equals_cross_oracle(gpu_lib, name):
    g = {"grid7x9": lambda: gg.grid(7, 9), "union": lambda: gg.disjoint_union(gg.path(9), gg.cycle(12)),
         "ws60": lambda: gg.watts_strogatz(60, 4, 0.2, 3), "kab": lambda: gg.complete_bipartite(4, 9)}[name]()
    say("all_pairs_cross", name)
    D, L = cross.allpairs_counts(g)
    want = cross.algorithm2(D, L)
    with gpu_lib.BC(g, form="sparse") as ctx:
        assert rel_err(ctx.all_pairs(), want) <= TOL


def weighted():
    return [gg.random_graph(40, 0.15, 5, weights=9), gg.kkp_undirected(6),
            gg.with_uniform_weights(gg.er_plus_tree(500, 6.0, 8), 8, 1, 255),
            gg.with_constant_weight(gg.grid(15, 17), 3),
            gg.disjoint_union(gg.with_uniform_weights(gg.path(30), 2, 1, 4), gg.random_graph(50, 0.1, 9, weights=7))]


@pytest.mark.parametrize("gi", range(len(weighted())))
def test_all_pairs_weighted(gpu_lib, gi):
    """Weighted graphs: D from the bucketed sweeps; the mask uses the
    weighted distances (Sec. 1.1 defines BC for weighted graphs alike)."""
    g = weighted()[gi]
    say("all_pairs_weighted", g.name, g.n, g.m)
    with gpu_lib.BC(g) as ctx:
        got = ctx.all_pairs()
    assert rel_err(got, oracle.bc(g)) <= TOL


def test_all_pairs_heaviest_weights(gpu_lib):
    """Every edge at the largest weight the weighted sweep takes (255), on a
    path and a grid: long distances, counts of 1 and of binomials."""
    for g in (gg.with_constant_weight(gg.path(300), 255), gg.with_constant_weight(gg.grid(12, 13), 255)):
        say("all_pairs_w255", g.name, g.n)
        with gpu_lib.BC(g) as ctx:
            got = ctx.all_pairs()
        assert rel_err(got, oracle.bc(g)) <= TOL


def test_all_pairs_ragged_mid_size(gpu_lib):
    """n = 3001: a ragged tail in both the vertex tiles (64) and the source
    chunks (256), in every form."""
    g = gg.er_plus_tree(3001, 10.0, 41, name="er3001")
    want = oracle.bc(g, threads=8)
    for form in FORMS:
        say("all_pairs_mid", form, g.n, g.m)
        with gpu_lib.BC(g, form=form) as ctx:
            assert rel_err(ctx.all_pairs(), want) <= TOL


def test_all_pairs_leaves_running_bc(gpu_lib):
    g = gg.er_plus_tree(700, 5.0, 31)
    sub = gg.Stream(9).bounded(np.full(100, g.n)).astype(np.int32)
    with gpu_lib.BC(g, form="hybrid") as ctx:
        ctx.run(sub)
        got = ctx.all_pairs()
        part = ctx.read()
        assert ctx.info().sources_run == sub.size
    assert rel_err(got, oracle.bc(g)) <= TOL
    assert rel_err(part, oracle.bc(g, sub)) <= 1e-5


@pytest.mark.parametrize("form", ["plain", "sparse"])
def test_all_pairs_overflow_reported_and_state_kept(gpu_lib, form):
    """Grid 35 x 35: corner-to-corner counts C(68, 34) exceed 2^64 - 1.  The
    call reports it and leaves the running BC's overflow state as it was."""
    g = gg.grid(35, 35)
    center = np.array([17 * 35 + 17], np.int32)
    with gpu_lib.BC(g, form=form) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.all_pairs()
        assert e.value.status == gpu_lib.BC_ERR_OVERFLOW
        ctx.run(center)
        got = ctx.read()
    assert rel_err(got, oracle.bc(g, center)) <= (TOL if form == "plain" else 1e-5)


def test_all_pairs_limits(gpu_lib):
    with gpu_lib.BC(gg.from_edges(0, [], []), form="sparse") as ctx:
        assert ctx.all_pairs().shape == (0,)
    g = gg.path(gpu_lib.BC_ALL_PAIRS_MAX_N + 1)
    with gpu_lib.BC(g, form="sparse", batch=64) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.all_pairs()
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED
    with gpu_lib.BC([gg.path(5), gg.path(6)]) as ctx:
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.all_pairs()
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED


def test_er16384_all_pairs_full_size(gpu_lib, oracle_all_sources):
    """The all-pairs workload at its full size (ER, n = 16384, mean degree
    256), with the algebraic form filling D and Lambda as the benchmark does,
    against the oracle's all-source BC."""
    g = gg.er16384()
    say("er16384_all_pairs", g.n, g.m)
    with gpu_lib.BC(g, form="algebraic", batch=512) as ctx:
        got = ctx.all_pairs()
    want = oracle_all_sources("er16384", g)
    assert rel_err(got, want) <= TOL
