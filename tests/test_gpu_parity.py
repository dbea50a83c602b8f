"""GPU parity: the HIP library, called through the C ABI, against the oracle.

Distances and path counts must match bit-exactly; BC and per-source
dependencies within the form's tolerance (max |x-y| / max(|y|, 1)):
1e-12 for the plain FP64 form, 1e-5 for the batched forms whose c(v) state is
stored in FP32.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-12, "sparse": 1e-5, "algebraic": 1e-5}
FORMS = ["plain", "sparse", "algebraic"]


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def small_graphs():
    return [gg.path(1), gg.path(2), gg.path(33), gg.star(50), gg.cycle(31), gg.cycle(32), gg.complete(64),
            gg.complete_bipartite(5, 7), gg.random_tree(100, 3),
            gg.disjoint_union(gg.path(7), gg.cycle(8), gg.star(6), gg.complete(4)),
            gg.grid(20, 20), gg.er1024(), gg.watts_strogatz(300, 6, 0.1, 7)]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("gi", range(13))
def test_bc_all_sources(gpu_lib, form, gi):
    g = small_graphs()[gi]
    say("bc_all_sources", form, g.name, g.n, g.m)
    want = oracle.bc(g)
    with gpu_lib.BC(g, form=form) as ctx:
        ctx.run()
        got = ctx.read()
    assert rel_err(got, want) <= TOL[form], g.name


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name", ["er1024", "grid20", "union", "ws300"])
def test_sssp_bit_exact(gpu_lib, form, name):
    g = {"er1024": gg.er1024, "grid20": lambda: gg.grid(20, 20),
         "union": lambda: gg.disjoint_union(gg.path(40), gg.er_plus_tree(200, 5.0, 3)),
         "ws300": lambda: gg.watts_strogatz(300, 6, 0.1, 7)}[name]()
    say("sssp_bit_exact", form, name, g.n)
    rng = gg.Stream(123)
    src = np.concatenate([np.arange(8), np.arange(g.n - 8, g.n), rng.bounded(np.full(16, g.n))]).astype(np.int32)
    with gpu_lib.BC(g, form=form) as ctx:
        dist, sigma, delta = ctx.sssp(src)
        bc_after = ctx.read()
    assert np.all(bc_after == 0.0), "bc_read_sssp must not add to BC"
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        np.testing.assert_array_equal(dist[i], d, err_msg=f"dist, source {s}")
        np.testing.assert_array_equal(sigma[i], sg, err_msg=f"sigma, source {s}")
        assert rel_err(delta[i], dl) <= TOL[form], f"delta, source {s}"


@pytest.mark.parametrize("form", FORMS)
def test_sigma_above_2_24_uses_exact_counts(gpu_lib, form):
    """grid 20x20: corner-to-corner count C(38,19) > 2^24."""
    g = gg.grid(20, 20)
    say("sigma_above_2_24", form)
    with gpu_lib.BC(g, form=form) as ctx:
        _, sigma, _ = ctx.sssp(np.array([0], np.int32))
    assert int(sigma[0, g.n - 1]) == 35345263800


@pytest.mark.parametrize("form", FORMS)
def test_overflow_reported(gpu_lib, form):
    """grid 35x35: C(68,34) > 2^64 - 1 must give BC_ERR_OVERFLOW, never a wrapped count."""
    g = gg.grid(35, 35)
    say("overflow", form)
    with gpu_lib.BC(g, form=form) as ctx:
        ctx.run(np.array([0], np.int32))
        with pytest.raises(gpu_lib.BCError) as ei:
            ctx.read()
        assert ei.value.status == gpu_lib.BC_ERR_OVERFLOW
        with pytest.raises(gpu_lib.BCError):
            ctx.run(np.array([1], np.int32))
        ctx.reset()
        ctx.run(np.array([35 * 17 + 17], np.int32))  # centre: counts stay below 2^64
        assert np.isfinite(ctx.read()).all()


@pytest.mark.parametrize("form", FORMS)
def test_largest_square_grid_within_u64(gpu_lib, form):
    g = gg.grid(34, 34)
    say("grid34", form)
    with gpu_lib.BC(g, form=form) as ctx:
        _, sigma, _ = ctx.sssp(np.array([0], np.int32))
    assert int(sigma[0, g.n - 1]) == 7219428434016265740  # C(66,33)


@pytest.mark.parametrize("form", FORMS)
def test_counts_past_2_63_through_every_limb(gpu_lib, form):
    """A 34 x 35 grid reaches C(67,33), between 2^63 and 2^64 - 1, at its far
    corner, and two vertices hanging off that corner keep the count: the step
    out of the corner's level reads a largest count with bit 63 set, which
    takes every one of the ten 7-bit limbs in the algebraic form's products.
    Counts are C(x + y, x) on the grid and must come back exactly."""
    base = gg.grid(34, 35)
    rows = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    keep = rows < base.col
    far = base.n - 1
    u = np.concatenate([rows[keep], [far, base.n]])
    v = np.concatenate([base.col[keep], [base.n, base.n + 1]])
    g = gg.from_edges(base.n + 2, u, v, name="grid34x35tail")
    say("grid34x35tail", form)
    with gpu_lib.BC(g, form=form) as ctx:
        d, sigma, delta = ctx.sssp(np.array([0], np.int32))
    x, y = np.divmod(np.arange(base.n), 35)
    want = [math.comb(int(a + b), int(a)) for a, b in zip(x, y)] + [math.comb(67, 33)] * 2
    assert math.comb(67, 33) > 2 ** 63
    assert [int(c) for c in sigma[0]] == want
    assert [int(t) for t in d[0]] == [int(a + b) for a, b in zip(x, y)] + [68, 69]
    assert rel_err(delta[0], oracle.sssp(g, 0)[2]) <= TOL[form]


@pytest.mark.parametrize("form", FORMS)
def test_multiset_ragged_and_accumulate(gpu_lib, form):
    g = gg.er_plus_tree(700, 5.0, 31)
    say("multiset_ragged", form)
    a = np.array([5, 5, 7, 699, 0], np.int32)
    b = np.arange(100, 400, dtype=np.int32)  # 300 sources: a full batch of 256 and a ragged tail
    with gpu_lib.BC(g, form=form) as ctx:
        ctx.run(a)
        assert rel_err(ctx.read(), oracle.bc(g, a)) <= TOL[form]
        ctx.run(b)
        assert rel_err(ctx.read(), oracle.bc(g, np.concatenate([a, b]))) <= TOL[form]
        ctx.reset()
        assert np.all(ctx.read() == 0.0)
        ctx.run(np.zeros(0, np.int32))
        assert np.all(ctx.read() == 0.0)


@pytest.mark.parametrize("form", FORMS)
def test_invalid_sources(gpu_lib, form):
    g = gg.path(10)
    with gpu_lib.BC(g, form=form) as ctx:
        with pytest.raises(gpu_lib.BCError) as ei:
            ctx.run(np.array([3, 10], np.int32))
        assert ei.value.status == gpu_lib.BC_ERR_INVALID_ARG
        ctx.run(np.array([3], np.int32))
        np.testing.assert_allclose(ctx.read(), oracle.bc(g, [3]), rtol=1e-12)


@pytest.mark.parametrize("form", FORMS)
def test_device_sources_and_deterministic_counts(gpu_lib, form):
    import torch
    g = gg.rmat(12, 16, 77)
    say("device_sources", form, g.n)
    src = torch.arange(0, g.n, 3, dtype=torch.int32, device="cuda:0")
    with gpu_lib.BC(g, form=form) as ctx:
        ctx.run(src)
        x = ctx.read()
        d1, s1, _ = ctx.sssp(np.arange(64, dtype=np.int32))
        d2, s2, _ = ctx.sssp(np.arange(64, dtype=np.int32))
    np.testing.assert_array_equal(d1, d2)
    np.testing.assert_array_equal(s1, s2)
    assert rel_err(x, oracle.bc(g, np.arange(0, g.n, 3))) <= TOL[form]


def test_rmat16_full_size_sampled(gpu_lib):
    """The benchmark workload (RMAT scale 16, batch 256) at full size: one full
    batch of per-source results bit-exact against the oracle, and BC over 512
    sources (two batches) within tolerance."""
    g = gg.rmat16()
    say("rmat16_full", g.n, g.m)
    rng = gg.Stream(2024)
    src = np.unique(np.concatenate([np.arange(8), np.arange(g.n - 8, g.n),
                                    rng.bounded(np.full(260, g.n))]))[:256].astype(np.int32)
    assert src.size == 256
    with gpu_lib.BC(g, form="sparse", batch=256) as ctx:
        dist, sigma, delta = ctx.sssp(src)
        for i in range(0, 256, 1):
            s = int(src[i])
            d, sg, dl = oracle.sssp_u64(g, s)
            assert np.array_equal(dist[i], d), f"dist source {s}"
            assert np.array_equal(sigma[i], sg), f"sigma source {s}"
            assert rel_err(delta[i], dl) <= 1e-5, f"delta source {s}"
        sub = rng.bounded(np.full(512, g.n)).astype(np.int32)
        ctx.run(sub)
        got = ctx.read()
    want = oracle.bc(g, sub, threads=8)
    err = rel_err(got, want)
    say("rmat16 BC(512 sources) max rel err", err)
    assert err <= 1e-5


def test_rmat16_algebraic_form_sampled(gpu_lib):
    """The algebraic form (products with the adjacency matrix on MFMA) at the
    benchmark's full size: one batch of per-source results, and BC over a
    ragged two-batch source list."""
    g = gg.rmat16()
    say("rmat16_algebraic", g.n, g.m)
    src = gg.Stream(99).bounded(np.full(256, g.n)).astype(np.int32)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        dist, sigma, delta = ctx.sssp(src)
        sub = src[:300 - 44]
        ctx.run(np.concatenate([sub, src[:44]]))
        got = ctx.read()
    for i in range(0, 256, 8):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {src[i]}"
        assert rel_err(delta[i], dl) <= 1e-5
    want = oracle.bc(g, np.concatenate([sub, src[:44]]), threads=8)
    assert rel_err(got, want) <= 1e-5


def test_algebraic_split_k(gpu_lib):
    """Forward products over a long K with fewer output tiles than two per
    compute unit run as two blocks per tile, each over half of K, meeting
    through agent-scope partial sums (ER n = 12000, mean degree 48, batch
    128: 96 tiles, K = 12032).  One batch of per-source results bit-exact, BC
    over a ragged two-batch source list."""
    g = gg.er_plus_tree(12000, 48.0, 77)
    say("algebraic_split_k", g.n, g.m)
    src = gg.sample_sources(g.n, 128, 78).astype(np.int32)
    sub = gg.sample_sources(g.n, 200, 79).astype(np.int32)
    with gpu_lib.BC(g, form="algebraic", batch=128) as ctx:
        dist, sigma, delta = ctx.sssp(src)
        ctx.run(sub)
        got = ctx.read()
        info = ctx.info()
    # k-tile counts: the forward's share within the totals, run within dense,
    # and each block counts its whole range of K = npad once per product pass
    npad = (g.n + 255) // 256 * 256
    assert 0 < info.mfma_ktiles_run_fwd <= info.mfma_ktiles_dense_fwd < info.mfma_ktiles_dense
    assert 0 < info.mfma_ktiles_run <= info.mfma_ktiles_dense
    assert info.mfma_ktiles_dense % (npad // 32) == 0
    for i in range(0, 128, 9):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {src[i]}"
        assert rel_err(delta[i], dl) <= 1e-5
    assert int(sigma.max()) > 255  # counts of more than one limb crossed the split
    assert rel_err(got, oracle.bc(g, sub, threads=8)) <= 1e-5


def test_algebraic_limbs_and_wide_counts(gpu_lib):
    """Counts of several 7-bit limbs (grid 20x20: up to C(38,19) > 2^32, so
    six limbs and uint64 storage) stay exact through the int8 products."""
    g = gg.grid(20, 20)
    say("algebraic_limbs")
    src = np.array([0, 19, 210, 399], np.int32)
    with gpu_lib.BC(g, form="algebraic") as ctx:
        dist, sigma, delta = ctx.sssp(src)
        ctx.run(src)
        got = ctx.read()
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
        assert rel_err(delta[i], dl) <= 1e-5
    assert rel_err(got, oracle.bc(g, src)) <= 1e-5


def test_rmat16_plain_form_sampled(gpu_lib):
    g = gg.rmat16()
    say("rmat16_plain", g.n, g.m)
    sub = gg.Stream(7).bounded(np.full(96, g.n)).astype(np.int32)
    with gpu_lib.BC(g, form="plain") as ctx:
        ctx.run(sub)
        got = ctx.read()
        dist, sigma, delta = ctx.sssp(sub[:8])
    assert rel_err(got, oracle.bc(g, sub, threads=8)) <= 1e-12
    for i in range(8):
        d, sg, dl = oracle.sssp_u64(g, int(sub[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
        assert rel_err(delta[i], dl) <= 1e-12


@pytest.mark.parametrize("split", [64, 100, 256])
@pytest.mark.parametrize("name", ["star4096", "rmat12", "kab"])
def test_split_rows_parity(gpu_lib, split, name):
    """Rows longer than split_degree are cut into segments whose partial sums
    meet through atomics; results must not depend on the cut."""
    g = {"star4096": lambda: gg.star(4096), "rmat12": lambda: gg.rmat(12, 16, 5),
         "kab": lambda: gg.complete_bipartite(3, 700)}[name]()
    say("split_rows", name, split, g.n, int(g.degrees().max()))
    want = oracle.bc(g)
    with gpu_lib.BC(g, form="sparse", split_degree=split) as ctx:
        ctx.run()
        got = ctx.read()
        src = np.array([0, 1, g.n - 1, g.n // 2], np.int32)
        dist, sigma, delta = ctx.sssp(src)
    assert rel_err(got, want) <= 1e-5
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
        assert rel_err(delta[i], dl) <= 1e-5


@pytest.mark.parametrize("form", FORMS)
def test_vertex_order_is_invisible(gpu_lib, form):
    """The internal numbering (degree order or input order) never shows in results."""
    g = gg.rmat(11, 16, 13)
    say("vertex_order", form, g.n)
    src = np.array([3, 17, 17, g.n - 1, 100], np.int32)
    out = {}
    for order in ("degree", "input"):
        with gpu_lib.BC(g, form=form, vertex_order=order) as ctx:
            ctx.run(src)
            out[order] = (ctx.read(),) + ctx.sssp(src[:3])
    want = oracle.bc(g, src)
    for order, (bc, dist, sigma, delta) in out.items():
        assert rel_err(bc, want) <= TOL[form], order
        for i, s in enumerate(src[:3]):
            d, sg, dl = oracle.sssp_u64(g, int(s))
            assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), order
            assert rel_err(delta[i], dl) <= TOL[form], order


def weighted_graphs():
    return [gg.random_graph(40, 0.15, 5, weights=9), gg.kkp_undirected(6),
            gg.with_uniform_weights(gg.er_plus_tree(500, 6.0, 8), 8, 1, 255),
            gg.with_constant_weight(gg.grid(15, 17), 3),
            gg.disjoint_union(gg.with_uniform_weights(gg.path(30), 2, 1, 4), gg.random_graph(50, 0.1, 9, weights=7)),
            gg.with_uniform_weights(gg.rmat(11, 16, 4), 4, 1, 255)]


@pytest.mark.parametrize("gi", range(6))
def test_weighted_bc_and_sssp(gpu_lib, gi):
    """Positive integer weights: bucketed shortest paths, one bucket per distance."""
    g = weighted_graphs()[gi]
    say("weighted", g.name, g.n, g.m)
    want = oracle.bc(g)
    src = np.unique(np.array([0, 1, g.n // 3, g.n - 1], np.int32))
    with gpu_lib.BC(g) as ctx:  # the automatic choice for weighted graphs
        assert ctx.info().form == gpu_lib.binding.BC_FORM_PLAIN_FP64
        ctx.run()
        got = ctx.read()
        dist, sigma, delta = ctx.sssp(src)
    assert rel_err(got, want) <= 1e-12
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d), f"dist source {s}"
        assert np.array_equal(sigma[i], sg), f"sigma source {s}"
        assert rel_err(delta[i], dl) <= 1e-12


def test_weighted_overflow_reported(gpu_lib):
    g = gg.with_constant_weight(gg.grid(35, 35), 2)
    say("weighted_overflow")
    with gpu_lib.BC(g) as ctx:
        ctx.run(np.array([0], np.int32))
        with pytest.raises(gpu_lib.BCError) as ei:
            ctx.read()
        assert ei.value.status == gpu_lib.BC_ERR_OVERFLOW


def test_weighted_rmat16_sampled(gpu_lib):
    """RMAT-16 with weights U{1..255}: a seeded source sample against the oracle."""
    g = gg.with_uniform_weights(gg.rmat16(), 77, 1, 255)
    say("weighted_rmat16", g.n, g.m)
    src = gg.sample_sources(g.n, 96, 77)
    with gpu_lib.BC(g) as ctx:
        ctx.run(src)
        got = ctx.read()
        dist, sigma, delta = ctx.sssp(src[:6])
    assert rel_err(got, oracle.bc(g, src, threads=8)) <= 1e-12
    for i in range(6):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
        assert rel_err(delta[i], dl) <= 1e-12


@pytest.mark.parametrize("log2", [6, 9])
def test_weighted_arena_retry(gpu_lib, log2):
    """A tiny relaxation ring forces sources onto the full-size re-run path;
    results must not change."""
    g = gg.with_uniform_weights(gg.er_plus_tree(800, 8.0, 21), 21, 1, 255)
    say("weighted_retry", log2)
    src = np.arange(0, g.n, 3, dtype=np.int32)
    with gpu_lib.BC(g, arena_log2=log2) as ctx:
        ctx.run(src)
        got = ctx.read()
        dist, sigma, delta = ctx.sssp(src[:5])
    assert rel_err(got, oracle.bc(g, src)) <= 1e-12
    for i in range(5):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
        assert rel_err(delta[i], dl) <= 1e-12


def many_graphs():
    gs = [gg.path(1), gg.path(2), gg.path(40), gg.cycle(31), gg.star(300), gg.complete(50), gg.grid(12, 13),
          gg.random_tree(500, 4), gg.complete_bipartite(4, 9), gg.er_plus_tree(700, 5.0, 6),
          gg.disjoint_union(gg.path(9), gg.cycle(12))]
    sizes = gg.Stream(31).bounded(np.full(40, 4096 - 64 + 1)) + 64
    gs += [gg.watts_strogatz(int(n), 6, 0.1, 1000 + i) for i, n in enumerate(sizes)]
    gs.append(gg.watts_strogatz(4096, 6, 0.1, 7))
    return gs


def test_many_graphs_one_launch(gpu_lib):
    """Many graphs in one persistent, graph-captured launch: each graph's BC
    equals its own oracle BC; replays accumulate; readouts use the
    concatenated numbering."""
    gs = many_graphs()
    say("many_graphs", len(gs), sum(g.n for g in gs))
    want = np.concatenate([oracle.bc(g, threads=8) for g in gs])
    with gpu_lib.BC(gs) as ctx:
        assert ctx.info().form == gpu_lib.binding.BC_FORM_MANY
        ctx.run()
        first = ctx.read()
        assert rel_err(first, want) <= 1e-5
        ctx.run()  # replay of the recorded launch
        ctx.run()
        assert rel_err(ctx.read(), 3 * want) <= 1e-5
        ctx.reset()
        assert np.all(ctx.read() == 0.0)
        ctx.run()
        assert rel_err(ctx.read(), want) <= 1e-5
        with pytest.raises(gpu_lib.BCError) as ei:
            ctx.run(np.array([0], np.int32))
        assert ei.value.status == gpu_lib.BC_ERR_UNSUPPORTED
        offs = np.concatenate([[0], np.cumsum([g.n for g in gs])])
        picks = [(9, 3), (10, 0), (len(gs) - 1, 100)]
        src = np.array([offs[g] + v for g, v in picks], np.int32)
        dist, sigma, delta = ctx.sssp(src)
    for i, (g, v) in enumerate(picks):
        d, sg, dl = oracle.sssp_u64(gs[g], v)
        lo, hi = offs[g], offs[g + 1]
        assert np.array_equal(dist[i][lo:hi], d) and np.array_equal(sigma[i][lo:hi], sg)
        assert np.all(dist[i][:lo] == -1) and np.all(dist[i][hi:] == -1)
        assert rel_err(delta[i][lo:hi], dl) <= 1e-5


def test_many_graphs_columns_from_memory(gpu_lib):
    """Graphs whose arcs do not fit the workgroup's staged 16-bit columns
    (K_300: 89 700 arcs; ER n=4096 degree 14: 57 400) read them from global
    memory, in the same launch as graphs that fit."""
    gs = [gg.complete(300), gg.er_plus_tree(4096, 12.0, 3), gg.path(600), gg.star(4096),
          gg.watts_strogatz(3000, 6, 0.1, 5)]
    say("many_graphs_wide", [g.col.size for g in gs])
    want = np.concatenate([oracle.bc(g, threads=8) for g in gs])
    with gpu_lib.BC(gs) as ctx:
        ctx.run()
        assert rel_err(ctx.read(), want) <= 1e-5


def test_many_graphs_overflow(gpu_lib):
    gs = [gg.path(5), gg.grid(35, 35)]  # C(68,34) > 2^64 - 1 in the second graph
    say("many_overflow")
    with gpu_lib.BC(gs) as ctx:
        ctx.run()
        with pytest.raises(gpu_lib.BCError) as ei:
            ctx.read()
        assert ei.value.status == gpu_lib.BC_ERR_OVERFLOW


def test_many_graphs_handed_back_units(gpu_lib):
    """Units that the compact sweep cannot finish go to the full sweep:
    counts above 2^32 - 1 (grid 20 x 20: up to C(38,19) ~ 3.5e10) and
    sources deeper than its level cap (a 1500-path, a 2500-cycle), in the
    same launch as units it does finish.  Replays add again."""
    gs = [gg.grid(20, 20), gg.path(1500), gg.watts_strogatz(1000, 6, 0.1, 3), gg.cycle(2500), gg.star(64)]
    say("many_handback", [g.n for g in gs])
    want = np.concatenate([oracle.bc(g, threads=8) for g in gs])
    with gpu_lib.BC(gs) as ctx:
        ctx.run()
        assert rel_err(ctx.read(), want) <= 1e-5
        ctx.run()
        assert rel_err(ctx.read(), 2 * want) <= 1e-5
