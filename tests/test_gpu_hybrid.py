"""GPU parity of the hybrid form and of the tuner that configures it.

The hybrid form takes each level l >= 1 either by CSR pulls (the level sweep
of Sec. 4) or by products with the adjacency matrix (Sec. 3.1), from the
level's union-frontier density against two thresholds.  Whatever the mix,
distances and path counts must equal the oracle's bit for bit and BC must stay
within the FP32-state tolerance.  Thresholds are forced through the tuning
cache file: a first create writes the graph's key, an appended entry for that
key overrides it.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5
# (forward threshold, backward threshold): all products, products forward
# only, products backward only, a density-dependent mix, all pulls
MIXES = [(0.0, 0.0), (0.0, 2.0), (2.0, 0.0), (0.3, 0.25), (2.0, 2.0)]


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def force_thresholds(gpu_lib, g, path, tf, tb, batch=256):
    """Writes a tuning-cache entry fixing the hybrid thresholds for g."""
    with gpu_lib.BC(g, form="hybrid", batch=batch, tune_cache=path):
        pass
    lines = [ln for ln in open(path).read().splitlines() if ln and not ln.startswith("#")]
    key = lines[-1].split("\t")[0]
    assert "form=4" in key and f"n={g.n} " in key
    with open(path, "a") as f:
        f.write(f"{key}\t{batch} {tf!r} {tb!r}\n")


def graphs():
    return {"er1024": gg.er1024(), "grid20": gg.grid(20, 20), "ws300": gg.watts_strogatz(300, 6, 0.1, 7),
            "union": gg.disjoint_union(gg.path(40), gg.er_plus_tree(200, 5.0, 3)), "complete64": gg.complete(64),
            "star50": gg.star(50), "path33": gg.path(33)}


@pytest.mark.parametrize("mix", range(len(MIXES)))
@pytest.mark.parametrize("name", ["er1024", "grid20", "ws300", "union", "complete64", "star50", "path33"])
def test_hybrid_forced_mix_bc(gpu_lib, tmp_path, name, mix):
    g = graphs()[name]
    tf, tb = MIXES[mix]
    say("hybrid_mix_bc", name, tf, tb)
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, tf, tb)
    want = oracle.bc(g)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.form == gpu_lib.BC_FORM_HYBRID
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED
        assert info.mfma_density_fwd == tf and info.mfma_density_bwd == tb
        ctx.run()
        got = ctx.read()
        planes = ctx.info().mfma_planes
    assert rel_err(got, want) <= TOL
    # the backward decides from the batch's own densities, so products appear
    # in the first batch already (wherever a level has a deeper one: not in
    # K_64, of diameter 1); the forward follows the previous batch
    if (tf, tb) == (0.0, 0.0) and name != "complete64":
        assert planes > 0
    if (tf, tb) == (2.0, 2.0):
        assert planes == 0


@pytest.mark.parametrize("mix", range(len(MIXES)))
@pytest.mark.parametrize("name", ["er1024", "grid20", "union"])
def test_hybrid_forced_mix_sssp_bit_exact(gpu_lib, tmp_path, name, mix):
    g = graphs()[name]
    tf, tb = MIXES[mix]
    say("hybrid_mix_sssp", name, tf, tb)
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, tf, tb)
    rng = gg.Stream(77)
    src = np.concatenate([np.arange(4), rng.bounded(np.full(60, g.n))]).astype(np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        dist, sigma, delta = ctx.sssp(src)
    for i, s in enumerate(src):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d), f"dist source {s}"
        assert np.array_equal(sigma[i], sg), f"sigma source {s}"
        assert rel_err(delta[i], dl) <= TOL, f"delta source {s}"


def test_hybrid_wide_counts_through_products(gpu_lib, tmp_path):
    """Grid 20x20 counts reach C(38,19) > 2^32: uint64 storage and several
    7-bit limbs, with every level by products."""
    g = gg.grid(20, 20)
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, 0.0, 0.0)
    src = np.array([0, 19, 380, 399, 210], np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        _, sigma, _ = ctx.sssp(src)
        ctx.run()
        got = ctx.read()
    for i, s in enumerate(src):
        assert np.array_equal(sigma[i], oracle.sssp_u64(g, int(s))[1])
    assert sigma.max() > 2 ** 32
    assert rel_err(got, oracle.bc(g)) <= TOL


def test_hybrid_overflow_reported(gpu_lib, tmp_path):
    g = gg.grid(35, 35)
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, 0.0, 0.0)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        ctx.run()
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.read()
        assert e.value.status == gpu_lib.BC_ERR_OVERFLOW


def test_tuner_measures_then_caches(gpu_lib, tmp_path):
    """A graph large enough for calibration: the tuner measures, the chosen
    width and thresholds are valid, a second context of the same graph takes
    them from the cache, and results stay exact."""
    g = gg.er_plus_tree(6000, 24.0, 11, name="er6000")
    path = str(tmp_path / "tune.txt")
    say("tuner", g.n, g.m)
    src = gg.Stream(5).bounded(np.full(700, g.n)).astype(np.int32)
    want = oracle.bc(g, src, threads=8)
    with gpu_lib.BC(g, form="hybrid", tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_MEASURED
        assert info.batch in (256, 512)
        for t in (info.mfma_density_fwd, info.mfma_density_bwd):
            assert t == 2.0 or 0.0 <= t <= 1.0
        assert info.sources_run == 0 and info.max_levels == 0
        first = (info.batch, info.mfma_density_fwd, info.mfma_density_bwd)
        say("tuned", first)
        ctx.run(src)
        assert rel_err(ctx.read(), want) <= TOL
    text = open(path).read()
    assert "form=4" in text and f"n={g.n} " in text
    with gpu_lib.BC(g, form="hybrid", tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED
        assert (info.batch, info.mfma_density_fwd, info.mfma_density_bwd) == first
        ctx.run(src)
        assert rel_err(ctx.read(), want) <= TOL
    with gpu_lib.BC(g, form="sparse") as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_MEASURED
        assert info.batch in (128, 256, 512)
        assert info.mfma_density_fwd == 2.0
        ctx.run(src)
        assert rel_err(ctx.read(), want) <= TOL


def test_rmat16_hybrid_sampled(gpu_lib):
    """The benchmark workload in the hybrid form with tuned thresholds: one
    batch of per-source results bit-exact, BC over 512 sources."""
    g = gg.rmat16()
    say("rmat16_hybrid", g.n, g.m)
    rng = gg.Stream(31)
    src = rng.bounded(np.full(256, g.n)).astype(np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256) as ctx:
        info = ctx.info()
        say("tuned", info.tune_source, info.mfma_density_fwd, info.mfma_density_bwd)
        dist, sigma, delta = ctx.sssp(src)
        for i in range(0, 256, 4):
            d, sg, dl = oracle.sssp_u64(g, int(src[i]))
            assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {src[i]}"
            assert rel_err(delta[i], dl) <= TOL
        sub = rng.bounded(np.full(512, g.n)).astype(np.int32)
        ctx.run(sub)
        got = ctx.read()
    assert rel_err(got, oracle.bc(g, sub, threads=8)) <= TOL


# The every-level mode: thresholds -1 in the cache (what the tuner writes when
# whole batches with every level by products beat its per-level choice) give
# the algebraic form's run inside the hybrid form, end of search included.
@pytest.mark.parametrize("name", ["er1024", "grid20", "union", "path33"])
def test_hybrid_every_level_mode(gpu_lib, tmp_path, name):
    """Forced every-level mode: reported thresholds 0 / 0, BC and per-source
    results as the oracle's, and the forward's k-tiles the same as the
    algebraic form's on the same sources (the empty last level is skipped)."""
    g = graphs()[name]
    say("hybrid_every", name)
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, -1.0, -1.0)
    rng = gg.Stream(91)
    src = np.concatenate([np.arange(3), rng.bounded(np.full(120, g.n))]).astype(np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED
        assert info.mfma_density_fwd == 0.0 and info.mfma_density_bwd == 0.0
        ctx.run(src)
        got = ctx.read()
        hy = ctx.info()
        dist, sigma, delta = ctx.sssp(src[:64])
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        ctx.run(src)
        al = ctx.info()
    assert hy.mfma_ktiles_dense_fwd == al.mfma_ktiles_dense_fwd
    assert rel_err(got, oracle.bc(g, src)) <= TOL
    for i in range(0, 64, 5):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg), f"source {src[i]}"
        assert rel_err(delta[i], dl) <= TOL


def test_hybrid_every_level_mode_not_with_edges(gpu_lib, tmp_path):
    """Edge betweenness needs the per-arc pulls: a context with edges reads the
    every-level entry as pulls at every level, and its edge BC is the
    oracle's."""
    g = graphs()["er1024"]
    path = str(tmp_path / "tune.txt")
    force_thresholds(gpu_lib, g, path, -1.0, -1.0)
    want_bc, want_eb = oracle.edge_bc(g)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path, edges=True) as ctx:
        info = ctx.info()
        assert info.mfma_density_fwd == 2.0 and info.mfma_density_bwd == 2.0
        ctx.run()
        got_bc, got_eb = ctx.read(), ctx.read_edges()
        assert ctx.info().mfma_planes == 0
    assert rel_err(got_bc, want_bc) <= TOL and rel_err(got_eb, want_eb) <= TOL
