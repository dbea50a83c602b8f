"""GPU tests of the tuner's shape choices: the forward products' rows per
workgroup (algebraic and hybrid forms) and the sources per work unit of
bc_create_many's queue.

Neither choice may change a result.  The forward products sum exact integer
counts (7-bit limbs, degrees within BC_ALGEBRAIC_MAX_DEGREE), so distances and
path counts are the same bit for bit with 128- and 256-row workgroups, and the
backward, which the choice does not touch, then writes the same dependencies.
A work unit's size only regroups the FP64 sums of the many-graph sweep.
Choices are forced through the tuning cache file: a first create writes the
graph's key, an appended entry for that key overrides it (the last entry for
a key wins).
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import oracle_threads

pytestmark = pytest.mark.gpu

TOL = 1e-5
UNIT_SIZES = (16, 32, 64, 128, 256)


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def last_key(path):
    lines = [ln for ln in open(path).read().splitlines() if ln and not ln.startswith("#")]
    return lines[-1].split("\t")[0]


def force_entry(gpu_lib, graph, path, fields, **kw):
    """Creates one context of `graph` with the cache file (writing its key),
    then appends an entry for that key with the given value fields."""
    with gpu_lib.BC(graph, tune_cache=path, **kw):
        pass
    key = last_key(path)
    with open(path, "a") as f:
        f.write(key + "\t" + " ".join(str(x) for x in fields) + "\n")
    return key


def test_algebraic_rows_measured_then_cached(gpu_lib, tmp_path):
    """A graph large enough for calibration: the algebraic form times both
    block shapes, reports the one it kept, a second context takes it from the
    cache file, and BC stays within tolerance of the oracle."""
    g = gg.er_plus_tree(2500, 24.0, 5, name="er2500")
    path = str(tmp_path / "tune.txt")
    src = gg.Stream(8).bounded(np.full(300, g.n)).astype(np.int32)
    want = oracle.bc(g, src, threads=oracle_threads())
    say("alg_rows_measured", g.n, g.m)
    with gpu_lib.BC(g, form="algebraic", batch=256, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_MEASURED
        assert info.mfma_fwd_rows in (128, 256)
        assert info.sources_run == 0 and info.max_levels == 0 and info.mfma_planes == 0
        rows = info.mfma_fwd_rows
        say("chose", rows)
        ctx.run(src)
        assert rel_err(ctx.read(), want) <= TOL
    text = open(path).read()
    assert f"n={g.n} " in text and f"form={gpu_lib.BC_FORM_ALGEBRAIC} " in text
    assert text.splitlines()[-1].split()[-1] == str(rows)
    with gpu_lib.BC(g, form="algebraic", batch=256, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED and info.mfma_fwd_rows == rows
        ctx.run(src)
        assert rel_err(ctx.read(), want) <= TOL


def check_ktiles(info, g, batch):
    """K-tiles are 2^20 flops whatever the block rows: those the issued
    products cover equal the issued planes' flops exactly, and those run are
    no more."""
    npad = max(256, (g.n + 255) // 256 * 256)
    classes = int(g.weight.max()) if g.weight is not None else 1
    assert info.mfma_planes > 0
    assert info.mfma_ktiles_dense * 2 ** 20 == info.mfma_planes * 2 * batch * npad * classes * npad
    assert 0 < info.mfma_ktiles_run <= info.mfma_ktiles_dense
    assert 0 < info.mfma_ktiles_run_fwd <= info.mfma_ktiles_dense_fwd < info.mfma_ktiles_dense


CASES = {
    # npad 4096, batch 256: 128 tiles of 128 rows, K whole in each block
    "er4096": (lambda: gg.er_plus_tree(4096, 16.0, 12, name="er4096"), 256),
    # K split in two halves per output tile (K = npad = 12032 >= 8192 with
    # fewer than 512 tiles): both block shapes meet through the split
    # workspace, 256-row blocks with half as many tiles
    "er12000_split": (lambda: gg.er_plus_tree(12000, 48.0, 77), 128),
    # weight classes 1..4: K = 4 npad, no split
    "er2100w4": (lambda: gg.with_uniform_weights(gg.er_plus_tree(2100, 12.0, 13), 14, 1, 4), 256),
    # a small graph (one tile row of 256) at batch 512
    "rmat9": (lambda: gg.rmat(9, 16, 15), 512),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_algebraic_rows_do_not_change_results(gpu_lib, tmp_path, name):
    """Both block shapes forced through the cache: per-source distances,
    counts and dependencies identical bit for bit, equal to the oracle's
    (dependencies within tolerance), and BC within rounding of each other."""
    make, batch = CASES[name]
    g = make()
    src = np.concatenate([np.arange(4), gg.Stream(9).bounded(np.full(60, g.n))]).astype(np.int32)
    out = {}
    path = str(tmp_path / "tune.txt")
    for rows in (128, 256):
        force_entry(gpu_lib, g, path, [batch, 2.0, 2.0, rows], form="algebraic", batch=batch)
        say("alg_rows", name, g.n, rows)
        with gpu_lib.BC(g, form="algebraic", batch=batch, tune_cache=path) as ctx:
            info = ctx.info()
            assert info.tune_source == gpu_lib.BC_TUNE_CACHED and info.mfma_fwd_rows == rows
            dist, sigma, delta = ctx.sssp(src)
            ctx.run(src)
            out[rows] = (dist, sigma, delta, ctx.read())
            check_ktiles(ctx.info(), g, batch)
    d1, s1, l1, b1 = out[128]
    d2, s2, l2, b2 = out[256]
    assert np.array_equal(d1, d2) and np.array_equal(s1, s2) and np.array_equal(l1, l2)
    assert rel_err(b2, b1) <= 1e-12
    for i in range(0, src.size, 7):
        d, sg, dl = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(d2[i], d) and np.array_equal(s2[i], sg), f"source {src[i]}"
        assert rel_err(l2[i], dl) <= TOL, f"source {src[i]}"
    assert rel_err(b2, oracle.bc(g, src, threads=oracle_threads())) <= TOL


def test_algebraic_rows_full_tiles_er16384(gpu_lib, tmp_path):
    """ER-16384 at batch 512 (a full chip of tiles, no K split) with 256-row
    workgroups forced: per-source results bit-equal to 128-row workgroups and
    to the oracle's counts."""
    g = gg.er16384()
    src = gg.Stream(10).bounded(np.full(64, g.n)).astype(np.int32)
    out = {}
    path = str(tmp_path / "tune.txt")
    for rows in (128, 256):
        force_entry(gpu_lib, g, path, [512, 2.0, 2.0, rows], form="algebraic", batch=512)
        say("alg_rows_er16384", rows)
        with gpu_lib.BC(g, form="algebraic", batch=512, tune_cache=path) as ctx:
            assert ctx.info().mfma_fwd_rows == rows
            out[rows] = ctx.sssp(src)
    for a, b in zip(out[128], out[256]):
        assert np.array_equal(a, b)
    for i in range(0, 64, 16):
        d, sg, _ = oracle.sssp_u64(g, int(src[i]))
        assert np.array_equal(out[256][0][i], d) and np.array_equal(out[256][1][i], sg)


def test_hybrid_rows_cached(gpu_lib, tmp_path):
    """The hybrid form with every level by products and 256-row forward
    workgroups: the cache entry's rows are used and BC matches the oracle."""
    g = gg.er1024()
    path = str(tmp_path / "tune.txt")
    force_entry(gpu_lib, g, path, [256, 0.0, 0.0, 256], form="hybrid", batch=256)
    with gpu_lib.BC(g, form="hybrid", batch=256, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED and info.mfma_fwd_rows == 256
        ctx.run()
        got = ctx.read()
        assert ctx.info().mfma_planes > 0
    assert rel_err(got, oracle.bc(g, threads=oracle_threads())) <= TOL


def test_sparse_reports_no_rows(gpu_lib):
    g = gg.er1024()
    with gpu_lib.BC(g, form="sparse", batch=256) as ctx:
        assert ctx.info().mfma_fwd_rows == 0


@pytest.mark.parametrize("fields", [[256, 2.0, 2.0, 192], [128, 2.0, 2.0, 128]])
def test_algebraic_unusable_cache_entry(gpu_lib, tmp_path, fields):
    """A cache entry with block rows other than 128 or 256, or a batch other
    than the requested one, is refused at create."""
    g = gg.er1024()
    path = str(tmp_path / "tune.txt")
    force_entry(gpu_lib, g, path, fields, form="algebraic", batch=256)
    with pytest.raises(gpu_lib.BCError) as ei:
        gpu_lib.BC(g, form="algebraic", batch=256, tune_cache=path)
    assert ei.value.status == gpu_lib.BC_ERR_INVALID_ARG


def many_graphs():
    return gg.ws_batch(48, 64, 700, seed=77)


def check_many(gs, got, picks):
    offs = np.concatenate([[0], np.cumsum([x.n for x in gs])])
    for i in picks:
        want = oracle.bc(gs[i], threads=oracle_threads())
        assert rel_err(got[offs[i]:offs[i + 1]], want) <= TOL, f"graph {i}"


def test_many_unit_size_measured_then_cached(gpu_lib, tmp_path):
    """Many graphs with enough vertices for calibration: the unit size is one
    of the timed candidates, a second context takes it from the cache file,
    and BC matches the oracle graph by graph."""
    gs = many_graphs()
    assert sum(x.n for x in gs) >= 2048
    path = str(tmp_path / "tune.txt")
    say("many_measured", len(gs))
    with gpu_lib.BC(gs, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_MEASURED and info.batch in UNIT_SIZES
        assert info.sources_run == 0
        unit = info.batch
        say("chose", unit)
        ctx.run()
        got = ctx.read()
    assert "many graphs=48 " in open(path).read()
    check_many(gs, got, [0, 5, 17, 47])
    with gpu_lib.BC(gs, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED and info.batch == unit
        ctx.run()
        assert rel_err(ctx.read(), got) <= 1e-12


@pytest.mark.parametrize("unit", [16, 256])
def test_many_unit_size_forced(gpu_lib, tmp_path, unit):
    """A unit size forced through the cache is used and only regroups sums."""
    gs = many_graphs()
    path = str(tmp_path / "tune.txt")
    force_entry(gpu_lib, gs, path, [unit, 2.0, 2.0, 0])
    with gpu_lib.BC(gs, tune_cache=path) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_CACHED and info.batch == unit
        ctx.run()
        got = ctx.read()
    with gpu_lib.BC(gs, batch=64) as ctx:
        assert ctx.info().tune_source == gpu_lib.BC_TUNE_DEFAULT and ctx.info().batch == 64
        ctx.run()
        ref = ctx.read()
    assert rel_err(got, ref) <= 1e-12
    check_many(gs, got, [1, 30])


def test_many_small_total_takes_default(gpu_lib, tmp_path):
    gs = [gg.path(20), gg.cycle(30), gg.complete(12)]
    with gpu_lib.BC(gs, tune_cache=str(tmp_path / "t.txt")) as ctx:
        info = ctx.info()
        assert info.tune_source == gpu_lib.BC_TUNE_DEFAULT and info.batch == 64
