"""Whole-workload parity: every benchmark workload's BC over all of its
sources (or, for the sampled weighted workload, a stated sample), in the form,
batch width and launch configuration bench.py times, element by element
against the oracle's BC over the same sources (Sec. 1.1: BC sums the
dependencies of every source, ordered pairs).

Error metric (the same everywhere): err = max_v |x_v - y_v| / max(|y_v|, 1);
each test prints it with its argmax vertex and the largest purely relative
error over vertices with BC >= 1.  Tolerances: 1e-5 where c(v) is stored in
FP32 (sparse, hybrid, algebraic, many graphs), 1e-12 for the plain FP64 form
and the weighted sweep."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import oracle_threads

pytestmark = pytest.mark.gpu


def report(label, got, want):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    e = np.abs(got - want) / np.maximum(np.abs(want), 1.0)
    i = int(np.argmax(e)) if e.size else -1
    big = np.abs(want) >= 1.0
    pure = float(np.max(np.abs(got - want)[big] / np.abs(want)[big])) if np.any(big) else 0.0
    err = float(e[i]) if e.size else 0.0
    print(f"[gpu-case] {label}: max err {err:.3e} at vertex {i} (BC {want[i] if e.size else 0:.6g}); "
          f"max relative err over BC >= 1: {pure:.3e}", flush=True)
    return err


@pytest.fixture(scope="module")
def rmat16():
    return gg.rmat16()


@pytest.mark.parametrize("form,batch,tol", [("hybrid", 256, 1e-5), ("hybrid", 0, 1e-5), ("plain", 0, 1e-12)])
def test_rmat16_all_sources(gpu_lib, oracle_all_sources, rmat16, form, batch, tol):
    """RMAT-16, all 46 735 sources: the headline's batched form at batch 256
    with its tuned level mix, the tuner's own batch width, and the plain FP64
    form that the headline is compared with."""
    g = rmat16
    want = oracle_all_sources("rmat16", g)
    print(f"[gpu-case] rmat16 all sources form={form} batch={batch}", flush=True)
    with gpu_lib.BC(g, form=form, batch=batch) as ctx:
        ctx.run()
        got = ctx.read()
        assert ctx.info().sources_run == g.n
    assert report(f"rmat16 {form} batch {batch}", got, want) <= tol


@pytest.mark.parametrize("form", ["algebraic", "hybrid", "sparse"])
def test_er16384_all_sources(gpu_lib, oracle_all_sources, form):
    """ER n = 16384, mean degree 256, all sources at batch 512: the algebraic
    form (every level by MFMA products), the hybrid form (its tuned mix) and
    the sparse form, as the benchmark runs them."""
    g = gg.er16384()
    want = oracle_all_sources("er16384", g)
    print(f"[gpu-case] er16384 all sources form={form}", flush=True)
    with gpu_lib.BC(g, form=form, batch=512) as ctx:
        ctx.run()
        got = ctx.read()
    assert report(f"er16384 {form}", got, want) <= 1e-5


def test_er1024_all_sources_plain(gpu_lib):
    """ER n = 1024 plus a spanning tree, all 1024 sources by the plain FP64
    form."""
    g = gg.er1024()
    with gpu_lib.BC(g, form="plain") as ctx:
        ctx.run()
        got = ctx.read()
    assert report("er1024 plain", got, oracle.bc(g, threads=oracle_threads())) <= 1e-12


def test_ws4096_all_graphs_one_launch(gpu_lib):
    """All 4096 Watts-Strogatz graphs in one persistent launch, as the
    benchmark runs them; 1024 of them (a seeded sample, plus the largest,
    the smallest, the first and the last) against the oracle graph by graph."""
    gs = gg.ws_batch(4096)
    sizes = np.array([x.n for x in gs])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    pick = sorted({0, len(gs) - 1, int(sizes.argmax()), int(sizes.argmin())} |
                  {int(i) for i in gg.sample_sources(len(gs), 1024, 44)})
    print(f"[gpu-case] ws4096 {len(gs)} graphs, {len(pick)} checked", flush=True)
    with gpu_lib.BC(gs) as ctx:
        ctx.run()
        got = ctx.read()
    assert np.all(np.isfinite(got)) and np.all(got >= 0.0)
    threads = oracle_threads()
    worst, at = 0.0, -1
    for i in pick:
        want = oracle.bc(gs[i], threads=threads)
        e = float(np.max(np.abs(got[offs[i]:offs[i + 1]] - want) / np.maximum(np.abs(want), 1.0)))
        if e > worst:
            worst, at = e, i
    print(f"[gpu-case] ws4096: max err {worst:.3e} in graph {at} (n = {gs[at].n if at >= 0 else 0})", flush=True)
    assert worst <= 1e-5


def test_rmat20w_256_sources(gpu_lib):
    """RMAT-20 with weights U{1..255}: the first 256 of the workload's 4096
    sampled sources by the bucketed per-source sweep, against the oracle's
    Dijkstra-based Brandes over the same sources."""
    g, src = gg.rmat20w()
    sub = src[:256]
    print(f"[gpu-case] rmat20w n={g.n} m={g.m}, 256 sources", flush=True)
    with gpu_lib.BC(g, form="plain") as ctx:
        ctx.run(sub)
        got = ctx.read()
    want = oracle.bc(g, sub, threads=oracle_threads())
    assert report("rmat20w plain, 256 sources", got, want) <= 1e-12
