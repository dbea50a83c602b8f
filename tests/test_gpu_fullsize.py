"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times, on the outputs the oracle can compute one by one (per-source
distances, counts and dependencies; BC over source subsets; single graphs of a
many-graph launch) and on properties that hold at any size."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def test_er16384_products_batch512(gpu_lib):
    """ER n = 16384, mean degree 256, batches of 512 as the benchmark runs
    them: the algebraic form (every level by MFMA products) and the hybrid
    form (its tuned mix).  One batch of per-source results bit-exact in d and
    lambda; BC over 1000 sources (the second batch ragged)."""
    g = gg.er16384()
    src = gg.sample_sources(g.n, 512, 41)
    sub = gg.sample_sources(g.n, 1000, 42)
    say("er16384 oracle BC over 1000 sources")
    want = oracle.bc(g, sub, threads=16)
    picks = list(range(0, 512, 32)) + [511]
    per = {i: oracle.sssp_u64(g, int(src[i])) for i in picks}
    for form in ("algebraic", "hybrid"):
        say("er16384", form, g.n, g.m)
        with gpu_lib.BC(g, form=form, batch=512) as ctx:
            dist, sigma, delta = ctx.sssp(src)
            ctx.run(sub)
            got = ctx.read()
        for i in picks:
            d, sg, dl = per[i]
            assert np.array_equal(dist[i], d), f"{form} dist source {src[i]}"
            assert np.array_equal(sigma[i], sg), f"{form} sigma source {src[i]}"
            assert rel_err(delta[i], dl) <= 1e-5, f"{form} delta source {src[i]}"
        err = rel_err(got, want)
        say("er16384", form, "BC max rel err", err)
        assert err <= 1e-5


def test_ws4096_full_launch_sampled_graphs(gpu_lib):
    """All 4096 Watts-Strogatz graphs in one launch, as the benchmark runs
    them; the BC of 26 graphs (the largest, the smallest, the first, the last
    and a seeded sample) against the oracle graph by graph."""
    gs = gg.ws_batch(4096)
    sizes = np.array([x.n for x in gs])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    pick = sorted({0, len(gs) - 1, int(sizes.argmax()), int(sizes.argmin())} |
                  {int(i) for i in gg.sample_sources(len(gs), 22, 43)})
    say("ws4096", len(gs), int(sizes.sum()))
    with gpu_lib.BC(gs) as ctx:
        ctx.run()
        got = ctx.read()
    assert np.all(np.isfinite(got)) and np.all(got >= 0.0)
    for i in pick:
        err = rel_err(got[offs[i]:offs[i + 1]], oracle.bc(gs[i], threads=16))
        assert err <= 1e-5, f"graph {i} (n = {gs[i].n}): {err}"


def test_rmat20w_full_size_sampled(gpu_lib):
    """RMAT scale 20 with weights U{1..255} and its 4096 sampled sources, by
    the bucketed per-source sweep as the benchmark runs it.
    - Three sources' distances and counts bit-exact, dependencies in FP64.
    - BC over the first 24 sources against the oracle.
    - BC over all 4096 sources at least that over the first 24: every
      dependency is non-negative and the 24 are among the 4096."""
    say("rmat20w generate")
    g, src = gg.rmat20w()
    say("rmat20w", g.n, g.m, src.size)
    with gpu_lib.BC(g, form="plain") as ctx:
        ctx.run(src)
        full = ctx.read()
        dist, sigma, delta = ctx.sssp(src[[0, 2048, 4095]])
    with gpu_lib.BC(g, form="plain") as ctx:
        ctx.run(src[:24])
        part = ctx.read()
    for i, s in enumerate(src[[0, 2048, 4095]]):
        d, sg, dl = oracle.sssp_u64(g, int(s))
        assert np.array_equal(dist[i], d), f"dist source {s}"
        assert np.array_equal(sigma[i], sg), f"sigma source {s}"
        assert rel_err(delta[i], dl) <= 1e-12, f"delta source {s}"
    say("rmat20w oracle BC over 24 sources")
    assert rel_err(part, oracle.bc(g, src[:24], threads=16)) <= 1e-12
    assert np.all(full >= part - 1e-9 * np.maximum(np.abs(part), 1.0))
