"""Kernel timing with HIP events: every launch (timing = 1) or every launch of
one source batch in k (timing = k).  Driven from the host, sampling changes
which launches carry events, never the launch count.  With replayed batches
(the default) the timed batches run host-driven and the others replay
without events; totals and counts are scaled by batches.  Results never
change."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

NAMES = ("fwd_pull", "bwd_pull", "batch_init")


def say(*a):
    print("[gpu-case]", *a, flush=True)


def test_batch_sampled_timing(gpu_lib):
    g = gg.rmat(12, 16, 7)
    say("timing", g.n, g.m)
    got = {}
    for k, host in ((0, False), (1, True), (5, True), (5, False)):
        with gpu_lib.BC(g, form="sparse", batch=64, timing=k, host_driven=host) as ctx:
            ctx.run()
            bc = ctx.read()
            got[(k, host)] = (bc, {name: ctx.timing(name) for name in NAMES})
    assert all(v == (0.0, 0) for v in got[(0, False)][1].values())
    for name in NAMES:
        ms1, n1 = got[(1, True)][1][name]
        ms5, n5 = got[(5, True)][1][name]
        msr, nr = got[(5, False)][1][name]
        assert n1 == n5 > 0, name
        assert ms1 > 0 and ms5 > 0 and msr > 0, name
        # the sampled total is the timed batches' average scaled to every launch
        assert 0.5 < (ms5 / n5) / (ms1 / n1) < 2.0, (name, ms1 / n1, ms5 / n5)
        # replayed: the timed (host-driven) batches' totals scaled by batches;
        # they launch speculative forward levels up to the deepest batch seen,
        # so counts and per-launch averages differ while totals agree
        assert nr > 0, name
        assert 0.5 < msr / ms1 < 2.0, (name, ms1, msr)
    for key in got:
        assert np.allclose(got[key][0], got[(0, False)][0], rtol=1e-12, atol=0.0), key
