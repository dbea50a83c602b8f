"""Kernel timing with HIP events: every launch (timing = 1) or every launch of
one source batch in k (timing = k).  Sampling changes which launches carry
events, never the launch count or the results."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def test_batch_sampled_timing(gpu_lib):
    g = gg.rmat(12, 16, 7)
    say("timing", g.n, g.m)
    got = {}
    for k in (0, 1, 5):
        with gpu_lib.BC(g, form="sparse", batch=64, timing=k) as ctx:
            ctx.run()
            bc = ctx.read()
            got[k] = (bc, {name: ctx.timing(name) for name in ("fwd_pull", "bwd_pull", "batch_init")})
    assert all(v == (0.0, 0) for v in got[0][1].values())
    for name in ("fwd_pull", "bwd_pull", "batch_init"):
        ms1, n1 = got[1][1][name]
        ms5, n5 = got[5][1][name]
        assert n1 == n5 > 0, name
        assert ms1 > 0 and ms5 > 0, name
        # the sampled total is the timed batches' average scaled to every launch
        assert 0.5 < (ms5 / n5) / (ms1 / n1) < 2.0, (name, ms1 / n1, ms5 / n5)
    for k in (1, 5):
        assert np.allclose(got[k][0], got[0][0], rtol=1e-12, atol=0.0)
