"""The allocation-free readout, bc_read_sssp_noalloc: the per-source
distances, path counts and dependencies of bc_read_sssp (Sec. 1.1), written
into caller device memory with no allocation, its staging held in the
library's fixed per-GPU array.  Checked against bc_read_sssp on the same
context: distances and counts bit-exact, dependencies to the form's
tolerance; two calls in a row, the second smaller; torch's allocator and the
context's own device memory untouched by the call."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def noalloc(ctx, src):
    import torch
    k, n = len(src), ctx.n
    d = torch.full((k, n), -7, dtype=torch.int32, device="cuda:0")
    sg = torch.full((k, n), -7, dtype=torch.int64, device="cuda:0")
    dl = torch.full((k, n), -7.0, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    allocs = torch.cuda.memory_stats()["allocation.all.allocated"]
    held = ctx.info().device_bytes
    ctx.sssp_noalloc(src, d, sg, dl)
    assert torch.cuda.memory_stats()["allocation.all.allocated"] == allocs, "the call allocated through torch"
    assert ctx.info().device_bytes == held, "the context grew during the call"
    return d.cpu().numpy(), sg.cpu().numpy().view(np.uint64), dl.cpu().numpy()


def cases():
    er = gg.er_plus_tree(700, 6.0, 2201)
    return {
        "plain": (er, dict(form="plain"), 1e-12),
        "sparse": (er, dict(form="sparse", batch=256), 1e-5),
        "hybrid": (er, dict(form="hybrid", batch=256), 1e-5),
        "algebraic": (er, dict(form="algebraic", batch=256), 1e-5),
        "weighted": (gg.with_uniform_weights(er, 2202, 1, 30), dict(form="plain"), 1e-12),
        "walgebraic": (gg.with_uniform_weights(er, 2203, 1, 4), dict(form="algebraic", batch=256), 1e-5),
        "many": ([gg.watts_strogatz(300, 6, 0.1, 7), gg.path(40), gg.er_plus_tree(200, 5.0, 8)], dict(), 1e-5),
    }


@pytest.mark.parametrize("name", ["plain", "sparse", "hybrid", "algebraic", "weighted", "walgebraic", "many"])
def test_noalloc_matches_read_sssp_twice(gpu_lib, name):
    g, kw, tol = cases()[name]
    print(f"[gpu-case] noalloc {name}", flush=True)
    with gpu_lib.BC(g, **kw) as ctx:
        n = ctx.n
        limit = 64 if isinstance(g, list) else 200
        first = gg.sample_sources(n, limit, 2204)
        second = first[::7][:9]  # a smaller second call
        ctx.run()  # the context has run work before (replays settled by the call)
        for src in (first, second):
            got = noalloc(ctx, src)
            want = ctx.sssp(src)
            assert np.array_equal(got[0], want[0]), f"{name}: distances"
            assert np.array_equal(got[1], want[1]), f"{name}: path counts"
            assert rel_err(got[2], want[2]) <= tol, f"{name}: dependencies"


def test_noalloc_limits(gpu_lib):
    """A request above the fixed staging gives BC_ERR_UNSUPPORTED; one that
    would need more frontier levels than the context holds gives
    BC_ERR_NOMEM, and works once an ordinary call has made the room."""
    import torch
    big = gg.er_plus_tree(20000, 6.0, 2205)
    with gpu_lib.BC(big, form="sparse", batch=256) as ctx:
        src = gg.sample_sources(big.n, 200, 2206)  # 200 * 20000 cells of 20 B: above 64 MiB
        d = torch.empty((200, big.n), dtype=torch.int32, device="cuda:0")
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.sssp_noalloc(src, dist=d)
        assert e.value.status == gpu_lib.BC_ERR_UNSUPPORTED
        small = src[:100]
        d2 = torch.empty((100, big.n), dtype=torch.int32, device="cuda:0")
        ctx.sssp_noalloc(small, dist=d2)
        assert np.array_equal(d2.cpu().numpy(), ctx.sssp(small)[0])
    deep = gg.grid(20, 20)  # 39 levels from a corner: more than a new context holds
    with gpu_lib.BC(deep, form="sparse", batch=64) as ctx:
        src = np.array([0, 399, 210], np.int32)
        d = torch.empty((3, deep.n), dtype=torch.int32, device="cuda:0")
        with pytest.raises(gpu_lib.BCError) as e:
            ctx.sssp_noalloc(src, dist=d)
        assert e.value.status == gpu_lib.BC_ERR_NOMEM
        want = ctx.sssp(src)[0]  # grows the level storage
        ctx.sssp_noalloc(src, dist=d)
        assert np.array_equal(d.cpu().numpy(), want)
