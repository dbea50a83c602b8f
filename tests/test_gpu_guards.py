"""Guards of the boundary on the GPU: the degree limit of the algebraic form,
allocation failure at every allocation a context makes, and calls refused
while the context's stream is being captured into a HIP graph.

- Degree: an output of a forward product sums at most deg 7-bit limb terms
  of at most 127 in int32, and its FP32 copy is exact while 127 * deg < 2^24;
  the limit is 65792 (exact path counts, Sec. 1.1, carried through the
  products of Sec. 3.1).  The star K_{1,65793} has one
  degree above that: the algebraic form refuses it, the hybrid form runs it by
  pulls, and BC equals the star's closed form ((n-1)(n-2) at the centre over
  ordered pairs, 0 at the leaves).
- Allocation: an allocator callback that returns NULL at the k-th request
  makes bc_create return BC_ERR_NOMEM with every earlier allocation handed
  back, for every k up to the number a successful create makes.
- Capture: every call returns BC_ERR_STATE and records nothing.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_0809_1906_amd import binding as B

pytestmark = pytest.mark.gpu


def rel_err(x, y):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1.0)))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def test_degree_above_limit_algebraic_refused_hybrid_pulls(gpu_lib):
    n = B.BC_ALGEBRAIC_MAX_DEGREE + 2  # centre degree = limit + 1
    g = gg.star(n)
    say("degree gate", n)
    with pytest.raises(B.BCError) as ei:
        gpu_lib.BC(g, form="algebraic", batch=256)
    assert ei.value.status == B.BC_ERR_UNSUPPORTED
    assert "BC_ALGEBRAIC_MAX_DEGREE" in str(ei.value)
    with gpu_lib.BC(g, form="hybrid", batch=256) as ctx:
        info = ctx.info()
        assert info.mfma_density_fwd > 1.0 and info.mfma_density_bwd > 1.0, "no level may go by products"
        ctx.run()
        got = ctx.read()
        assert ctx.info().mfma_planes == 0
    want = np.zeros(n)
    want[0] = float(n - 1) * float(n - 2)
    assert rel_err(got, want) <= 1e-5
    # the oracle agrees on a sample of sources (the centre and leaves)
    src = np.array([0, 1, 2, n // 2, n - 1], np.int32)
    with gpu_lib.BC(g, form="hybrid", batch=256) as ctx:
        ctx.run(src)
        assert rel_err(ctx.read(), oracle.bc(g, src)) <= 1e-5


def test_degree_at_limit_algebraic_exact(gpu_lib):
    """The largest degree the algebraic form takes: the star K_{1,65792}.
    From a leaf, level 2 holds the other leaves, each with one path through
    the centre; counts and distances bit-exact, BC at the closed form."""
    n = B.BC_ALGEBRAIC_MAX_DEGREE + 1
    g = gg.star(n)
    say("degree limit", n)
    with gpu_lib.BC(g, form="algebraic", batch=256) as ctx:
        dist, sigma, _ = ctx.sssp(np.array([0, 1, n - 1], np.int32))
        ctx.run(np.arange(0, n, 97, dtype=np.int32))
        got = ctx.read()
    for i, s in enumerate([0, 1, n - 1]):
        d, sg, _ = oracle.sssp_u64(g, s)
        assert np.array_equal(dist[i], d) and np.array_equal(sigma[i], sg)
    assert rel_err(got, oracle.bc(g, np.arange(0, n, 97, dtype=np.int32), threads=16)) <= 1e-5


class CountingAllocator:
    """Device memory from torch's caching allocator; request number `fail_at`
    (0-based) returns NULL.  Records what is live."""

    def __init__(self, fail_at=-1):
        import torch
        self.torch = torch
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}

        def _alloc(nbytes, stream, user):
            k = self.calls
            self.calls += 1
            if k == self.fail_at:
                return None
            p = self.torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or 0)
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, stream, user):
            assert ptr in self.live, "freed a pointer the allocator did not hand out"
            del self.live[ptr]
            self.torch.cuda.caching_allocator_delete(ptr)

        self.alloc = B.ALLOC_FN(_alloc)
        self.free = B.FREE_FN(_free)


def create_raw(g, form, batch, alloc, stream, edges=False):
    opt = B.bc_options_init()
    opt.form = B.FORMS[form]
    opt.batch = batch
    opt.device = 0
    opt.stream = stream.cuda_stream
    opt.edges = 1 if edges else 0
    opt.allocator.alloc = alloc.alloc
    opt.allocator.free = alloc.free
    many = isinstance(g, (list, tuple))
    graphs = list(g) if many else [g]
    arr = (B.bc_graph * len(graphs))()
    keep = []
    for i, x in enumerate(graphs):
        rp = np.ascontiguousarray(x.row_ptr, np.int32)
        col = np.ascontiguousarray(x.col, np.int32)
        w = None if x.weight is None else np.ascontiguousarray(x.weight, np.uint32)
        keep.append((rp, col, w))
        arr[i].n, arr[i].nnz = x.n, int(col.size)
        arr[i].row_ptr, arr[i].col = rp.ctypes.data, col.ctypes.data
        arr[i].weight = w.ctypes.data if w is not None else None
        arr[i].mem = B.BC_MEM_HOST
    ctx = ctypes.c_void_p()
    if many:
        opt.form = 0
        st = B.load().bc_create_many(arr, len(graphs), ctypes.byref(opt), ctypes.byref(ctx))
    else:
        st = B.load().bc_create(ctypes.byref(arr[0]), ctypes.byref(opt), ctypes.byref(ctx))
    return st, ctx


CASES = [("plain", 0, None), ("sparse", 256, None), ("sparse", 64, "edges"), ("algebraic", 256, None),
         ("hybrid", 256, None), ("plain", 0, "weighted"), ("auto", 0, "many")]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_nomem_at_every_allocation_leaves_nothing(gpu_lib, case):
    import torch
    form, batch, extra = CASES[case]
    g = gg.er_plus_tree(500, 6.0, 2102)
    if extra == "weighted":
        g = gg.with_uniform_weights(g, 2103, 1, 9)
    elif extra == "many":
        g = [g, gg.path(9), gg.watts_strogatz(120, 6, 0.1, 5)]
    stream = torch.cuda.current_stream(0)
    ok = CountingAllocator()
    st, ctx = create_raw(g, form, batch, ok, stream, edges=extra == "edges")
    assert st == B.BC_OK
    total = ok.calls
    assert total >= 5
    B.load().bc_destroy(ctx)
    assert not ok.live, "destroy must hand back every allocation"
    say("nomem", form, batch, extra, "allocations", total)
    for k in range(total):
        a = CountingAllocator(fail_at=k)
        st, ctx = create_raw(g, form, batch, a, stream, edges=extra == "edges")
        assert st == B.BC_ERR_NOMEM, f"allocation {k} of {total}: status {st}"
        assert ctx.value is None
        assert not a.live, f"allocation {k} of {total}: {len(a.live)} allocations left behind"
        assert B.bc_last_error(None)


def test_nomem_in_run_then_recovers(gpu_lib):
    """bc_run grows its source staging on demand; a failed allocation there
    returns BC_ERR_NOMEM, adds nothing to BC, and the next call succeeds."""
    import torch
    g = gg.er_plus_tree(400, 6.0, 2104)
    a = CountingAllocator()
    st, ctx = create_raw(g, "sparse", 128, a, torch.cuda.current_stream(0))
    assert st == B.BC_OK
    lib = B.load()
    try:
        a.fail_at = a.calls  # the next request: staging for 300 explicit sources
        src = np.arange(0, 400, dtype=np.int32)[:300]
        assert lib.bc_run(ctx, src.ctypes.data, 300, B.BC_MEM_HOST) == B.BC_ERR_NOMEM
        out = np.zeros(g.n)
        assert lib.bc_read(ctx, out.ctypes.data, B.BC_MEM_HOST) == B.BC_OK
        assert not np.any(out), "a failed run must add nothing"
        assert lib.bc_run(ctx, src.ctypes.data, 300, B.BC_MEM_HOST) == B.BC_OK
        assert lib.bc_read(ctx, out.ctypes.data, B.BC_MEM_HOST) == B.BC_OK
        assert rel_err(out, oracle.bc(g, src)) <= 1e-5
    finally:
        lib.bc_destroy(ctx)
    assert not a.live


@pytest.mark.parametrize("form", ["plain", "sparse", "hybrid"])
def test_calls_refused_under_stream_capture(gpu_lib, form):
    """While the context's stream is being captured into a HIP graph, every
    call that could synchronise or launch returns BC_ERR_STATE; after the
    capture ends the context works and its BC holds only what ran outside."""
    import torch
    g = gg.er_plus_tree(300, 5.0, 2105)
    s = torch.cuda.Stream(device=0)
    ctx = gpu_lib.BC(g, form=form, stream=s)
    try:
        x = torch.zeros(16, device="cuda:0")
        graph = torch.cuda.CUDAGraph()
        codes = []
        lib = B.load()
        out = np.zeros(g.n)
        with torch.cuda.graph(graph, stream=s, capture_error_mode="relaxed"):
            x.add_(1.0)
            codes.append(lib.bc_run(ctx.handle, None, -1, B.BC_MEM_HOST))
            codes.append(lib.bc_read(ctx.handle, out.ctypes.data, B.BC_MEM_HOST))
            codes.append(lib.bc_reset(ctx.handle))
        assert codes == [B.BC_ERR_STATE] * 3, codes
        assert "captured" in B.bc_last_error(ctx.handle)
        graph.replay()
        torch.cuda.synchronize()
        assert float(x[0]) == 1.0
        ctx.run()
        assert rel_err(ctx.read(), oracle.bc(g)) <= (1e-12 if form == "plain" else 1e-5)
    finally:
        ctx.close()
