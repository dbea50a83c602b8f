"""ctypes binding of the C ABI in include/bc.h.

Argument marshalling only: every step of the computation runs in the HIP
library (libbc.so).  The names mirror the C entry points.  PyTorch is used for
device memory (its caching allocator backs the library's allocations) and for
streams; nothing here computes betweenness.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbc.so")

BC_OK = 0
BC_ERR_INVALID_ARG = 1
BC_ERR_INVALID_GRAPH = 2
BC_ERR_NOMEM = 3
BC_ERR_DEVICE = 4
BC_ERR_OVERFLOW = 5
BC_ERR_STATE = 6
BC_ERR_UNSUPPORTED = 7
STATUS_NAMES = {0: "BC_OK", 1: "BC_ERR_INVALID_ARG", 2: "BC_ERR_INVALID_GRAPH", 3: "BC_ERR_NOMEM",
                4: "BC_ERR_DEVICE", 5: "BC_ERR_OVERFLOW", 6: "BC_ERR_STATE", 7: "BC_ERR_UNSUPPORTED"}

BC_MEM_HOST = 0
BC_MEM_DEVICE = 1

BC_FORM_AUTO = 0
BC_FORM_PLAIN_FP64 = 1
BC_FORM_SPARSE = 2
BC_FORM_ALGEBRAIC = 3
BC_FORM_HYBRID = 4
BC_FORM_MANY = 5
FORMS = {"auto": BC_FORM_AUTO, "plain": BC_FORM_PLAIN_FP64, "sparse": BC_FORM_SPARSE,
         "algebraic": BC_FORM_ALGEBRAIC, "hybrid": BC_FORM_HYBRID}

BC_ALL_PAIRS_MAX_N = 32768
BC_ALGEBRAIC_MAX_WEIGHT = 8
BC_ALGEBRAIC_MAX_DEGREE = 65792
BC_SAMPLED_MAX_S = 4096
BC_NOALLOC_SCRATCH_BYTES = 64 << 20
BC_TUNE_DEFAULT = 0
BC_TUNE_MEASURED = 1
BC_TUNE_CACHED = 2

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class bc_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("mem", ctypes.c_int)]


class bc_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class bc_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("form", ctypes.c_int), ("batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("allocator", bc_allocator),
                ("timing", ctypes.c_int32), ("split_degree", ctypes.c_int32),
                ("vertex_order", ctypes.c_int32), ("arena_log2", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("grid", ctypes.c_int32), ("edges", ctypes.c_int32),
                ("host_driven", ctypes.c_int32)]


class bc_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("max_degree", ctypes.c_int32),
                ("weighted", ctypes.c_int32), ("form", ctypes.c_int), ("batch", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("sources_run", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("mfma_density_fwd", ctypes.c_double),
                ("mfma_density_bwd", ctypes.c_double), ("tune_source", ctypes.c_int32),
                ("mfma_planes", ctypes.c_int64), ("mfma_ktiles_run", ctypes.c_int64),
                ("mfma_ktiles_dense", ctypes.c_int64), ("mfma_ktiles_run_fwd", ctypes.c_int64),
                ("mfma_ktiles_dense_fwd", ctypes.c_int64), ("mfma_fwd_rows", ctypes.c_int32)]


# Every symbol include/bc.h declares, with its ctypes signature.
SIGNATURES = {
    "bc_options_init": (None, [ctypes.POINTER(bc_options)]),
    "bc_create": (ctypes.c_int, [ctypes.POINTER(bc_graph), ctypes.POINTER(bc_options), ctypes.POINTER(ctypes.c_void_p)]),
    "bc_create_many": (ctypes.c_int, [ctypes.POINTER(bc_graph), ctypes.c_int32, ctypes.POINTER(bc_options),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "bc_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]),
    "bc_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "bc_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "bc_read_edges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "bc_all_pairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "bc_sampled_distances": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int]),
    "bc_read_sssp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "bc_read_sssp_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "bc_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(bc_info)]),
    "bc_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "bc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "bc_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "bc_destroy": (None, [ctypes.c_void_p]),
}

_lib = None


def load():
    """Load libbc.so; raises RuntimeError when the HIP library is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class BCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(status: int, ctx=None):
    if status != BC_OK:
        msg = load().bc_last_error(ctx)
        raise BCError(status, msg.decode() if msg else "")


# ---- thin wrappers with the C names ------------------------------------------------

def bc_options_init() -> bc_options:
    opt = bc_options()
    load().bc_options_init(ctypes.byref(opt))
    return opt


def bc_create(graph: bc_graph, options: Optional[bc_options]) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = load().bc_create(ctypes.byref(graph), ctypes.byref(options) if options is not None else None,
                          ctypes.byref(ctx))
    _check(st, None)
    return ctx


def bc_create_many(graphs, count: int, options: Optional[bc_options]) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = load().bc_create_many(graphs, count, ctypes.byref(options) if options is not None else None,
                               ctypes.byref(ctx))
    _check(st, None)
    return ctx


def bc_run(ctx, sources_ptr, count: int, mem: int) -> None:
    _check(load().bc_run(ctx, sources_ptr, count, mem), ctx)


def bc_read(ctx, out_ptr, mem: int) -> None:
    _check(load().bc_read(ctx, out_ptr, mem), ctx)


def bc_reset(ctx) -> None:
    _check(load().bc_reset(ctx), ctx)


def bc_read_edges(ctx, out_ptr, mem: int) -> None:
    _check(load().bc_read_edges(ctx, out_ptr, mem), ctx)


def bc_all_pairs(ctx, out_ptr, mem: int) -> None:
    _check(load().bc_all_pairs(ctx, out_ptr, mem), ctx)


def bc_sampled_distances(ctx, sources_ptr, count: int, sample_ptr, nsample: int, limit: int, out_ptr,
                         mem: int) -> None:
    _check(load().bc_sampled_distances(ctx, sources_ptr, count, sample_ptr, nsample, limit, out_ptr, mem), ctx)


def bc_read_sssp(ctx, sources_ptr, count: int, dist_ptr, sigma_ptr, delta_ptr) -> None:
    _check(load().bc_read_sssp(ctx, sources_ptr, count, dist_ptr, sigma_ptr, delta_ptr), ctx)


def bc_read_sssp_noalloc(ctx, sources_ptr, count: int, dist_ptr, sigma_ptr, delta_ptr) -> None:
    _check(load().bc_read_sssp_noalloc(ctx, sources_ptr, count, dist_ptr, sigma_ptr, delta_ptr), ctx)


def bc_get_info(ctx) -> bc_info:
    info = bc_info()
    _check(load().bc_get_info(ctx, ctypes.byref(info)), ctx)
    return info


def bc_get_timing(ctx, kernel: str):
    ms = ctypes.c_double()
    launches = ctypes.c_int64()
    _check(load().bc_get_timing(ctx, kernel.encode(), ctypes.byref(ms), ctypes.byref(launches)), ctx)
    return ms.value, launches.value


def bc_status_string(status: int) -> str:
    return load().bc_status_string(status).decode()


def bc_last_error(ctx=None) -> str:
    return load().bc_last_error(ctx).decode()


def bc_destroy(ctx) -> None:
    load().bc_destroy(ctx)


# ---- convenience object ---------------------------------------------------------------

class _TorchAllocator:
    """Backs library allocations with torch's caching allocator."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(nbytes, stream, user):
            try:
                return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
            except Exception:
                return None

        def _free(ptr, stream, user):
            try:
                self.torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch is already gone
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class BC:
    """A context on one graph.

    >>> ctx = BC(graph, form="sparse")        # graph: object with n, row_ptr, col, weight
    >>> many = BC([g0, g1, g2])               # a list: one context over many small graphs
    >>> ctx.run()                              # every source
    >>> bc = ctx.read()                        # numpy float64[n], ordered pairs
    """

    def __init__(self, graph, form: str = "auto", batch: int = 0, device: int = 0, stream=None,
                 allocator: str = "torch", timing=False, split_degree: int = 0,
                 vertex_order: str = "degree", arena_log2: int = 0, tune_cache: Optional[str] = None,
                 grid: int = 0, edges: bool = False, host_driven: bool = False):
        import torch
        load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the betweenness library needs an MI355X")
        self.torch = torch
        self.device = device
        self.n = int(sum(g.n for g in graph)) if isinstance(graph, (list, tuple)) else int(graph.n)
        self.nnz = (int(sum(np.asarray(g.col).size for g in graph)) if isinstance(graph, (list, tuple))
                    else int(np.asarray(graph.col).size))
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        opt = bc_options_init()
        opt.form = FORMS[form]
        opt.batch = batch
        opt.device = device
        opt.stream = self._stream.cuda_stream
        opt.timing = int(timing)  # False / True / k: events on one launch in k
        opt.split_degree = split_degree
        opt.vertex_order = {"degree": 0, "input": 1}[vertex_order]
        opt.arena_log2 = arena_log2
        self._tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        opt.tune_cache = self._tune_cache
        opt.grid = grid
        opt.edges = 1 if edges else 0
        opt.host_driven = 1 if host_driven else 0
        self._alloc = None
        if allocator == "torch":
            self._alloc = _TorchAllocator(device)
            opt.allocator.alloc = self._alloc.alloc
            opt.allocator.free = self._alloc.free
        self._ctx = None
        graphs = graph if isinstance(graph, (list, tuple)) else [graph]
        keep = []
        arr = (bc_graph * max(len(graphs), 1))()
        for i, gr in enumerate(graphs):
            rp = np.ascontiguousarray(gr.row_ptr, dtype=np.int32)
            col = np.ascontiguousarray(gr.col, dtype=np.int32)
            w = None if gr.weight is None else np.ascontiguousarray(gr.weight, dtype=np.uint32)
            keep.append((rp, col, w))
            arr[i].n = int(gr.n)
            arr[i].nnz = int(col.size)
            arr[i].row_ptr = rp.ctypes.data
            arr[i].col = col.ctypes.data if col.size else None
            arr[i].weight = w.ctypes.data if w is not None and w.size else None
            arr[i].mem = BC_MEM_HOST
        with torch.cuda.device(device):
            if isinstance(graph, (list, tuple)):
                self._ctx = bc_create_many(arr, len(graphs), opt)
            else:
                self._ctx = bc_create(arr[0], opt)

    # -- lifecycle --
    def close(self):
        if self._ctx is not None:
            bc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls --
    def run(self, sources=None) -> None:
        if sources is None:
            bc_run(self._ctx, None, -1, BC_MEM_HOST)
            return
        if hasattr(sources, "is_cuda") and sources.is_cuda:
            s = sources.to(self.torch.int32).contiguous()
            bc_run(self._ctx, s.data_ptr(), s.numel(), BC_MEM_DEVICE)
            return
        s = np.ascontiguousarray(sources, dtype=np.int32)
        bc_run(self._ctx, s.ctypes.data if s.size else None, int(s.size), BC_MEM_HOST)

    def read(self) -> np.ndarray:
        out = np.zeros(max(self.n, 1), dtype=np.float64)
        bc_read(self._ctx, out.ctypes.data, BC_MEM_HOST)
        return out[: self.n]

    def read_edges(self) -> np.ndarray:
        """Edge betweenness per arc of the graph's CSR (contexts made with edges=True)."""
        out = np.zeros(max(self.nnz, 1), dtype=np.float64)
        bc_read_edges(self._ctx, out.ctypes.data, BC_MEM_HOST)
        return out[: self.nnz]

    def all_pairs(self) -> np.ndarray:
        """BC over every ordered pair by Algorithm 2 (Sec. 4.2.1) from all-pairs
        distances and path counts; the running BC is not touched."""
        out = np.zeros(max(self.n, 1), dtype=np.float64)
        bc_all_pairs(self._ctx, out.ctypes.data, BC_MEM_HOST)
        return out[: self.n]

    def sampled_distances(self, sources, sample, limit: int = 0, out=None):
        """Distances from each source by Algorithm 1 (Sec. 4.1.1) with the
        distinguished set sources + sample and the given search limit (0 =
        ceil(sqrt(n))): int32 [len(sources), n], -1 where no walk was found.
        With `out` (an int32 device tensor of that shape) the rows are written
        there and `out` is returned; otherwise a host array."""
        s = np.ascontiguousarray(sources, dtype=np.int32)
        x = np.ascontiguousarray(sample, dtype=np.int32)
        sp = s.ctypes.data if s.size else None
        xp = x.ctypes.data if x.size else None
        if out is not None:
            if (not out.is_cuda or out.dtype != self.torch.int32 or not out.is_contiguous()
                    or tuple(out.shape) != (s.size, self.n)):
                raise ValueError("out must be a contiguous int32 device tensor of shape (len(sources), n)")
            bc_sampled_distances(self._ctx, sp, int(s.size), xp, int(x.size), int(limit), out.data_ptr(),
                                 BC_MEM_DEVICE)
            return out
        res = np.zeros((max(s.size, 1), max(self.n, 1)), np.int32)
        bc_sampled_distances(self._ctx, sp, int(s.size), xp, int(x.size), int(limit), res.ctypes.data, BC_MEM_HOST)
        return res[: s.size, : self.n]

    def read_device(self):
        out = self.torch.empty(max(self.n, 1), dtype=self.torch.float64, device=f"cuda:{self.device}")
        bc_read(self._ctx, out.data_ptr(), BC_MEM_DEVICE)
        return out[: self.n]

    def reset(self) -> None:
        bc_reset(self._ctx)

    def sssp(self, sources):
        """(dist int32[k,n], sigma uint64[k,n], delta float64[k,n]) for k sources."""
        s = np.ascontiguousarray(sources, dtype=np.int32)
        k = int(s.size)
        dist = np.zeros((k, max(self.n, 1)), np.int32)
        sigma = np.zeros((k, max(self.n, 1)), np.uint64)
        delta = np.zeros((k, max(self.n, 1)), np.float64)
        bc_read_sssp(self._ctx, s.ctypes.data, k, dist.ctypes.data, sigma.ctypes.data, delta.ctypes.data)
        return dist[:, : self.n], sigma[:, : self.n], delta[:, : self.n]

    def sssp_noalloc(self, sources, dist=None, sigma=None, delta=None):
        """bc_read_sssp_noalloc into caller device tensors of shape (k, n):
        dist int32, sigma int64 (the uint64 counts' bits), delta float64; any
        may be None.  Allocates nothing."""
        s = np.ascontiguousarray(sources, dtype=np.int32)
        k = int(s.size)
        want = {"dist": (dist, self.torch.int32), "sigma": (sigma, self.torch.int64),
                "delta": (delta, self.torch.float64)}
        for name, (t, dt) in want.items():
            if t is not None and (not t.is_cuda or t.dtype != dt or not t.is_contiguous()
                                  or tuple(t.shape) != (k, self.n)):
                raise ValueError(f"{name} must be a contiguous {dt} device tensor of shape (len(sources), n)")
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        bc_read_sssp_noalloc(self._ctx, s.ctypes.data if k else None, k, ptr(dist), ptr(sigma), ptr(delta))

    def info(self) -> bc_info:
        return bc_get_info(self._ctx)

    def timing(self, kernel: str):
        return bc_get_timing(self._ctx, kernel)

    @property
    def handle(self):
        return self._ctx
