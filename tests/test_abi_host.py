"""The C-ABI library on the host: it loads, exports every declared symbol,
and rejects invalid input before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import graphgen as gg
import paper_0809_1906_amd as bcgpu
from paper_0809_1906_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = bcgpu.load()
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), f"{name} declared in bc.h but not exported"
    assert set(names) == set(B.SIGNATURES), "binding signatures out of step with bc.h"


def test_status_strings():
    for code, name in B.STATUS_NAMES.items():
        assert bcgpu.bc_status_string(code).startswith(name)


def test_options_defaults():
    opt = bcgpu.bc_options_init()
    assert opt.struct_size == ctypes.sizeof(B.bc_options)
    assert opt.form == B.BC_FORM_AUTO and opt.batch == 0 and opt.device == -1
    assert opt.tune_cache is None


def test_struct_layouts_match_header(tmp_path):
    """sizeof and every field offset of the C structs, from a C program
    compiled against bc.h, equal the ctypes mirrors."""
    structs = {"bc_options": B.bc_options, "bc_info": B.bc_info, "bc_graph": B.bc_graph,
               "bc_allocator": B.bc_allocator}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bc.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, value = line.split()
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(value) == want, f"{name}.{field}: C {value}, ctypes {want}"


def _graph_struct(n, rp, col, w=None):
    rp = np.ascontiguousarray(rp, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    g = B.bc_graph()
    g.n = n
    g.nnz = int(col.size)
    g.row_ptr = rp.ctypes.data
    g.col = col.ctypes.data if col.size else None
    if w is not None:
        w = np.ascontiguousarray(w, np.uint32)
        g.weight = w.ctypes.data
    g.mem = B.BC_MEM_HOST
    return g, (rp, col, w)


def _create_status(n, rp, col, w=None, opt=None):
    g, keep = _graph_struct(n, rp, col, w)
    ctx = ctypes.c_void_p()
    st = bcgpu.load().bc_create(ctypes.byref(g), ctypes.byref(opt) if opt is not None else None, ctypes.byref(ctx))
    assert ctx.value is None, "a failed create must leave no context"
    return st, bcgpu.bc_last_error(None)


@pytest.mark.parametrize("case,n,rp,col,w", [
    ("asymmetric", 3, [0, 1, 1, 1], [1], None),
    ("self-loop", 2, [0, 2, 3], [0, 1, 0], None),
    ("duplicate", 2, [0, 2, 4], [1, 1, 0, 0], None),
    ("unsorted", 3, [0, 2, 3, 4], [2, 1, 0, 0], None),
    ("out-of-range", 2, [0, 1, 2], [5, 0], None),
    ("row_ptr[0]", 2, [1, 1, 2], [1, 0], None),
    ("row_ptr[n] != nnz", 2, [0, 1, 1], [1, 0], None),
    ("decreasing", 3, [0, 2, 1, 2], [1, 2], None),
    ("zero weight", 2, [0, 1, 2], [1, 0], [0, 0]),
    ("asymmetric weight", 2, [0, 1, 2], [1, 0], [3, 4]),
])
def test_invalid_graphs_rejected_on_host(case, n, rp, col, w):
    st, msg = _create_status(n, rp, col, w)
    assert st == B.BC_ERR_INVALID_GRAPH, (case, st, msg)
    assert msg


def test_weight_times_diameter_bound():
    g = gg.path(3)
    st, msg = _create_status(g.n, g.row_ptr, g.col, np.full(g.nnz, 2 ** 30, np.uint32))
    assert st == B.BC_ERR_INVALID_GRAPH and "2^31" in msg


def test_invalid_arguments():
    lib = bcgpu.load()
    ctx = ctypes.c_void_p()
    assert lib.bc_create(None, None, ctypes.byref(ctx)) == B.BC_ERR_INVALID_ARG
    g, keep = _graph_struct(2, [0, 1, 2], [1, 0])
    assert lib.bc_create(ctypes.byref(g), None, None) == B.BC_ERR_INVALID_ARG
    opt = bcgpu.bc_options_init()
    opt.batch = 100  # not a multiple of 64
    assert lib.bc_create(ctypes.byref(g), ctypes.byref(opt), ctypes.byref(ctx)) == B.BC_ERR_INVALID_ARG
    opt = bcgpu.bc_options_init()
    opt.struct_size = 3
    assert lib.bc_create(ctypes.byref(g), ctypes.byref(opt), ctypes.byref(ctx)) == B.BC_ERR_INVALID_ARG
    opt = bcgpu.bc_options_init()
    opt.form = 42
    assert lib.bc_create(ctypes.byref(g), ctypes.byref(opt), ctypes.byref(ctx)) == B.BC_ERR_INVALID_ARG
    opt = bcgpu.bc_options_init()
    opt.timing = -1  # timing is 0 (off) or one launch in k >= 1
    assert lib.bc_create(ctypes.byref(g), ctypes.byref(opt), ctypes.byref(ctx)) == B.BC_ERR_INVALID_ARG
    # calls on a NULL context
    assert lib.bc_run(None, None, -1, 0) == B.BC_ERR_INVALID_ARG
    assert lib.bc_read(None, None, 0) == B.BC_ERR_INVALID_ARG
    assert lib.bc_reset(None) == B.BC_ERR_INVALID_ARG
    assert lib.bc_all_pairs(None, None, 0) == B.BC_ERR_INVALID_ARG
    assert lib.bc_sampled_distances(None, None, 0, None, 0, 0, None, 0) == B.BC_ERR_INVALID_ARG
    lib.bc_destroy(None)


def test_batched_forms_refuse_weights_before_device_work():
    g = gg.with_uniform_weights(gg.path(5), 1, 1, 9)
    for form in (B.BC_FORM_SPARSE, B.BC_FORM_HYBRID):
        opt = bcgpu.bc_options_init()
        opt.form = form
        st, msg = _create_status(g.n, g.row_ptr, g.col, g.weight, opt)
        assert st == B.BC_ERR_UNSUPPORTED and "weighted" in msg


def test_algebraic_form_refuses_weights_above_its_classes():
    """The algebraic form takes one product class per weight, up to
    BC_ALGEBRAIC_MAX_WEIGHT; a heavier edge is refused before device work."""
    assert B.BC_ALGEBRAIC_MAX_WEIGHT == 8
    g = gg.with_constant_weight(gg.path(5), B.BC_ALGEBRAIC_MAX_WEIGHT + 1)
    opt = bcgpu.bc_options_init()
    opt.form = B.BC_FORM_ALGEBRAIC
    st, msg = _create_status(g.n, g.row_ptr, g.col, g.weight, opt)
    assert st == B.BC_ERR_UNSUPPORTED and "BC_ALGEBRAIC_MAX_WEIGHT" in msg


def test_edges_refused_where_not_computed():
    """Edge betweenness needs per-arc terms: the algebraic form (row sums
    only) and many-graph contexts refuse it before any device work."""
    lib = bcgpu.load()
    g = gg.path(5)
    opt = bcgpu.bc_options_init()
    opt.form = B.BC_FORM_ALGEBRAIC
    opt.edges = 1
    st, msg = _create_status(g.n, g.row_ptr, g.col, None, opt)
    assert st == B.BC_ERR_UNSUPPORTED and "edge" in msg
    arr = (B.bc_graph * 1)()
    gs, keep = _graph_struct(g.n, g.row_ptr, g.col)
    arr[0] = gs
    opt = bcgpu.bc_options_init()
    opt.edges = 1
    ctx = ctypes.c_void_p()
    assert lib.bc_create_many(arr, 1, ctypes.byref(opt), ctypes.byref(ctx)) == B.BC_ERR_UNSUPPORTED


def test_many_graphs_host_checks():
    lib = bcgpu.load()
    big = gg.path(5000)
    small = gg.path(10)
    weighted = gg.with_uniform_weights(gg.path(6), 3, 1, 5)
    for graphs, want in (([small, big], B.BC_ERR_UNSUPPORTED), ([small, weighted], B.BC_ERR_UNSUPPORTED)):
        arr = (B.bc_graph * len(graphs))()
        keep = []
        for i, gr in enumerate(graphs):
            g, k = _graph_struct(gr.n, gr.row_ptr, gr.col, gr.weight)
            keep.append(k)
            arr[i] = g
        ctx = ctypes.c_void_p()
        st = lib.bc_create_many(arr, len(graphs), None, ctypes.byref(ctx))
        assert st == want and ctx.value is None
    # an invalid member graph is reported with its index
    arr = (B.bc_graph * 2)()
    g0, k0 = _graph_struct(small.n, small.row_ptr, small.col)
    g1, k1 = _graph_struct(3, [0, 1, 1, 1], [1])
    arr[0], arr[1] = g0, g1
    ctx = ctypes.c_void_p()
    assert lib.bc_create_many(arr, 2, None, ctypes.byref(ctx)) == B.BC_ERR_INVALID_GRAPH
    assert "graph 1" in bcgpu.bc_last_error(None)
