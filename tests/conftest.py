import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library on a machine with an MI355X; fails loudly when it is not built."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_0809_1906_amd as bcgpu
    import paper_0809_1906_amd.binding  # noqa: F401
    bcgpu.load()  # raises if the shared library is missing
    return bcgpu


def oracle_threads() -> int:
    """Host threads for oracle runs: the CPUs this process may use, at most 16
    (one GPU's share of a GPU host's cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


_ORACLE_CACHE = {}


@pytest.fixture(scope="session")
def oracle_all_sources():
    """oracle_all_sources(name, graph) -> the oracle's all-source BC of a
    benchmark graph, computed once per session and shared between tests."""
    import oracle

    def get(name, g):
        if name not in _ORACLE_CACHE:
            print(f"[gpu-case] oracle all sources {name} n={g.n} m={g.m}", flush=True)
            _ORACLE_CACHE[name] = oracle.bc(g, threads=oracle_threads())
        return _ORACLE_CACHE[name]

    return get
