"""Seeded synthetic inputs (graphs, source samples) shared by the oracle side
and the GPU side.  Holds no betweenness arithmetic."""
from .rng import BASE_SEED, Stream, mix64, substream  # noqa: F401
from .graphs import *  # noqa: F401,F403
from .graphs import Graph, from_edges  # noqa: F401
