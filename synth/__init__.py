"""Seeded synthetic inputs shared by tests, benchmark and both sides of parity checks."""
from .graphs import *  # noqa: F401,F403
from .graphs import BASE_SEED, Graph, GraphBatch  # noqa: F401
