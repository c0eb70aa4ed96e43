"""Seeded synthetic inputs (maps, values, series) shared by the oracle
tests, the GPU tests and the benchmark.  No cartogram arithmetic here."""
from .maps import *  # noqa: F401,F403
