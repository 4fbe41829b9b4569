"""Seeded synthetic inputs (permittivity maps and sources) shared by the oracle
tests, the GPU tests and the benchmark.  Holds no solver arithmetic."""
from . import geometry, sources, configs  # noqa: F401
