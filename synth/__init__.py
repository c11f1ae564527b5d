"""Seeded synthetic inputs (scenes, cameras, ray batches, workloads).

Input generation only: this package holds none of the renderer's
arithmetic and serves the oracle, the tests, the smoke check and the
benchmark alike.
"""
from . import cameras, scenes, workloads  # noqa: F401
