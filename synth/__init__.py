"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

Nothing in this package computes any part of the method; it only builds
graphs (``synth.graphs``), random iterates (``synth.arrays``) and the named
workload recipes (``synth.workloads``).
"""
from . import graphs, arrays, workloads  # noqa: F401
