"""Seeded synthetic inputs (lattices, symmetry groups, term tables, vectors).

The only module that both the GPU path's tests/benchmarks and the oracle
use.  It draws numbers and describes inputs; it computes nothing of the
method itself.
"""
from . import configs, lattice, rng, terms  # noqa: F401
