"""Plain FP64 CPU oracle for multilevel compact U(1) lattice gauge theory.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product library never
imports or links anything from here.
"""
from .oracle import (OracleLattice, atan2, bessel_ratio, build_oracle, connected_profile,  # noqa: F401
                     max_threads, philox4x64_10, set_threads, sincos)
