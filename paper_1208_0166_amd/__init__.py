"""u1ml: Luscher-Weisz multilevel Monte Carlo for compact U(1) lattice gauge
theory in 3+1 dimensions on AMD Instinct MI355X (gfx950).

The method runs in the HIP library ``lib/libu1ml.so`` behind the C ABI of
``include/u1ml.h``; :mod:`paper_1208_0166_amd.u1ml` is its Python binding.
"""
from . import u1ml  # noqa: F401
