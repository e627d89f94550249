"""MI355X (gfx950) engine for conjunctive ML-UDF queries with adaptive routing.

The compute path is libhydro.so (hand-written HIP, C ABI in include/hydro.h); ``hydro`` is its
ctypes binding.
"""
from . import hydro  # noqa: F401
