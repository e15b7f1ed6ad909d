"""MI355X (gfx950) library for the linear Sternheimer solves of the SternheimerGW method.

The compute path is libsgw.so (hand-written HIP kernels behind a C ABI declared
in include/sgw.h); ``sgw`` is its thin ctypes binding and ``workload`` moves a
problem's arrays onto the device through it.
"""
from . import sgw  # noqa: F401
