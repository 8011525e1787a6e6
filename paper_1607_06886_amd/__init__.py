"""MI355X (gfx950) implementation of PUMP's exploration hot path.

The planner lives in the HIP library libpump.so (C ABI in include/pump.h);
``paper_1607_06886_amd._lib`` is its thin ctypes binding and
``paper_1607_06886_amd.scenes`` draws seeded synthetic inputs.
"""

__all__ = ["scenes"]
