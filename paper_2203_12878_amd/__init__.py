"""MI355X-native data-race-freedom checking of memory access protocols.

Submodules are imported lazily: `workloads` needs only numpy; `drf` loads
the in-tree gfx950 library libdrf.so and PyTorch (for device memory and
streams).
"""
__all__ = ["drf", "workloads", "server"]
