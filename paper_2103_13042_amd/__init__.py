"""SpAMM (sparse approximate matrix multiplication) for AMD Instinct MI355X.

The kernels live in libspamm.so (HIP, gfx950); ``binding`` is its ctypes
interface.  Importing the package does not load the library, so the seeded
input generators (``inputs``) work on hosts without it; any use of the GPU
entry points loads it and fails loudly if it is missing.
"""

from __future__ import annotations

__all__ = [
    "bdim", "levels", "pyramid_size", "leaf_supported", "workspace_bytes", "workspace",
    "norms", "pyramid", "pyramid_levels", "plan", "plan_buffers", "prepare", "execute", "schedule",
    "execute_scheduled", "multiply",
    "search_valid_ratio", "SpammError",
]


def __getattr__(name):
    if name in __all__ or name in ("binding", "library"):
        import importlib

        binding = importlib.import_module(".binding", __name__)
        return binding if name == "binding" else getattr(binding, name)
    raise AttributeError(name)
