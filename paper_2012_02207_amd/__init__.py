"""MI355X-native collisional FMM force pass (gfx950 HIP kernels behind a C ABI).

``forces`` / ``FMM`` live in :mod:`paper_2012_02207_amd.fmm` and load the HIP
library on first use; :mod:`paper_2012_02207_amd.workloads` holds the seeded
input generators.
"""
import importlib

__all__ = ["forces", "FMM", "FmmError"]


def __getattr__(name):
    if name in ("forces", "FMM", "FmmError"):
        return getattr(importlib.import_module(".fmm", __name__), name)
    raise AttributeError(name)
