"""Batched strong-lens forward model and likelihood on AMD MI355X (gfx950).

The compute path is the HIP library liblens.so (C ABI: include/lens_api.h);
``lens`` is its ctypes binding.  ``synth`` draws seeded synthetic inputs.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "lens"]
