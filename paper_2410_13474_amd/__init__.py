"""MI355X-native NU-FDS reconstruction (libnufds) and its Python binding.

The reconstruction runs in the HIP kernels of libnufds.so (built in-tree by
``paper_2410_13474_amd.build_lib``); :mod:`paper_2410_13474_amd.nufds` only
marshals arguments to its C ABI.
"""
from . import nufds  # noqa: F401
from .nufds import Plan, plan_geometry, synth_hologram, NufdsError  # noqa: F401

__all__ = ["nufds", "Plan", "plan_geometry", "synth_hologram", "NufdsError"]
