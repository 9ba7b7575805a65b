"""MI355X-native pseudospectral Navier-Stokes / MHD hot path.

The compute path is the HIP library ``libps.so`` (C ABI declared in
``include/ps.h``); :mod:`paper_1003_4322_amd.binding` is its thin ctypes
binding.  :mod:`paper_1003_4322_amd.synth` generates seeded synthetic inputs.
"""
__all__ = ["binding", "synth"]
