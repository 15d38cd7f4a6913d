"""MI355X-native FR x conservative-DVM Boltzmann-BGK hot path (libfrdvm).

The compute path is the HIP library ``libfrdvm.so`` (C ABI in
``include/fr_dvm.h``); ``frdvm`` is its ctypes binding.
"""
from .frdvm import FrDvm, FrDvmError, lib  # noqa: F401
