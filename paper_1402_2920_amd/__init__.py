"""MI355X (gfx950) implementation of the consistent two-phase lattice
Boltzmann step of Zelko & Duenweg (arXiv:1402.2920).

The compute path is the HIP library ``liblb2p.so`` (C ABI in
``include/lb2p.h``); ``lb2p`` is its ctypes binding.
"""
from . import lb2p  # noqa: F401

__all__ = ["lb2p"]
