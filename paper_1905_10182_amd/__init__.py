"""MI355X-native D3Q27 central-moment lattice Boltzmann method with Hermite
external forcing (De Rosis, Huang & Coreixas, PRE 2019, arXiv:1905.10182).

The solver runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/cmlbm.h (libcmlbm.so); ``Lattice`` is its thin Python binding.
"""
from .cmlbm import CmlbmError, Lattice, load_library, make_params, required_bytes  # noqa: F401

__all__ = ["Lattice", "CmlbmError", "load_library", "make_params", "required_bytes"]
