"""MI355X-native ternary wetting lattice Boltzmann solver (Liang et al.,
arXiv:1710.09534): a C-ABI HIP library for gfx950 plus a thin ctypes binding.

``paper_1710_09534_amd.tlb`` loads the HIP library (it raises if the library
is missing -- there is no CPU fallback); ``paper_1710_09534_amd.workloads``
builds seeded inputs and does not touch the GPU.
"""
__version__ = "0.1.0"
