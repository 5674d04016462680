"""FP64 CPU oracle of the ternary phase-field lattice Boltzmann step with the
ternary wetting boundary scheme (Liang et al., arXiv:1710.09534).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1710_09534_amd``) and the GPU library never
falls back to it.

The arithmetic lives in ``tlb_oracle.c`` (D2Q9) and ``tlb3d_oracle.c``
(the D3Q19 version), plain C built with ``-O2 -ffp-contract=off``; this
module only marshals numpy arrays through ctypes.
"""
from .oracle import (  # noqa: F401
    FIELDS,
    FIELDS3,
    STAGES,
    Oracle,
    Oracle3D,
    build,
    chem_potential,
    cos12,
    equilibria,
    lattice,
    lattice3,
    library_path,
    params,
    sources,
    wetting_ghost,
)
