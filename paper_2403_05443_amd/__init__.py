"""MI355X (gfx950) lattice Boltzmann library for rigid ellipsoidal particles.

The method is that of Thampi, Stratford & Henrich (arXiv 2403.05443); the
compute path is the HIP library ``liblbell.so`` behind the C ABI in
``include/lbell.h``; ``lbell`` is its Python binding.
"""
from . import lbell  # noqa: F401
from .lbell import Lattice, LBError, Surrogate, make_box  # noqa: F401
