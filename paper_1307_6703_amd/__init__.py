"""MI355X (gfx950) lattice Boltzmann library for a van der Waals liquid-vapor
fluid under a periodic force and wall shear (Coclite, Gonnella, Lamura,
arXiv:1307.6703). The HIP library liblbvdw.so does all the work; this package
binds it (``lbvdw``)."""
from .lbvdw import Batch, LBError, Lattice, load_library, make_params  # noqa: F401

__all__ = ["Batch", "LBError", "Lattice", "load_library", "make_params"]
