"""MI355X (gfx950) lattice Boltzmann library for a van der Waals liquid-vapor
fluid under a periodic force and wall shear (Coclite, Gonnella, Lamura,
arXiv:1307.6703). The HIP library liblbvdw.so does all the work; this package
binds it (``lbvdw``)."""
from .lbvdw import (FP32, FP32_SR, FP64, Batch, LBError, Lattice, Lattice17,  # noqa: F401
                    lattice17, load_library, make_params, precision)

__all__ = ["Batch", "FP32", "FP32_SR", "FP64", "LBError", "Lattice", "Lattice17", "lattice17",
           "load_library", "make_params", "precision"]
