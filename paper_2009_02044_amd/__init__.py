"""MI355X (gfx950) HIP implementation of the 3+1D Glasma colored-particle-in-cell
evolution (Ipp & Mueller, arXiv:2009.02044): leapfrog and semi-implicit field
updates of SU(2)/SU(3) links and electric fields driven by the charges of two MV
nuclei, with observables, behind the C-ABI of include/glasma.h.

The compute path is libglasma.so only; importing this package fails if it is
missing.  torch provides device memory and the stream.
"""
from ._lib import lib, GlasmaError, LIB_PATH  # noqa: F401  (raises if the library is missing)
from .glasma import Lattice, Batch, SlabEnergy, host_group_op, boost_invariant_fields  # noqa: F401

__all__ = ["Lattice", "Batch", "SlabEnergy", "GlasmaError", "host_group_op", "boost_invariant_fields", "lib",
           "LIB_PATH"]
