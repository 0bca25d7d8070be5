"""MI355X (gfx950) electromagnetic lattice Boltzmann hot path.

Hand-written HIP kernels behind the C ABI in include/lbm_em.h, loaded
through ctypes.  See sim.Simulation.
"""
from ._lib import LbmEmError, lib  # noqa: F401
from .sim import Batch, Simulation, far_field_objective, step_many  # noqa: F401
