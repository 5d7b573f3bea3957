"""MI355X-native lattice Boltzmann solver for particle-resolved turbulence.

The compute path is the HIP library ``liblbm.so`` (gfx950) behind the C ABI
in ``include/lbm.h``; ``lbm`` is its ctypes binding.
"""
from .lbm import (BC_IBB, BC_IBM, BC_NONE, STORE_F16S, STORE_F32, WALL_NONE,
                  WALL_PIPE_Z, Config, Lattice, LbmError, lib, workspace_size)

__all__ = ["Config", "Lattice", "LbmError", "lib", "workspace_size", "BC_NONE", "BC_IBB",
           "BC_IBM", "STORE_F32", "STORE_F16S", "WALL_NONE", "WALL_PIPE_Z"]
