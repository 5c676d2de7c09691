"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only *generates inputs*: meshes (coordinates, cells, the
vertex-to-dof map used for periodic identification), Dirichlet dof sets,
initial and boundary fields, random permutations and colouring priorities.
It holds none of the solver's arithmetic (no element matrices, no assembly,
no Krylov iteration); the oracle (``oracle/``) and the HIP library
(``paper_1602_03643_amd``) each implement that on their own.
"""
from .meshes import (Mesh, unit_square, periodic_square, channel,
                     permute_mesh, cell_priorities)
from .problems import (Problem, taylor_green, channel_flow, CHANNEL_SIZES,
                       tg_exact_velocity, tg_exact_pressure)

__all__ = ["Mesh", "unit_square", "periodic_square", "channel", "permute_mesh",
           "cell_priorities", "Problem", "taylor_green", "channel_flow",
           "CHANNEL_SIZES", "tg_exact_velocity", "tg_exact_pressure"]
