"""Seeded synthetic inputs shared by the oracle tests and the GPU library:
geometry only, none of the lattice Boltzmann arithmetic."""
from .geometry import (DIRS, INLET, NDIR, OUTLET, WALL, Geometry, Iolet, box, tubes,  # noqa: F401
                       build_site_list, channel, cylinder, iolet_code, long_pipe)
from .trees import coupled_pair, ensemble, branching_artery, tree_geometry  # noqa: F401
from . import workloads  # noqa: F401
