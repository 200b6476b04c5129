"""MI355X (gfx950) engine for the GCMe nonbonded force/energy path.

The HIP library ``libgcme.so`` (built in-tree from ``csrc/``) implements the
cell list, the cutoff pair kernels and smooth PME; this package is its thin
Python front end.  Importing the package does not need a GPU; creating an
engine does, and raises if the library has not been built.
"""
from ._binding import GCMeError, load  # noqa: F401
from .engine import GCMe, ReplicaParams, params_from_workload  # noqa: F401
from .autograd import GCMeEnergy, gcme_energy  # noqa: F401

__all__ = ["GCMe", "GCMeError", "GCMeEnergy", "ReplicaParams", "gcme_energy", "params_from_workload", "load"]
