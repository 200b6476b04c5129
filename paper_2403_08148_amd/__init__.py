"""MI355X (gfx950) engine for the GCMe nonbonded force/energy path.

The HIP library ``libgcme.so`` (built in-tree from ``csrc/``) implements the
cell list, the cutoff pair kernels and smooth PME; this package is its thin
Python front end.  Importing the package does not need a GPU; creating an
engine does, and raises if the library has not been built.
"""
from ._binding import GCMeError, load  # noqa: F401
from .engine import GCMe, ReplicaParams, params_from_workload  # noqa: F401
from .autograd import GCMeEnergy, GCMeForces, gcme_energy, gcme_forces  # noqa: F401

__all__ = ["GCMe", "GCMeError", "GCMeEnergy", "GCMeForces", "ReplicaParams", "gcme_energy", "gcme_forces", "params_from_workload", "load"]
