"""ctypes binding of libgcme.so: the C ABI of include/gcme.h with the same
names.  Argument marshalling only; every step of the method runs in the HIP
kernels of the library.  Raises if the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcme.so")

GCME_OK, GCME_EINVAL, GCME_EUNSUPPORTED, GCME_EGEOMETRY, GCME_ENONNEUTRAL, GCME_ESTATE, \
    GCME_EDEVICE, GCME_ENOMEM, GCME_EOVERFLOW = range(9)
GCME_FP64, GCME_MIXED = 0, 1
GCME_E_EX, GCME_E_REAL, GCME_E_RECIP, GCME_E_CORR, GCME_E_SELF, GCME_E_POT, GCME_E_KIN, GCME_E_SLAB, \
    GCME_E_BOND, GCME_N_TERMS = range(10)
GCME_MAX_TYPES = 4
GCME_FLAG_STRICT_CONTACT = 1
GCME_FLAG_ALL_RECIPROCAL = 2
GCME_FLAG_SLAB_CORRECTION = 4

STATUS_NAMES = {0: "GCME_OK", 1: "GCME_EINVAL", 2: "GCME_EUNSUPPORTED", 3: "GCME_EGEOMETRY",
                4: "GCME_ENONNEUTRAL", 5: "GCME_ESTATE", 6: "GCME_EDEVICE", 7: "GCME_ENOMEM",
                8: "GCME_EOVERFLOW"}

EXPORTED = ["gcme_create", "gcme_set_params", "gcme_set_bonds", "gcme_set_images", "gcme_set_state", "gcme_get_state", "gcme_forces_energy",
            "gcme_step", "gcme_sync", "gcme_last_error", "gcme_get_tuning", "gcme_set_tuning",
            "gcme_autotune", "gcme_count_pairs", "gcme_profile_step", "gcme_stage_name", "gcme_destroy",
            "gcme_forces_energy_noalloc", "gcme_time_stages"]
GCME_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
GCME_N_STAGES = 12


class gcme_create_info(C.Structure):
    _fields_ = [("n_replicas", C.c_int32), ("n_beads", C.POINTER(C.c_int32)), ("precision", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("seed", C.c_uint64)]


class gcme_params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("cutoff", C.c_double), ("beta", C.c_double),
                ("grid", C.c_int32 * 3), ("order", C.c_int32), ("lB", C.c_double), ("n_types", C.c_int32),
                ("A", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)),
                ("mass", C.POINTER(C.c_double)), ("kT", C.c_double), ("dt", C.c_double), ("gamma", C.c_double),
                ("flags", C.c_uint32), ("kmax", C.c_double), ("bond_k", C.c_double), ("bond_b", C.c_double)]


class gcme_io(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("force", C.c_void_p), ("energy", C.c_void_p), ("virial", C.c_void_p),
                ("dE_dA", C.c_void_p), ("dE_dsigma", C.c_void_p), ("dE_da", C.c_void_p),
                ("dE_dsigma_bead", C.c_void_p), ("dE_da_bead", C.c_void_p), ("force_vjp", C.c_void_p)]


class gcme_tuning(C.Structure):
    _fields_ = [("cells_per_cutoff", C.c_int32), ("beads_per_cluster", C.c_int32),
                ("charges_per_cluster", C.c_int32), ("list_slack_pct", C.c_int32),
                ("direct_pairs", C.c_int32), ("stream_layout", C.c_int32), ("mesh_tile_x", C.c_int32),
                ("mesh_tile_y", C.c_int32), ("gather_tile_x", C.c_int32), ("gather_tile_y", C.c_int32),
                ("half_pairs", C.c_int32)]


class GCMeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libgcme.so (built in-tree by paper_2403_08148_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.gcme_create.argtypes = [C.POINTER(gcme_create_info), C.POINTER(H)]
    L.gcme_set_params.argtypes = [H, C.c_int32, C.POINTER(gcme_params)]
    L.gcme_set_bonds.argtypes = [H, C.c_int64, C.POINTER(C.c_int32)]
    L.gcme_set_images.argtypes = [H, C.c_int64, C.POINTER(C.c_int32)]
    L.gcme_set_state.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.gcme_get_state.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]
    L.gcme_forces_energy.argtypes = [H, C.POINTER(gcme_io)]
    L.gcme_step.argtypes = [H, C.c_int32, C.POINTER(gcme_io)]
    L.gcme_sync.argtypes = [H]
    L.gcme_last_error.argtypes = [H]
    L.gcme_last_error.restype = C.c_char_p
    L.gcme_get_tuning.argtypes = [H, C.POINTER(gcme_tuning)]
    L.gcme_set_tuning.argtypes = [H, C.POINTER(gcme_tuning)]
    L.gcme_autotune.argtypes = [H]
    L.gcme_count_pairs.argtypes = [H, C.POINTER(C.c_uint64)]
    L.gcme_profile_step.argtypes = [H, C.c_int32, C.POINTER(C.c_double)]
    L.gcme_time_stages.argtypes = [H, C.c_int32, C.POINTER(C.c_double)]
    L.gcme_stage_name.argtypes = [C.c_int32]
    L.gcme_stage_name.restype = C.c_char_p
    L.gcme_destroy.argtypes = [H]
    L.gcme_destroy.restype = None
    L.gcme_forces_energy_noalloc.argtypes = [C.POINTER(gcme_params), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    for name in EXPORTED:
        if name not in ("gcme_last_error", "gcme_destroy", "gcme_stage_name"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(handle, status):
    if status != GCME_OK:
        msg = load().gcme_last_error(handle)
        raise GCMeError(status, msg.decode() if msg else "")
    return status
