"""FP64 CPU oracle for the GCMe nonbonded path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path (the HIP library in
``paper_2403_08148_amd``) never imports it, and it never imports the product.

Thin ctypes binding over ``gcme_oracle.c``; every function here only marshals
numpy arrays.  What each C routine computes, and which passage of the paper it
follows, is documented in the C source.

Array conventions (host numpy):
  pos   float64 [N, 3] (AoS), any real coordinates
  type  int32   [N]
  z     int32   [N] charge numbers
Returned forces are float64 [N, 3].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcme_oracle.c")
_LIB = os.path.join(_HERE, "libgcme_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("rc", C.c_double), ("beta", C.c_double),
                ("lB", C.c_double), ("nt", C.c_int), ("A", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double))]


class _Recip(C.Structure):
    _fields_ = [("mode", C.c_int), ("kmax", C.c_double), ("K", C.c_int * 3), ("order", C.c_int)]


class _Extra(C.Structure):
    _fields_ = [("slab", C.c_int), ("nbonds", C.c_int), ("bonds", C.POINTER(C.c_int)),
                ("bond_k", C.c_double), ("bond_b", C.c_double), ("nimages", C.c_int),
                ("images", C.POINTER(C.c_int))]


RECIP_NONE, RECIP_EWALD, RECIP_SPME = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        u64p = C.POINTER(C.c_uint64)
        L.gco_u_ex.restype = C.c_double
        L.gco_u_ex.argtypes = [C.c_double, C.c_double, C.c_double]
        L.gco_u_elec.restype = C.c_double
        L.gco_u_elec.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.gco_phi_real.restype = C.c_double
        L.gco_phi_real.argtypes = [C.c_double, C.c_double, C.c_double]
        L.gco_real_space.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), C.c_int, C.c_int, ip,
                                     dp, dp, dp, dp, dp, dp]
        L.gco_real_space_images.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), dp, dp, dp]
        L.gco_constants.argtypes = [C.c_int, ip, ip, C.POINTER(_Params), dp, dp, dp]
        L.gco_ewald_recip.restype = C.c_int
        L.gco_ewald_recip.argtypes = [C.c_int, dp, ip, dp, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.gco_fft.argtypes = [C.c_int, dp, C.c_int]
        L.gco_bspline.restype = C.c_double
        L.gco_bspline.argtypes = [C.c_int, C.c_double]
        L.gco_bspline_moduli.argtypes = [C.c_int, C.c_int, dp]
        L.gco_spme_recip.argtypes = [C.c_int, dp, ip, dp, C.c_double, C.c_double, ip, C.c_int,
                                     dp, dp, dp, dp]
        L.gco_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.gco_gauss3.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, dp]
        L.gco_forces.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), C.POINTER(_Recip), dp, dp, dp]
        L.gco_forces_ext.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), C.POINTER(_Recip),
                                     C.POINTER(_Extra), dp, dp, dp]
        L.gco_slab.restype = C.c_double
        L.gco_slab.argtypes = [C.c_int, dp, ip, dp, C.c_double, dp, dp]
        L.gco_mirror_images.argtypes = [dp, dp, C.c_int, ip]
        L.gco_per_bead_adjoint.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), dp, dp]
        L.gco_force_vjp.argtypes = [C.c_int, dp, ip, ip, C.POINTER(_Params), dp, dp, dp, dp]
        L.gco_bonds.restype = C.c_double
        L.gco_bonds.argtypes = [C.c_int, dp, dp, C.c_int, ip, C.c_double, C.c_double, dp, dp]
        L.gco_md.argtypes = [C.c_int, dp, dp, dp, ip, ip, ip, C.POINTER(_Params), C.POINTER(_Recip),
                             C.POINTER(_Extra), dp, C.c_double, C.c_double, C.c_double, C.c_uint64,
                             C.c_uint64, C.c_uint64, C.c_int, dp]
        L.gco_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


@dataclass
class Params:
    """Force-field parameters of one periodic box (reduced units, kT = 1)."""
    box: tuple
    rc: float
    beta: float
    lB: float
    A: np.ndarray       # [nt, nt]
    sigma: np.ndarray   # [nt]
    a: np.ndarray       # [nt]

    def _c(self):
        self._A = np.ascontiguousarray(self.A, dtype=np.float64).ravel()
        self._s = np.ascontiguousarray(self.sigma, dtype=np.float64)
        self._a = np.ascontiguousarray(self.a, dtype=np.float64)
        p = _Params()
        p.box[:] = [float(x) for x in self.box]
        p.rc, p.beta, p.lB = float(self.rc), float(self.beta), float(self.lB)
        p.nt = len(self._s)
        p.A, p.sigma, p.a = _d(self._A), _d(self._s), _d(self._a)
        return p


def _prep(pos, type_, z):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    z = np.ascontiguousarray(z, dtype=np.int32)
    return pos, type_, z


def u_ex(r, A, s2):
    return lib().gco_u_ex(float(r), float(A), float(s2))


def u_elec(r, lB, zz, aij):
    return lib().gco_u_elec(float(r), float(lB), float(zz), float(aij))


def phi_real(r, alpha, beta):
    return lib().gco_phi_real(float(r), float(alpha), float(beta))


def real_space(pos, type_, z, p: Params, use_cells=True, sample=None, adjoint=False, energies=True):
    """Min-image real space (GCM + smeared-Coulomb bracket), r < rc.
    Returns dict with F (forces on all beads, or on ``sample``), E_ex, E_real,
    W[6] (xx,yy,zz,xy,xz,yz), and with adjoint: Eex_tt [nt,nt], dE_dsigma,
    dE_da (real-space part).  energies=False (with a sample) computes only the
    sampled forces, visiting only the sampled beads."""
    pos, type_, z = _prep(pos, type_, z)
    N = len(pos)
    pc = p._c()
    nt = pc.nt
    if sample is not None:
        sample = np.ascontiguousarray(sample, dtype=np.int32)
        F = np.zeros((len(sample), 3))
    else:
        F = np.zeros((N, 3))
    E2 = np.zeros(2) if energies else None
    W = np.zeros(6) if energies else None
    ett = np.zeros(nt * nt) if adjoint else None
    dsg = np.zeros(nt) if adjoint else None
    dea = np.zeros(nt) if adjoint else None
    rc = lib().gco_real_space(N, _d(pos), _i(type_), _i(z), C.byref(pc), int(bool(use_cells)),
                              0 if sample is None else len(sample), _i(sample),
                              _d(F), _d(E2), _d(W), _d(ett), _d(dsg), _d(dea))
    if rc != 0:
        raise ValueError("oracle real_space: rc must be <= L/2")
    out = dict(F=F)
    if energies:
        out.update(E_ex=E2[0], E_real=E2[1], W=W)
    if adjoint:
        out.update(Eex_tt=ett.reshape(nt, nt), dE_dsigma=dsg, dE_da=dea)
    return out


def real_space_images(pos, type_, z, p: Params):
    pos, type_, z = _prep(pos, type_, z)
    N = len(pos)
    pc = p._c()
    F = np.zeros((N, 3))
    E2 = np.zeros(2)
    W = np.zeros(6)
    lib().gco_real_space_images(N, _d(pos), _i(type_), _i(z), C.byref(pc), _d(F), _d(E2), _d(W))
    return dict(F=F, E_ex=E2[0], E_real=E2[1], W=W)


def constants(type_, z, p: Params):
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    z = np.ascontiguousarray(z, dtype=np.int32)
    pc = p._c()
    ec, es = C.c_double(), C.c_double()
    dself = np.zeros(pc.nt)
    lib().gco_constants(len(z), _i(type_), _i(z), C.byref(pc), C.byref(ec), C.byref(es), _d(dself))
    return dict(E_corr=ec.value, E_self=es.value, dE_da_self=dself)


def ewald_recip(pos, z, box, beta, lB, kmax):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    z = np.ascontiguousarray(z, dtype=np.int32)
    N = len(pos)
    F = np.zeros((N, 3))
    E = C.c_double()
    W = np.zeros(6)
    b = np.asarray(box, dtype=np.float64)
    nk = lib().gco_ewald_recip(N, _d(pos), _i(z), _d(b), float(beta), float(lB), float(kmax),
                               _d(F), C.byref(E), _d(W))
    return dict(F=F, E_recip=E.value, W=W, n_kvec_half=nk)


def spme_recip(pos, z, box, beta, lB, K, order, want_phi=False):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    z = np.ascontiguousarray(z, dtype=np.int32)
    N = len(pos)
    F = np.zeros((N, 3))
    E = C.c_double()
    W = np.zeros(6)
    b = np.asarray(box, dtype=np.float64)
    Karr = np.ascontiguousarray(K, dtype=np.int32)
    phi = np.zeros(tuple(int(k) for k in K)) if want_phi else None
    lib().gco_spme_recip(N, _d(pos), _i(z), _d(b), float(beta), float(lB), _i(Karr), int(order),
                         _d(F), C.byref(E), _d(W), _d(phi))
    out = dict(F=F, E_recip=E.value, W=W)
    if want_phi:
        out["phi"] = phi
    return out


def fft(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128).copy()
    buf = x.view(np.float64)
    lib().gco_fft(len(x), _d(buf), int(sign))
    return buf.view(np.complex128)


def bspline(n, x):
    return lib().gco_bspline(int(n), float(x))


def bspline_moduli(K, p):
    out = np.zeros(int(K))
    lib().gco_bspline_moduli(int(K), int(p), _d(out))
    return out


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib().gco_philox4x64_10(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def gauss3(seed, step, bead_id, replica):
    out = np.zeros(3)
    lib().gco_gauss3(C.c_uint64(seed), C.c_uint64(step), C.c_uint64(bead_id), C.c_uint64(replica), _d(out))
    return out


def _recip(mode, kmax=0.0, K=(0, 0, 0), order=0):
    r = _Recip()
    r.mode, r.kmax, r.order = int(mode), float(kmax), int(order)
    r.K[:] = [int(k) for k in K]
    return r


def forces(pos, type_, z, p: Params, recip_mode=RECIP_SPME, kmax=0.0, K=(0, 0, 0), order=5):
    """Total forces and the five energy terms of eq. ewald plus GCM:
    E = [E_ex, E_real, E_recip, E_corr, E_self]; W = pair + reciprocal virial."""
    pos, type_, z = _prep(pos, type_, z)
    N = len(pos)
    pc = p._c()
    rec = _recip(recip_mode, kmax, K, order)
    F = np.zeros((N, 3))
    E = np.zeros(5)
    W = np.zeros(6)
    rc = lib().gco_forces(N, _d(pos), _i(type_), _i(z), C.byref(pc), C.byref(rec), _d(F), _d(E), _d(W))
    if rc != 0:
        raise ValueError("oracle forces: rc must be <= L/2")
    return dict(F=F, E=E, W=W)


def slab(pos, z, box, lB):
    """Slab correction of a slab with a vacuum gap along z (see gco_slab):
    energy, forces [N, 3] and virial of that term alone."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    z = np.ascontiguousarray(z, dtype=np.int32)
    F = np.zeros_like(pos)
    W = np.zeros(6)
    b = np.ascontiguousarray(box, dtype=np.float64)
    E = lib().gco_slab(len(pos), _d(pos), _i(z), _d(b), float(lB), _d(F), _d(W))
    return dict(E=E, F=F, W=W)


def bonds(pos, box, pairs, k, b):
    """Harmonic bonds k/2 (r - b)^2 over the minimum image (see gco_bonds):
    energy, forces [N, 3] and virial of that term alone."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    F = np.zeros_like(pos)
    W = np.zeros(6)
    bx = np.ascontiguousarray(box, dtype=np.float64)
    E = lib().gco_bonds(len(pos), _d(pos), _d(bx), len(pairs), _i(pairs), float(k), float(b), _d(F), _d(W))
    return dict(E=E, F=F, W=W)


def per_bead_adjoint(pos, type_, z, p: Params):
    """dE/dsigma_i and dE/da_i of every bead (see gco_per_bead_adjoint)."""
    pos, type_, z = _prep(pos, type_, z)
    N = len(pos)
    pc = p._c()
    ds, da = np.zeros(N), np.zeros(N)
    if lib().gco_per_bead_adjoint(N, _d(pos), _i(type_), _i(z), C.byref(pc), _d(ds), _d(da)) != 0:
        raise ValueError("oracle: rc must be <= L/2")
    return dict(dE_dsigma=ds, dE_da=da)


def force_vjp(pos, type_, z, p: Params, v):
    """sum_i v_i . dF_i/dtheta for theta = A (symmetric, [nt, nt]), sigma
    and a ([nt] each); v is [N, 3] (see gco_force_vjp)."""
    pos, type_, z = _prep(pos, type_, z)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    nt = len(p.sigma)
    pc = p._c()
    dA, ds, da = np.zeros(nt * nt), np.zeros(nt), np.zeros(nt)
    if lib().gco_force_vjp(len(pos), _d(pos), _i(type_), _i(z), C.byref(pc), _d(v), _d(dA), _d(ds), _d(da)) != 0:
        raise ValueError("oracle: rc must be <= L/2")
    return dict(dA=dA.reshape(nt, nt), dsigma=ds, da=da)


def mirror_images(pos, box, images):
    """Image beads moved to their sources' reflections across z = 0 (see
    gco_mirror_images); images is [n, 2] of (image, source)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3).copy()
    images = np.ascontiguousarray(images, dtype=np.int32).reshape(-1, 2)
    bx = np.ascontiguousarray(box, dtype=np.float64)
    lib().gco_mirror_images(_d(pos), _d(bx), len(images), _i(images))
    return pos


class Extra:
    """Terms beyond the nonbonded force field: the slab correction, harmonic
    bonds (bead-index pairs) and image charges ((image, source) pairs)."""

    def __init__(self, slab=False, pairs=None, bond_k=0.0, bond_b=0.0, images=None):
        self.pairs = np.ascontiguousarray(pairs if pairs is not None else np.zeros((0, 2)),
                                          dtype=np.int32).reshape(-1, 2)
        self.images = np.ascontiguousarray(images if images is not None else np.zeros((0, 2)),
                                           dtype=np.int32).reshape(-1, 2)
        self.c = _Extra()
        self.c.slab = 1 if slab else 0
        self.c.nbonds = len(self.pairs)
        self.c.bonds = _i(self.pairs)
        self.c.bond_k, self.c.bond_b = float(bond_k), float(bond_b)
        self.c.nimages = len(self.images)
        self.c.images = _i(self.images)


def forces_ext(pos, type_, z, p: Params, extra: Extra, recip_mode=RECIP_SPME, kmax=0.0, K=(0, 0, 0),
               order=5):
    """forces() plus the extra terms: E = [E_ex, E_real, E_recip, E_corr,
    E_self, E_slab, E_bond]."""
    pos, type_, z = _prep(pos, type_, z)
    N = len(pos)
    pc = p._c()
    rec = _recip(recip_mode, kmax, K, order)
    F = np.zeros((N, 3))
    E = np.zeros(7)
    W = np.zeros(6)
    rc = lib().gco_forces_ext(N, _d(pos), _i(type_), _i(z), C.byref(pc), C.byref(rec), C.byref(extra.c),
                              _d(F), _d(E), _d(W))
    if rc != 0:
        raise ValueError("oracle forces: rc must be <= L/2")
    return dict(F=F, E=E, W=W)


def md(pos, vel, type_, z, ids, p: Params, mass, dt, gamma, kT, seed, replica, step0, n_steps,
       recip_mode=RECIP_SPME, kmax=0.0, K=(0, 0, 0), order=5, extra: Extra | None = None):
    """n_steps of velocity Verlet (gamma == 0) or BAOAB Langevin; returns
    (pos, vel, F, Elog[n_steps, 2] = (potential, kinetic)).  A type of
    infinite mass stays fixed (its beads must start at rest)."""
    pos, type_, z = _prep(pos, type_, z)
    pos = pos.copy()
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3).copy()
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    N = len(pos)
    pc = p._c()
    rec = _recip(recip_mode, kmax, K, order)
    ex = extra if extra is not None else Extra()
    F = forces_ext(pos, type_, z, p, ex, recip_mode, kmax, K, order)["F"].copy()
    Elog = np.zeros((n_steps, 2))
    rc = lib().gco_md(N, _d(pos), _d(vel), _d(F), _i(type_), _i(z), _i(ids), C.byref(pc), C.byref(rec),
                      C.byref(ex.c), _d(mass), float(dt), float(gamma), float(kT), C.c_uint64(seed),
                      C.c_uint64(replica), C.c_uint64(step0), int(n_steps), _d(Elog))
    if rc != 0:
        raise ValueError("oracle md failed")
    return pos, vel, F, Elog


def num_threads() -> int:
    return lib().gco_num_threads()
