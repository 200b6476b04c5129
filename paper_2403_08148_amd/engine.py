"""Python front end of the GCMe engine: a thin wrapper that hands torch
device tensors to the C ABI (include/gcme.h).  torch provides device memory
and the stream; all arithmetic runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _binding as B


@dataclass
class ReplicaParams:
    box: Sequence[float]
    cutoff: float
    beta: float
    grid: Sequence[int]
    order: int
    lB: float
    A: np.ndarray
    sigma: np.ndarray
    a: np.ndarray
    mass: Optional[np.ndarray] = None
    kT: float = 1.0
    dt: float = 0.02
    gamma: float = 1.0
    flags: int = 0
    kmax: float = 0.0  # > 0: exact reciprocal sum over |k| <= kmax instead of the mesh
    bond_k: float = 0.0  # harmonic bonds bond_k/2 (r - bond_b)^2 (set_bonds)
    bond_b: float = 0.0


def c_params(p: ReplicaParams):
    """The gcme_params struct of p, and the host arrays it points to (keep
    them alive while the struct is in use)."""
    nt = len(p.sigma)
    A = np.ascontiguousarray(np.asarray(p.A, dtype=np.float64).reshape(nt, nt))
    s = np.ascontiguousarray(p.sigma, dtype=np.float64)
    a = np.ascontiguousarray(p.a, dtype=np.float64)
    m = np.ascontiguousarray(p.mass, dtype=np.float64) if p.mass is not None else None
    dp = C.POINTER(C.c_double)
    cp = B.gcme_params((C.c_double * 3)(*[float(x) for x in p.box]), float(p.cutoff), float(p.beta),
                       (C.c_int32 * 3)(*[int(k) for k in p.grid]), int(p.order), float(p.lB), nt,
                       A.ctypes.data_as(dp), s.ctypes.data_as(dp), a.ctypes.data_as(dp),
                       m.ctypes.data_as(dp) if m is not None else None, float(p.kT), float(p.dt),
                       float(p.gamma), int(p.flags), float(p.kmax), float(p.bond_k), float(p.bond_b))
    return cp, (A, s, a, m)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class GCMe:
    """One engine context over one or more independent periodic replicas.

    Per-bead tensors are float64/int32 on the engine's CUDA device, replica-
    concatenated; coordinates may be given as [N, 3] or [3, N] (the ABI uses
    [3, N]).  Outputs are returned as torch tensors on the same device.
    """

    def __init__(self, n_beads, precision: str = "mixed", device: int = 0, seed: int = 0,
                 stream=None):
        import torch
        self.torch = torch
        self.lib = B.load()
        if isinstance(n_beads, int):
            n_beads = [n_beads]
        self.n_beads = [int(n) for n in n_beads]
        self.R = len(self.n_beads)
        self.N = sum(self.n_beads)
        self.device = torch.device("cuda", device)
        self.precision = precision
        if stream is None or stream.cuda_stream == 0:
            # a dedicated (non-default) torch stream: handle 0 would mean
            # "library-owned stream" to the C ABI, invisible to torch events
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        nb = (C.c_int32 * self.R)(*self.n_beads)
        info = B.gcme_create_info(self.R, C.cast(nb, C.POINTER(C.c_int32)),
                                  B.GCME_FP64 if precision == "fp64" else B.GCME_MIXED, device,
                                  C.c_void_p(stream.cuda_stream), seed)
        h = C.c_void_p()
        B.check(None, self.lib.gcme_create(C.byref(info), C.byref(h)))
        self.h = h
        self.params = [None] * self.R

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.gcme_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ------------------------------------------------------------
    def set_params(self, p: ReplicaParams, replica: int = -1):
        cp, _keep = c_params(p)
        B.check(self.h, self.lib.gcme_set_params(self.h, int(replica), C.byref(cp)))
        for r in (range(self.R) if replica < 0 else [replica]):
            self.params[r] = p

    def set_bonds(self, pairs):
        """Harmonic bonds between concatenated bead indices ([n, 2], both
        beads of a bond in one replica); replaces the previous list."""
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        B.check(self.h, self.lib.gcme_set_bonds(self.h, len(pr), pr.ctypes.data_as(C.POINTER(C.c_int32))))

    def set_images(self, pairs):
        """Image charges: [n, 2] (image bead, source bead) concatenated
        indices; replaces the previous list."""
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        B.check(self.h, self.lib.gcme_set_images(self.h, len(pr), pr.ctypes.data_as(C.POINTER(C.c_int32))))

    def _soa(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device)
        if t.dim() == 2 and t.shape[0] == self.N and t.shape[1] == 3 and self.N != 3:
            t = t.t()
        return t.contiguous()

    def set_state(self, pos, type_, z, vel=None):
        torch = self.torch
        pos = self._soa(pos)
        vel = self._soa(vel) if vel is not None else None
        type_ = torch.as_tensor(type_, dtype=torch.int32, device=self.device).contiguous()
        z = torch.as_tensor(z, dtype=torch.int32, device=self.device).contiguous()
        self._engine_waits()
        B.check(self.h, self.lib.gcme_set_state(self.h, _ptr(pos), _ptr(vel), _ptr(type_), _ptr(z)))

    # The library works on its own stream.  Inputs made on torch's current
    # stream must be complete before it reads them, and its outputs before
    # torch's stream reads them: two event waits, no host synchronisation.
    def _engine_waits(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _caller_waits(self, outs=()):
        cur = self.torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        # outputs made on the library's stream are read on the caller's
        for t in outs:
            t.record_stream(cur)

    def get_state(self):
        torch = self.torch
        pos = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        vel = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        pos.record_stream(self.stream)
        vel.record_stream(self.stream)
        self._engine_waits()
        step = C.c_uint64()
        B.check(self.h, self.lib.gcme_get_state(self.h, _ptr(pos), _ptr(vel), C.byref(step)))
        self._caller_waits()
        return pos, vel, step.value

    # -- evaluation -------------------------------------------------------
    def _io(self, pos=None, force=True, energy=True, virial=True, adjoint=False, per_bead=False, force_vjp=None):
        with self.torch.cuda.stream(self.stream):
            return self._io_on_stream(pos, force, energy, virial, adjoint, per_bead, force_vjp)

    def _io_on_stream(self, pos, force, energy, virial, adjoint, per_bead=False, force_vjp=None):
        torch = self.torch
        out = {}
        keep = []
        io = B.gcme_io()
        if pos is not None:
            p = self._soa(pos)
            # the engine reads it asynchronously on its stream
            p.record_stream(self.stream)
            keep.append(p)
            io.pos = p.data_ptr()
        if force:
            out["force"] = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
            io.force = out["force"].data_ptr()
        if energy:
            out["energy"] = torch.empty((self.R, B.GCME_N_TERMS), dtype=torch.float64, device=self.device)
            io.energy = out["energy"].data_ptr()
        if virial:
            out["virial"] = torch.empty((self.R, 6), dtype=torch.float64, device=self.device)
            io.virial = out["virial"].data_ptr()
        if adjoint:
            T = B.GCME_MAX_TYPES
            out["dE_dA"] = torch.empty((self.R, T, T), dtype=torch.float64, device=self.device)
            out["dE_dsigma"] = torch.empty((self.R, T), dtype=torch.float64, device=self.device)
            out["dE_da"] = torch.empty((self.R, T), dtype=torch.float64, device=self.device)
            io.dE_dA = out["dE_dA"].data_ptr()
            io.dE_dsigma = out["dE_dsigma"].data_ptr()
            io.dE_da = out["dE_da"].data_ptr()
        if force_vjp is not None:
            # v = dL/dF per bead: the adjoint outputs then hold sum_i v_i . dF_i/dtheta
            v = self._soa(force_vjp)
            v.record_stream(self.stream)
            keep.append(v)
            io.force_vjp = v.data_ptr()
        if per_bead:
            # per-bead radius derivatives, original bead order
            out["dE_dsigma_bead"] = torch.empty(self.N, dtype=torch.float64, device=self.device)
            out["dE_da_bead"] = torch.empty(self.N, dtype=torch.float64, device=self.device)
            io.dE_dsigma_bead = out["dE_dsigma_bead"].data_ptr()
            io.dE_da_bead = out["dE_da_bead"].data_ptr()
        return io, out, keep

    def forces_energy(self, pos=None, force=True, energy=True, virial=True, adjoint=False, per_bead=False,
                      force_vjp=None):
        self._engine_waits()
        io, out, keep = self._io(pos, force, energy, virial, adjoint, per_bead, force_vjp)
        B.check(self.h, self.lib.gcme_forces_energy(self.h, C.byref(io)))
        self._caller_waits(out.values())
        return out

    def step(self, n_steps: int, observe: bool = False, **kw):
        self._engine_waits()
        if observe:
            io, out, keep = self._io(None, **kw)
            B.check(self.h, self.lib.gcme_step(self.h, int(n_steps), C.byref(io)))
            self._caller_waits(out.values())
            return out
        B.check(self.h, self.lib.gcme_step(self.h, int(n_steps), None))
        self._caller_waits()
        return None

    def sync(self):
        B.check(self.h, self.lib.gcme_sync(self.h))

    def count_pairs(self) -> int:
        n = C.c_uint64()
        B.check(self.h, self.lib.gcme_count_pairs(self.h, C.byref(n)))
        return n.value

    def tuning(self):
        t = B.gcme_tuning()
        B.check(self.h, self.lib.gcme_get_tuning(self.h, C.byref(t)))
        return dict(cells_per_cutoff=t.cells_per_cutoff, beads_per_cluster=t.beads_per_cluster,
                    charges_per_cluster=t.charges_per_cluster, list_slack_pct=t.list_slack_pct,
                    direct_pairs=t.direct_pairs, stream_layout=t.stream_layout, mesh_tile_x=t.mesh_tile_x,
                    mesh_tile_y=t.mesh_tile_y, gather_tile_x=t.gather_tile_x, gather_tile_y=t.gather_tile_y,
                    half_pairs=t.half_pairs)

    def set_tuning(self, cells_per_cutoff=-1, beads_per_cluster=-1, charges_per_cluster=-1, list_slack_pct=-1,
                   direct_pairs=-1, stream_layout=-1, mesh_tile_x=-1, mesh_tile_y=-1, gather_tile_x=-1,
                   gather_tile_y=-1, half_pairs=-1):
        t = B.gcme_tuning(cells_per_cutoff, beads_per_cluster, charges_per_cluster, list_slack_pct, direct_pairs,
                          stream_layout, mesh_tile_x, mesh_tile_y, gather_tile_x, gather_tile_y, half_pairs)
        B.check(self.h, self.lib.gcme_set_tuning(self.h, C.byref(t)))

    def profile_step(self, n_reps: int = 10) -> dict:
        """Device time (ms) of each stage of a step: the stage's kernels are
        replayed n_reps times back to back from a HIP graph between two HIP
        events on the engine's stream (state, forces and mesh restored)."""
        ms = (C.c_double * B.GCME_N_STAGES)()
        B.check(self.h, self.lib.gcme_profile_step(self.h, int(n_reps), ms))
        return {self.lib.gcme_stage_name(i).decode(): ms[i] for i in range(B.GCME_N_STAGES)}

    def time_stages(self, n_steps: int = 20) -> dict:
        """Device time (ms) of each stage's kernels inside real steps (HIP
        event-record nodes in the step graph); takes n_steps steps."""
        ms = (C.c_double * B.GCME_N_STAGES)()
        B.check(self.h, self.lib.gcme_time_stages(self.h, int(n_steps), ms))
        return {self.lib.gcme_stage_name(i).decode(): ms[i] for i in range(B.GCME_N_STAGES)}

    def autotune(self):
        B.check(self.h, self.lib.gcme_autotune(self.h))
        return self.tuning()


def params_from_workload(w, **over) -> ReplicaParams:
    """ReplicaParams from a gcme_workloads.Workload-like object."""
    d = dict(box=w.box, cutoff=w.rc, beta=w.beta, grid=w.grid, order=w.order, lB=w.lB, A=w.A,
             sigma=w.sigma, a=w.a, mass=w.mass, kT=w.kT, dt=w.dt, gamma=w.gamma)
    d.update(over)
    return ReplicaParams(**d)
