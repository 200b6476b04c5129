"""Differentiable GCMe energy: a torch.autograd.Function over the engine.

The potential energy of each replica (U_ex + U_real + U_recip + U_corr +
U_self, the terms of the GCM and Ewald-split smeared Coulomb energies of the
method's Sec. 2) is returned as a function of

  * the bead positions: dE/dr_i = -F_i, the engine's forces;
  * the pair strengths A_tu of eq. (u_ex) per replica: E is linear in A, so
    dE/dA_tu is the type-pair excluded-volume energy over A_tu (hand-written
    adjoint in the pair kernel);
  * the smearing radii a_t of eq. (u_elec) and, either tied to them (one
    radius per bead type) or free, the excluded-volume radii sigma_t
    (adjoint sums of the pair kernels plus the derivative of U_self).

U_recip and U_corr depend on neither A nor the radii, so the mesh part is not
differentiated.  All derivatives come from the library's kernels; this module
only routes them.
"""
from __future__ import annotations

import dataclasses

import torch

E_POT = 5  # index of the total potential energy in the energy row


def _sym(A):
    return 0.5 * (A + A.transpose(-1, -2))


class GCMeEnergy(torch.autograd.Function):
    """energy[R] = GCMeEnergy.apply(pos, A, a, sigma, engine, params)

    pos:    [N, 3] float64 on the engine's device (replica-concatenated)
    A:      [R, nt, nt] float64 (used symmetrised: (A + A^T) / 2)
    a:      [R, nt] float64 smearing radii
    sigma:  [R, nt] float64 excluded-volume radii, or None to tie sigma = a
    engine: a GCMe with its state already set (types and charges)
    params: list of R ReplicaParams supplying everything else

    Each call sets the replicas' parameters (which rebuilds the engine's
    per-type tables) and runs one force/energy evaluation with the adjoint.
    """

    @staticmethod
    def forward(ctx, pos, A, a, sigma, engine, params):
        R = engine.R
        tied = sigma is None
        As = _sym(A.detach()).cpu()
        ac = a.detach().cpu()
        sc = ac if tied else sigma.detach().cpu()
        for r in range(R):
            p = dataclasses.replace(params[r], A=As[r].numpy(), a=ac[r].numpy(), sigma=sc[r].numpy())
            engine.set_params(p, r)
        need_adj = any(t is not None and t.requires_grad for t in (A, a, sigma))
        out = engine.forces_energy(pos=pos.detach(), force=True, energy=True, virial=False, adjoint=need_adj)
        engine.sync()
        E = out["energy"][:, E_POT].clone()
        nt = A.shape[-1]
        if need_adj:
            dA = out["dE_dA"][:, :nt, :nt]
            da = out["dE_da"][:, :nt]
            ds = out["dE_dsigma"][:, :nt]
        else:
            dA = da = ds = None
        ctx.tied = tied
        ctx.nt = nt
        ctx.pdev = A.device
        ctx.counts = list(engine.n_beads)
        ctx.save_for_backward(out["force"], *(t for t in (dA, da, ds) if t is not None))
        ctx.has_adj = need_adj
        return E

    @staticmethod
    def backward(ctx, gE):
        saved = ctx.saved_tensors
        F = saved[0]
        dev = F.device
        gE = gE.to(dev)
        # dE_r/dr_i = -F_i for the beads of replica r
        per_bead = torch.repeat_interleave(gE, torch.tensor(ctx.counts, device=dev))
        g_pos = -(F * per_bead.unsqueeze(0)).t()
        g_A = g_a = g_s = None
        if ctx.has_adj:
            dA, da, ds = saved[1], saved[2], saved[3]
            # the kernel returns dE/dA for each unordered type pair; through
            # the symmetrisation each of the two matrix entries gets half of
            # an off-diagonal value
            nt = ctx.nt
            eye = torch.eye(nt, dtype=dA.dtype, device=dev)
            gA = dA * (0.5 * (1.0 - eye) + eye)
            g_A = (gA * gE[:, None, None]).to(ctx.pdev)
            if ctx.tied:
                g_a = ((da + ds) * gE[:, None]).to(ctx.pdev)
            else:
                g_a = (da * gE[:, None]).to(ctx.pdev)
                g_s = (ds * gE[:, None]).to(ctx.pdev)
        return g_pos, g_A, g_a, g_s, None, None


def gcme_energy(engine, params, pos, A, a, sigma=None):
    """Functional form of GCMeEnergy.apply (see its docstring)."""
    return GCMeEnergy.apply(pos, A, a, sigma, engine, params)


def _set_params(engine, params, A, a, sigma):
    As = _sym(A.detach()).cpu()
    ac = a.detach().cpu()
    sc = ac if sigma is None else sigma.detach().cpu()
    for r in range(engine.R):
        engine.set_params(dataclasses.replace(params[r], A=As[r].numpy(), a=ac[r].numpy(), sigma=sc[r].numpy()), r)


class GCMeForces(torch.autograd.Function):
    """forces[N, 3] = GCMeForces.apply(A, a, sigma, engine, params, pos)

    The forces as a function of the pair strengths and radii (same arguments
    as GCMeEnergy), for force matching: the backward of a loss L(F) passes
    v = dL/dF to the library's force vector-Jacobian product, the sums
    sum_i v_i . dF_i/dtheta accumulated in the pair kernels (only the pair
    terms of eq. u_ex and of eq. ewald's real-space term depend on A and the
    radii).  The engine keeps the forward's parameters until the backward.
    """

    @staticmethod
    def forward(ctx, A, a, sigma, engine, params, pos):
        _set_params(engine, params, A, a, sigma)
        out = engine.forces_energy(pos=pos.detach(), force=True, energy=False, virial=False)
        engine.sync()
        ctx.engine, ctx.pos, ctx.tied, ctx.nt, ctx.pdev = engine, pos.detach(), sigma is None, A.shape[-1], A.device
        return out["force"].t().contiguous()

    @staticmethod
    def backward(ctx, gF):
        eng = ctx.engine
        out = eng.forces_energy(pos=ctx.pos, force=False, energy=False, virial=False, adjoint=True,
                                force_vjp=gF.detach().to(torch.float64).contiguous())
        eng.sync()
        nt = ctx.nt
        dA, da, ds = out["dE_dA"][:, :nt, :nt], out["dE_da"][:, :nt], out["dE_dsigma"][:, :nt]
        # a type pair's value is for the symmetric parameter: half to each of
        # the two matrix entries through the symmetrisation
        eye = torch.eye(nt, dtype=dA.dtype, device=dA.device)
        g_A = (dA * (0.5 * (1.0 - eye) + eye)).to(ctx.pdev)
        if ctx.tied:
            return g_A, (da + ds).to(ctx.pdev), None, None, None, None
        return g_A, da.to(ctx.pdev), ds.to(ctx.pdev), None, None, None


def gcme_forces(engine, params, pos, A, a, sigma=None):
    """Functional form of GCMeForces.apply (see its docstring)."""
    return GCMeForces.apply(A, a, sigma, engine, params, pos)


__all__ = ["GCMeEnergy", "gcme_energy", "GCMeForces", "gcme_forces", "E_POT"]
