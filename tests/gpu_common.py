"""Helpers shared by the GPU tests: run the HIP engine and the FP64 oracle on
the same seeded inputs and compare.  (Not collected by pytest.)"""
import numpy as np

from oracle import oracle as O


def make_engine(ws, precision, seed=1, tuning=None, kmax=None):
    """kmax: None (every replica on its mesh) or one value per replica (> 0:
    that replica's reciprocal sum taken exactly over |k| <= kmax)."""
    from paper_2403_08148_amd import GCMe, params_from_workload
    eng = GCMe([w.N for w in ws], precision=precision, seed=seed)
    for r, w in enumerate(ws):
        over = {} if kmax is None else dict(kmax=float(kmax[r]))
        eng.set_params(params_from_workload(w, **over), replica=r)
    if tuning:
        eng.set_tuning(**tuning)
    pos = np.concatenate([w.pos for w in ws])
    typ = np.concatenate([w.type for w in ws])
    z = np.concatenate([w.z for w in ws])
    vel = np.concatenate([w.vel for w in ws])
    eng.set_state(pos, typ, z, vel)
    return eng


def gpu_eval(eng, adjoint=False, pos=None):
    out = eng.forces_energy(pos=pos, adjoint=adjoint)
    eng.sync()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["force"] = res["force"].T.copy()
    return res


def oracle_params(w, **over):
    d = dict(box=w.box, rc=w.rc, beta=w.beta, lB=w.lB, A=w.A, sigma=w.sigma, a=w.a)
    d.update(over)
    return O.Params(**d)


def oracle_eval(w, adjoint=False, kmax=0.0, pos=None, **over):
    """The oracle's forces, energy terms and virial: SPME on the workload's
    mesh, or with kmax > 0 the exact reciprocal sum over |k| <= kmax (at
    w.pos, or at pos; `over` replaces oracle parameters)."""
    p = oracle_params(w, **over)
    pos = w.pos if pos is None else pos
    if kmax > 0:
        ref = O.forces(pos, w.type, w.z, p, recip_mode=O.RECIP_EWALD, kmax=kmax)
    else:
        ref = O.forces(pos, w.type, w.z, p, recip_mode=O.RECIP_SPME, K=w.grid, order=w.order)
    if adjoint:
        rs = O.real_space(pos, w.type, w.z, p, adjoint=True)
        c = O.constants(w.type, w.z, p)
        ref["Eex_tt"] = rs["Eex_tt"]
        ref["dE_dsigma"] = rs["dE_dsigma"]
        ref["dE_da"] = rs["dE_da"] + c["dE_da_self"]
    return ref


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_bead_err(a, b):
    """Largest per-bead force error, each bead on the scale of its own force
    or, if smaller, the RMS force: max_i |a_i - b_i| / max(|b_i|, F_rms).
    A single bead off by a relative e moves this by e, where the norm above
    moves by e / sqrt(N)."""
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    fr = np.sqrt((b * b).sum(1).mean())
    d = np.linalg.norm(a - b, axis=1)
    return float((d / np.maximum(np.linalg.norm(b, axis=1), max(fr, 1e-300))).max())


def snap(pos, box):
    """Positions rounded to the nearest point of the 2^-32 L lattice of each
    edge, as the engine stores them (wrapped into [0, L))."""
    L = np.asarray(box, dtype=np.float64)
    f = np.asarray(pos, dtype=np.float64) / L
    f -= np.floor(f)
    u = np.mod(np.rint(f * 4294967296.0), 4294967296.0)
    return u / 4294967296.0 * L


def fp64_force_tol(w, ref=None, pos=None, evaluate=None):
    """Force tolerance of the FP64 engine on positions off the lattice: the
    engine computes the forces of the stored (rounded) positions, so its
    error against the oracle at the given positions is the oracle's own
    change under that rounding, plus FP64 rounding.  Returns (relative RMS
    tolerance, per-bead tolerance): twice the oracle's change in each metric
    plus 1e-12."""
    pos = w.pos if pos is None else pos
    evaluate = evaluate or (lambda x: oracle_eval(w, pos=x)["F"])
    F0 = evaluate(pos) if ref is None else ref
    F1 = evaluate(snap(pos, w.box))
    return 2.0 * rel_rms(F1, F0) + 1e-12, 2.0 * per_bead_err(F1, F0) + 1e-12


def rel(a, b, floor=1e-12):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), floor)


def energy_errors(got5, ref5):
    """Errors of [E_ex, E_real, E_recip, E_corr, E_self]: relative per term,
    except E_real, which is a sum of nearly cancelling signed pair terms and
    is measured on the electrostatic energy scale |E_real| + |E_recip| +
    |E_corr| + |E_self| (the magnitudes that make up U_elec)."""
    got5, ref5 = np.asarray(got5, dtype=float), np.asarray(ref5, dtype=float)
    err = rel(got5, ref5)
    scale = np.abs(ref5[1:5]).sum()
    if scale > 0:
        err[1] = abs(got5[1] - ref5[1]) / scale
    return err
