"""Full-size parity of the largest workloads against the FP64 oracle.

* N = 2,097,152 bulk (three species, rc = 2.5, SPME 256^3): forces on a
  random sample of beads against the oracle's real-space sum for those beads
  plus its full SPME; every energy term against the oracle's full sums; the
  mixed-precision run against the plain FP64 GPU run on all beads; and the
  electrostatic forces alone (A = 0) on a sample of charged beads, through
  the 256^3 mesh path.  Per bead, max_i |dF_i| / max(|F_i|, F_rms) is held to
  ten times the RMS tolerance.
* 256 batched replicas of uneven size and parameters: every replica's forces
  and energies against the oracle run on that replica alone.
* N = 200,000 with the polyelectrolyte workload's composition, box and mesh
  (50% charged, 40 x 40 x 50, SPME 96 x 96 x 128) as a periodic bulk box:
  sampled forces and every energy term against the oracle.
"""
import numpy as np
import pytest

import gcme_workloads as W
from oracle import oracle as O
import dataclasses

from tests.gpu_common import energy_errors, gpu_eval, make_engine, oracle_eval, oracle_params, per_bead_err, rel_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    w = W.config4()
    print(f"case {w.name} N={w.N} grid={w.grid}", flush=True)
    got = {}
    w0 = dataclasses.replace(w, A=np.zeros_like(np.asarray(w.A, dtype=np.float64)))
    for prec in ("mixed", "fp64"):
        for direct in (3, 0):  # list-free pair kernels, neighbour lists
            eng = make_engine([w], prec, tuning=dict(direct_pairs=direct))
            got[(prec, direct)] = gpu_eval(eng)
            eng.close()
            print(f"  gpu {prec} direct_pairs={direct} done", flush=True)
        eng = make_engine([w0], prec)
        got[(prec, "A0")] = gpu_eval(eng)
        eng.close()
        print(f"  gpu {prec} A=0 done", flush=True)
    p = oracle_params(w)
    idx = np.sort(np.random.default_rng(404).choice(w.N, 600, replace=False))
    rs = O.real_space(w.pos, w.type, w.z, p, sample=idx, energies=False)
    q = np.flatnonzero(w.z != 0)
    rec = O.spme_recip(w.pos[q], w.z[q], w.box, w.beta, w.lB, w.grid, w.order)
    Frec = np.zeros((w.N, 3))
    Frec[q] = rec["F"]
    F_ref = rs["F"] + Frec[idx]
    # electrostatics alone on 600 charged beads: the real-space bracket of the
    # oracle with A = 0 plus the same SPME forces
    qidx = np.sort(np.random.default_rng(405).choice(q, 600, replace=False))
    rs0 = O.real_space(w.pos, w.type, w.z, oracle_params(w0), sample=qidx, energies=False)
    F0_ref = rs0["F"] + Frec[qidx]
    print("  oracle sampled forces + SPME done", flush=True)
    full = O.real_space(w.pos, w.type, w.z, p)
    c = O.constants(w.type, w.z, p)
    E_ref = np.array([full["E_ex"], full["E_real"], rec["E_recip"], c["E_corr"], c["E_self"]])
    W_ref = full["W"] + rec["W"]
    print("  oracle energies done", flush=True)
    return w, got, idx, F_ref, E_ref, W_ref, qidx, F0_ref


@pytest.mark.parametrize("direct", [3, 0])
@pytest.mark.parametrize("precision,ftol,etol", [("fp64", 1e-9, 1e-10), ("mixed", 1e-5, 1e-6)])
def test_two_million_beads_against_oracle(big, precision, ftol, etol, direct):
    w, got, idx, F_ref, E_ref, W_ref = big[:6]
    g = got[(precision, direct)]
    ferr = rel_rms(g["force"][idx], F_ref)
    fb = per_bead_err(g["force"][idx], F_ref)
    eerr = energy_errors(g["energy"][0][:5], E_ref)
    wscale = np.linalg.norm(W_ref) + np.abs(E_ref[:3]).sum()
    werr = np.linalg.norm(g["virial"][0] - W_ref) / wscale
    print(f"  {precision} direct_pairs={direct}: sampled force {ferr:.2e} per-bead {fb:.2e} energies "
          f"{np.array2string(eerr, precision=2)} virial {werr:.2e}", flush=True)
    assert ferr < ftol
    assert fb < 10 * ftol
    assert np.all(eerr < etol), eerr
    assert werr < 10 * max(ftol, etol)


@pytest.mark.parametrize("precision,ftol", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_two_million_beads_electrostatic_forces_alone(big, precision, ftol):
    w, got, idx, F_ref, E_ref, W_ref, qidx, F0_ref = big
    F = got[(precision, "A0")]["force"][qidx]
    ferr, fb = rel_rms(F, F0_ref), per_bead_err(F, F0_ref)
    print(f"  {precision} A=0, 600 charged beads: electrostatic force {ferr:.2e} per-bead {fb:.2e}", flush=True)
    assert ferr < ftol
    assert fb < 10 * ftol


def test_two_million_beads_mixed_against_fp64(big):
    w, got, idx, F_ref, E_ref, W_ref = big[:6]
    for direct in (3, 0):
        ferr = rel_rms(got[("mixed", direct)]["force"], got[("fp64", direct)]["force"])
        print(f"  mixed vs fp64 GPU, all {w.N} beads, direct_pairs={direct}: force {ferr:.2e}", flush=True)
        assert ferr < 1e-5
    # both pair paths in FP64: the same pairs, sums in another order
    ferr = rel_rms(got[("fp64", 3)]["force"], got[("fp64", 0)]["force"])
    print(f"  list-free vs lists, FP64, all beads: force {ferr:.2e}", flush=True)
    assert ferr < 1e-12


@pytest.fixture(scope="module")
def slab_shape():
    w = W.config3()
    print(f"case {w.name} N={w.N} box={w.box} grid={w.grid}", flush=True)
    got = {}
    for prec in ("mixed", "fp64"):
        eng = make_engine([w], prec)
        got[prec] = gpu_eval(eng)
        eng.close()
        print(f"  gpu {prec} done", flush=True)
    p = oracle_params(w)
    idx = np.sort(np.random.default_rng(303).choice(w.N, 600, replace=False))
    rs = O.real_space(w.pos, w.type, w.z, p, sample=idx, energies=False)
    q = np.flatnonzero(w.z != 0)
    rec = O.spme_recip(w.pos[q], w.z[q], w.box, w.beta, w.lB, w.grid, w.order)
    Frec = np.zeros((w.N, 3))
    Frec[q] = rec["F"]
    full = O.real_space(w.pos, w.type, w.z, p)
    c = O.constants(w.type, w.z, p)
    E_ref = np.array([full["E_ex"], full["E_real"], rec["E_recip"], c["E_corr"], c["E_self"]])
    print("  oracle done", flush=True)
    return w, got, idx, rs["F"] + Frec[idx], E_ref


@pytest.mark.parametrize("precision,ftol,etol", [("fp64", 1e-9, 1e-10), ("mixed", 1e-5, 1e-6)])
def test_slab_shaped_bulk_against_oracle(slab_shape, precision, ftol, etol):
    # the polyelectrolyte workload's composition (50% charged), box 40 x 40 x 50
    # and 96 x 96 x 128 mesh, as a periodic bulk box
    w, got, idx, F_ref, E_ref = slab_shape
    g = got[precision]
    ferr = rel_rms(g["force"][idx], F_ref)
    fb = per_bead_err(g["force"][idx], F_ref)
    eerr = energy_errors(g["energy"][0][:5], E_ref)
    print(f"  {precision}: sampled force {ferr:.2e} per-bead {fb:.2e} energies {np.array2string(eerr, precision=2)}",
          flush=True)
    assert ferr < ftol
    assert fb < 10 * ftol
    assert np.all(eerr < etol), eerr
    assert rel_rms(got["mixed"]["force"], got["fp64"]["force"]) < 1e-5


@pytest.mark.parametrize("precision,ftol,etol", [("fp64", 1e-9, 1e-10), ("mixed", 1e-5, 1e-6)])
def test_256_batched_replicas_against_oracle(precision, ftol, etol):
    ws = W.config5()
    print(f"case batched R={len(ws)} N={sum(w.N for w in ws)} prec={precision}", flush=True)
    eng = make_engine(ws, precision)
    got = gpu_eval(eng)
    eng.close()
    off = 0
    worst_f, worst_e = 0.0, 0.0
    for r, w in enumerate(ws):
        ref = oracle_eval(w)
        ferr = rel_rms(got["force"][off:off + w.N], ref["F"])
        eerr = energy_errors(got["energy"][r][:5], ref["E"])
        worst_f = max(worst_f, ferr)
        worst_e = max(worst_e, float(np.max(eerr)))
        assert ferr < ftol, (r, ferr)
        assert np.all(eerr < etol), (r, eerr)
        off += w.N
    print(f"  worst replica: force {worst_f:.2e} energy {worst_e:.2e}", flush=True)
