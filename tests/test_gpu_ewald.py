"""The exact reciprocal sum (gcme_params.kmax > 0) against the oracle's own
exact k-space sum over the same wave vectors (|k| <= kmax, tin-foil, the
reciprocal term of eq. ewald), element by element.

* the plain-method configuration: N = 1536 at rho = 2.5, 20% charged,
  beta = 1, rc = 3 and the exact sum |k| <= 8, in FP64 and mixed precision;
* batched replicas, some on the exact sum and some on their mesh, each
  against the oracle in its own mode;
* steps: forces observed at the end of a run equal a fresh evaluation at the
  same positions;
* a replica with the exact sum and no charged beads.
"""
import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import energy_errors, gpu_eval, make_engine, oracle_eval, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-9, 1e-10), "mixed": (1e-5, 1e-6)}


def _cmp(got_F, got_E, got_W, ref, ftol, etol):
    ferr = rel_rms(got_F, ref["F"])
    eerr = energy_errors(got_E[:5], ref["E"])
    wscale = np.linalg.norm(ref["W"]) + np.abs(ref["E"][:3]).sum()
    werr = np.linalg.norm(got_W - ref["W"]) / wscale
    print(f"  force {ferr:.2e} energy {np.array2string(eerr, precision=2)} virial {werr:.2e}", flush=True)
    assert ferr < ftol
    assert np.all(eerr < etol), eerr
    assert werr < 10 * max(ftol, etol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plain_method_exact_sum(precision):
    w = W.config1()
    print(f"case {w.name} exact k-sum |k| <= {w.kmax} prec={precision}", flush=True)
    eng = make_engine([w], precision, kmax=[w.kmax])
    got = gpu_eval(eng)
    eng.close()
    ref = oracle_eval(w, kmax=w.kmax)
    _cmp(got["force"], got["energy"][0], got["virial"][0], ref, *TOL[precision])
    # the electrostatic forces alone (the GCM forces are far larger)
    from oracle import oracle as O
    from tests.gpu_common import oracle_params
    p0 = oracle_params(w, A=np.zeros_like(w.A))
    ref_el = O.forces(w.pos, w.type, w.z, p0, recip_mode=O.RECIP_EWALD, kmax=w.kmax)
    eng = make_engine([w], precision, kmax=[w.kmax])
    from paper_2403_08148_amd import params_from_workload
    eng.set_params(params_from_workload(w, A=np.zeros_like(w.A), kmax=w.kmax))
    el = gpu_eval(eng)
    eng.close()
    ferr = rel_rms(el["force"], ref_el["F"])
    print(f"  electrostatic forces alone: {ferr:.2e}", flush=True)
    assert ferr < TOL[precision][0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_exact_and_mesh(precision):
    ws = [W.small_bulk(N=520, seed=21, charged_frac=0.3, box=(6.1, 6.0, 5.9), rc=2.5, grid=(24, 24, 24)),
          W.small_bulk(N=901, seed=22, charged_frac=0.2, a_types=(0.35, 0.6), box=(7.1, 7.4, 6.6), rc=2.5,
                       grid=(24, 24, 24)),
          W.small_bulk(N=700, seed=23, charged_frac=0.25, box=(6.6, 7.0, 6.4), rc=2.5, grid=(24, 27, 24)),
          W.small_bulk(N=300, seed=24, charged_frac=0.0, box=(5.2, 5.2, 5.2), rc=2.5, grid=(16, 16, 16))]
    kmax = [7.0, 0.0, 6.0, 5.0]
    print(f"case batched exact/mesh {[w.N for w in ws]} kmax={kmax} prec={precision}", flush=True)
    eng = make_engine(ws, precision, kmax=kmax)
    got = gpu_eval(eng)
    eng.close()
    off = 0
    for r, w in enumerate(ws):
        ref = oracle_eval(w, kmax=kmax[r])
        sl = slice(off, off + w.N)
        off += w.N
        print(f" replica {r} N={w.N} kmax={kmax[r]}", flush=True)
        _cmp(got["force"][sl], got["energy"][r], got["virial"][r], ref, *TOL[precision])
    # no charged beads: no reciprocal energy
    assert got["energy"][3][2] == 0.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_sum_in_steps(precision):
    w = W.small_bulk(N=640, seed=25, charged_frac=0.3, box=(6.3, 6.3, 6.3), rc=2.5, grid=(24, 24, 24))
    print(f"case exact k-sum steps prec={precision}", flush=True)
    eng = make_engine([w], precision, seed=3, kmax=[6.5])
    obs = eng.step(8, observe=True)
    eng.sync()
    F_run = obs["force"].cpu().numpy()
    E_run = obs["energy"].cpu().numpy()[0]
    pos, _, step = eng.get_state()
    assert step == 8
    again = gpu_eval(eng)
    eng.close()
    ferr = rel_rms(F_run.T, again["force"])
    print(f"  run vs fresh evaluation: force {ferr:.2e}", flush=True)
    assert ferr < (1e-12 if precision == "fp64" else 1e-6)
    np.testing.assert_allclose(E_run[:5], again["energy"][0][:5], rtol=1e-10 if precision == "fp64" else 1e-6,
                               atol=1e-9)
    # and the oracle at the final positions
    w.pos = pos.cpu().numpy().T.copy()
    ref = oracle_eval(w, kmax=6.5)
    _cmp(again["force"], again["energy"][0], again["virial"][0], ref, *TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_all_reciprocal_limit(precision):
    # Every bead with the same smearing radius a: beta = alpha = sqrt(pi)/(2a)
    # (G = a/sqrt(pi)) makes the real-space bracket vanish (up to the
    # rounding of alpha against beta), and
    # the whole smeared Coulomb energy sits in the reciprocal sum (here exact,
    # |k| <= 17: exp(-k^2/(4 beta^2)) < 1e-20 beyond it).
    a = 0.5
    beta = np.sqrt(np.pi) / (2.0 * a)
    w = W.small_bulk(N=420, seed=26, charged_frac=0.3, a_types=(a,), box=(6.0, 6.2, 5.8), rc=2.5,
                     beta=beta, grid=(24, 24, 24))
    print(f"case all-reciprocal beta = alpha = {beta:.6f} prec={precision}", flush=True)
    eng = make_engine([w], precision, kmax=[17.0])
    got = gpu_eval(eng)
    eng.close()
    # E_real: zero up to the rounding of alpha against beta
    scale = np.abs(got["energy"][0][2:5]).sum()
    assert abs(got["energy"][0][1]) < 1e-12 * scale
    ref = oracle_eval(w, kmax=17.0)
    _cmp(got["force"], got["energy"][0], got["virial"][0], ref, *TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_all_reciprocal_flag(precision):
    # GCME_FLAG_ALL_RECIPROCAL sets beta = sqrt(pi)/(2a) itself and skips the
    # real-space electrostatic pairs: E_real is exactly zero, and forces and
    # energies agree with the explicit beta = alpha run (whose real-space
    # term is the rounding of alpha - beta) and with the oracle.
    from paper_2403_08148_amd import GCMe, params_from_workload
    from paper_2403_08148_amd._binding import GCMeError, GCME_FLAG_ALL_RECIPROCAL
    a = 0.5
    beta = np.sqrt(np.pi) / (2.0 * a)
    w = W.small_bulk(N=420, seed=26, charged_frac=0.3, a_types=(a,), box=(6.0, 6.2, 5.8), rc=2.5,
                     beta=beta, grid=(24, 24, 24))
    print(f"case all-reciprocal flag prec={precision}", flush=True)
    eng = make_engine([w], precision, kmax=[17.0])
    ref_gpu = gpu_eval(eng)
    eng.set_params(params_from_workload(w, beta=3.0, kmax=17.0, flags=GCME_FLAG_ALL_RECIPROCAL))
    got = gpu_eval(eng)
    assert got["energy"][0][1] == 0.0
    ferr = rel_rms(got["force"], ref_gpu["force"])
    print(f"  flag vs explicit beta = alpha: force {ferr:.2e}", flush=True)
    assert ferr < (1e-13 if precision == "fp64" else 1e-6)
    np.testing.assert_allclose(got["energy"][0][2:5], ref_gpu["energy"][0][2:5], rtol=1e-12)
    _cmp(got["force"], got["energy"][0], got["virial"][0], oracle_eval(w, kmax=17.0), *TOL[precision])
    # dE/da is not provided under the flag; unequal radii are rejected
    with pytest.raises(GCMeError):
        eng.forces_energy(adjoint=True)
    eng.close()
    w2 = W.small_bulk(N=300, seed=27, charged_frac=0.3, a_types=(0.4, 0.6), box=(6.0, 6.0, 6.0), rc=2.5,
                      grid=(24, 24, 24))
    e2 = GCMe([w2.N], precision=precision)
    with pytest.raises(GCMeError):
        e2.set_params(params_from_workload(w2, flags=GCME_FLAG_ALL_RECIPROCAL))
    e2.close()
