"""Equation of state of the neutral GCM fluid from the engine's own MD
(section "Parametrization": eq. pres_virial, eq. pres_approx and Fig.
water_p_excess_vs_rho): a physics check of the excluded-volume forces and
virial at scale.

omega = (p - rho kT)/(A rho^2), with the excess pressure from the virial,
<sum_pairs r_ij . f_ij>/(3V) (eq. pres_virial; the ideal part rho kT is the
thermostat's, so the kinetic temperature's O(dt^2) BAOAB bias does not
enter).

* Parity: at four (rho, A) state points omega equals the FP64 oracle's own
  MD value (tests/golden/eos_oracle.json, written by eos_oracle.py beside
  it) within 5 combined standard errors.
* The scan over rho = 2..6 and A = 15, 25, 35: omega stays below the
  mean-field value 1/2 (A rho^2/2 is the excess pressure of uncorrelated
  beads: eq. u_ex integrates to A) and rises towards it with rho and with
  A; at fixed rho the excess pressure over A is one master curve, within
  2% across A (Fig. water_p_excess_vs_rho a); at rho = 6 omega is within 2%
  of the paper's large-rho plateau 0.499 (Fig. water_p_excess_vs_rho b).
"""
import json
import os

import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import make_engine

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "eos_oracle.json")
PAPER_PLATEAU = 0.499  # Fig. water_p_excess_vs_rho b, section "Parametrization"


def _omega(rho, A, precision="mixed", proto=None):
    """omega and its block error by the oracle reference's protocol."""
    pr = proto or json.load(open(GOLDEN))["protocol"]
    N = pr["N"]
    L = (N / rho) ** (1.0 / 3.0)
    w = W.small_bulk(N=N, seed=pr["seed"], charged_frac=0.0, a_types=(pr["a"],), A=[[A]], rc=pr["rc"],
                     grid=(16, 16, 16), box=(L, L, L))
    V = L ** 3
    eng = make_engine([w], precision, seed=pr["noise_seed"])
    eng.step(pr["equil"])
    eng.sync()
    om, T = [], []
    for _ in range(pr["nobs"]):
        obs = eng.step(pr["gap"], observe=True)
        eng.sync()
        Wv = obs["virial"].cpu().numpy()[0]
        om.append((Wv[0] + Wv[1] + Wv[2]) / (3.0 * V) / (A * rho * rho))
        T.append(2.0 * obs["energy"].cpu().numpy()[0][6] / (3.0 * N))
    eng.close()
    om = np.array(om)
    blocks = om.reshape(pr["blocks"], -1).mean(1)
    return float(om.mean()), float(blocks.std(ddof=1) / np.sqrt(pr["blocks"])), float(np.mean(T))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_gcm_eos_matches_oracle_md(precision):
    ref = json.load(open(GOLDEN))
    print(f"case GCM EOS against the oracle's MD, prec={precision}", flush=True)
    for st in ref["states"]:
        om, err, T = _omega(st["rho"], st["A"], precision, ref["protocol"])
        tol = 5.0 * np.hypot(err, st["err"])
        print(f"  A {st['A']:.0f} rho {st['rho']}: engine {om:.5f} +- {err:.5f}, oracle {st['omega']:.5f} +- "
              f"{st['err']:.5f}; <T> {T:.4f}", flush=True)
        assert abs(om - st["omega"]) < tol
        assert abs(T - 1.0) < 0.03


def test_gcm_eos_density_scan():
    print("case GCM EOS scan, rho 2..6, A 15/25/35", flush=True)
    rhos, As = (2.0, 2.5, 3.0, 4.0, 5.0, 6.0), (15.0, 25.0, 35.0)
    om = np.zeros((len(As), len(rhos)))
    er = np.zeros_like(om)
    for a, A in enumerate(As):
        for r, rho in enumerate(rhos):
            om[a, r], er[a, r], _ = _omega(rho, A)
            print(f"  A {A:.0f} rho {rho}: omega {om[a, r]:.5f} +- {er[a, r]:.5f}", flush=True)
    assert np.all(om < 0.5)
    assert np.all(np.diff(om, axis=1) > 0)          # rises with rho
    assert np.all(np.diff(om, axis=0) > 0)          # and with A
    excess_over_A = om * np.asarray(rhos) ** 2      # (p - rho kT)/A
    spread = excess_over_A.max(0) / excess_over_A.min(0) - 1.0
    print(f"  master curve: largest spread over A {spread.max():.4f}", flush=True)
    assert np.all(spread < 0.02)
    assert np.all(np.abs(om[:, -1] / PAPER_PLATEAU - 1.0) < 0.02)


def test_gcm_rdf_first_peak():
    """The radial distribution function of the same fluid at rho = 2.5 has its
    first maximum near 0.8 d: the separation the paper takes as the bond
    length b = 0.8 d because the RDF of the neutral GCMe fluid peaks there.
    g(r) from 30 snapshots of the engine's MD, histogrammed on the host."""
    from scipy.spatial import cKDTree
    rho, N = 2.5, 4000
    L = (N / rho) ** (1.0 / 3.0)
    w = W.small_bulk(N=N, seed=33, charged_frac=0.0, a_types=(0.5,), A=[[25.0]], rc=3.0, grid=(16, 16, 16),
                     box=(L, L, L))
    print(f"case GCM RDF, N = {N}, rho = {rho}", flush=True)
    eng = make_engine([w], "mixed", seed=9)
    eng.step(600)
    dr, rmax = 0.02, 2.0
    hist = np.zeros(int(rmax / dr))
    for _ in range(30):
        eng.step(25)
        pos, _, _ = eng.get_state()
        p = np.mod(pos.cpu().numpy().T, L)
        d = cKDTree(p, boxsize=L).sparse_distance_matrix(cKDTree(p, boxsize=L), rmax, output_type="ndarray")["v"]
        hist += np.histogram(d[d > 0], bins=len(hist), range=(0.0, rmax))[0]
    eng.close()
    r = (np.arange(len(hist)) + 0.5) * dr
    shell = 4.0 * np.pi * r * r * dr
    g = hist / (30 * N * rho * shell)
    k = int(np.argmax(g))
    print(f"  first maximum g({r[k]:.2f}) = {g[k]:.3f}; g(0.1) = {g[5]:.3f}; g(1.8) = {g[90]:.3f}", flush=True)
    assert 0.7 <= r[k] <= 0.9
    assert g[k] > 1.05 and g[5] < 0.5
    assert abs(g[85:].mean() - 1.0) < 0.1
