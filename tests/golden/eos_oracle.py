"""Reference values of the GCM equation of state from the FP64 oracle's own
molecular dynamics, for tests/test_gpu_eos.py.  Calls only oracle/.

The quantity is the paper's omega of eq. pres_approx, (p - rho kT)/(A rho^2),
with the excess pressure from the virial of eq. pres_virial,
p - rho kT = <sum_pairs r_ij . f_ij> / (3V), for the neutral GCM fluid
(a = sigma = 0.5, one species) at a few (rho, A) state points of the
paper's Fig. water_p_excess_vs_rho (section "Parametrization").

Protocol, shared with the GPU test: N = 4000 beads, uniform random start
(gcme_workloads.small_bulk, seed 31), BAOAB Langevin at kT = 1, gamma = 1,
dt = 0.02 (Philox noise, seed 7), rc = 3; 800 steps of equilibration, then
80 observations 25 steps apart; omega from the mean virial, its error from
10 block means.

Run:  python tests/golden/eos_oracle.py   (writes eos_oracle.json beside it)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gcme_workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

N, SEED, NOISE_SEED = 4000, 31, 7
EQUIL, NOBS, GAP, NBLOCKS = 800, 80, 25, 10
STATES = [(25.0, 2.5), (25.0, 5.0), (15.0, 2.0), (35.0, 3.0)]  # (A, rho)


def state_workload(rho, A):
    L = (N / rho) ** (1.0 / 3.0)
    return W.small_bulk(N=N, seed=SEED, charged_frac=0.0, a_types=(0.5,), A=[[A]], rc=3.0, grid=(16, 16, 16),
                        box=(L, L, L))


def omega(rho, A):
    w = state_workload(rho, A)
    p = O.Params(w.box, w.rc, w.beta, w.lB, w.A, w.sigma, w.a)
    V = float(np.prod(w.box))
    ids = np.arange(N, dtype=np.int32)
    pos, vel = w.pos, w.vel
    step = 0

    def run(n):
        nonlocal pos, vel, step
        pos, vel, _, _ = O.md(pos, vel, w.type, w.z, ids, p, w.mass, w.dt, w.gamma, w.kT, NOISE_SEED, 0, step, n,
                              recip_mode=O.RECIP_NONE)
        step += n

    run(EQUIL)
    om = []
    for _ in range(NOBS):
        run(GAP)
        Wv = O.forces(pos, w.type, w.z, p, recip_mode=O.RECIP_NONE)["W"]
        om.append((Wv[0] + Wv[1] + Wv[2]) / (3.0 * V) / (A * rho * rho))
    om = np.array(om)
    blocks = om.reshape(NBLOCKS, -1).mean(1)
    return float(om.mean()), float(blocks.std(ddof=1) / np.sqrt(NBLOCKS))


def main():
    O.build(force=False)
    out = {"protocol": dict(N=N, seed=SEED, noise_seed=NOISE_SEED, equil=EQUIL, nobs=NOBS, gap=GAP, blocks=NBLOCKS,
                            dt=0.02, gamma=1.0, kT=1.0, rc=3.0, a=0.5),
           "states": []}
    for A, rho in STATES:
        t0 = time.time()
        om, err = omega(rho, A)
        print(f"A {A} rho {rho}: omega {om:.5f} +- {err:.5f} ({time.time() - t0:.0f} s)", flush=True)
        out["states"].append(dict(A=A, rho=rho, omega=om, err=err))
    with open(os.path.join(HERE, "eos_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
