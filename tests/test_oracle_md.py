"""Pins of the oracle's integrators and noise generator.

* Philox4x64-10 equals numpy's ``Philox`` bit generator (a library routine
  implementing the same published generator); numpy returns the block of
  counter + 1 first.
* The Gaussian transform has zero mean, unit variance and Gaussian kurtosis.
* Velocity Verlet conserves the total energy with an error that falls as
  dt^2 (second-order integrator), at the paper's soft-core step sizes.
* BAOAB Langevin holds the kinetic temperature at kT (paper: Langevin NVT).
"""
import numpy as np
import pytest

import gcme_workloads as W


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 7, 11, 13), (123, 456)),
                                      ((2**64 - 2, 2**63, 1, 99), (2**64 - 1, 42))])
def test_philox_matches_numpy(oracle, ctr, key):
    g = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    raw = g.random_raw(4)
    c = list(ctr)
    c[0] = (c[0] + 1) % 2**64
    np.testing.assert_array_equal(oracle.philox4x64_10(c, key), raw)


def test_gauss_moments(oracle):
    xs = np.array([oracle.gauss3(7, s, i, 0) for s in range(40) for i in range(500)]).ravel()
    assert abs(xs.mean()) < 4 / np.sqrt(len(xs))
    assert abs(xs.var() - 1) < 4 * np.sqrt(2 / len(xs))
    k = ((xs - xs.mean()) ** 4).mean() / xs.var() ** 2
    assert abs(k - 3) < 4 * np.sqrt(24 / len(xs))
    # keyed: a different bead id gives different noise
    assert not np.allclose(oracle.gauss3(7, 3, 1, 0), oracle.gauss3(7, 3, 2, 0))


def _md(oracle, w, dt, n, gamma=0.0):
    from oracle.oracle import Params, RECIP_SPME
    p = Params(w.box, w.rc, w.beta, w.lB, w.A, w.sigma, w.a)
    ids = np.arange(w.N, dtype=np.int32)
    return oracle.md(w.pos, w.vel, w.type, w.z, ids, p, w.mass, dt, gamma, 1.0, 17, 0, 0, n,
                     recip_mode=RECIP_SPME, K=w.grid, order=w.order)


def test_velocity_verlet_energy_drift_second_order(oracle):
    w = W.small_bulk(N=250, seed=31, charged_frac=0.3, box=(4.7, 4.6, 4.8), rc=2.2, grid=(16, 16, 16))
    drifts = []
    for dt in (0.02, 0.01):
        n = int(round(0.4 / dt))
        _, _, _, E = _md(oracle, w, dt, n)
        tot = E[:, 0] + E[:, 1]
        drifts.append(np.max(np.abs(tot - tot[0])))
    # halving dt cuts the energy fluctuation ~4x; allow 2.8x..5.5x
    assert 2.8 < drifts[0] / drifts[1] < 5.5
    # from random positions ~2000 kT of potential energy turns kinetic in 0.4 tau
    assert drifts[0] < 1e-2 * abs(E[0, 0])


def test_baoab_temperature(oracle):
    w = W.small_bulk(N=200, seed=32, charged_frac=0.3, box=(4.3, 4.3, 4.3), rc=2.1, grid=(16, 16, 16))
    # random start releases heat; the thermostat needs ~6 tau to remove it
    _, _, _, E = _md(oracle, w, 0.02, 1500, gamma=1.0)
    ke = E[300:, 1]
    T = 2 * ke.mean() / (3 * w.N)
    assert abs(T - 1.0) < 0.05
