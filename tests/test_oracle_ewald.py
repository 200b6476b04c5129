"""Pins of the oracle's long-range terms (eq. ewald) against facts fixed
outside the oracle:

* point-charge limit: rock-salt and CsCl lattices with tiny smearing radius
  reproduce the textbook Madelung constants (fixes the prefactors and signs of
  U_recip, U_corr and the real-space bracket together);
* two opposite charges in a cubic box: the Ewald energy equals the isolated
  smeared pair + Born self energies minus the tin-foil dipole term
  2 pi lB r^2 /(3 L^3), up to O(r^4/L^5);
* the total is independent of the splitting parameter beta (converged sums),
  and G = a/sqrt(pi) (beta = alpha) makes the real-space bracket vanish;
* forces and the reciprocal virial are minus derivatives of the energy;
* the mesh transform agrees with numpy's FFT; B-splines have unit partition
  and unit integral; SPME converges to the exact k-sum as the mesh refines.
"""
import json
import math
import os

import numpy as np
import pytest

import gcme_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _P(box, rc, beta, lB, A, sigma, a):
    from oracle.oracle import Params
    return Params(box, rc, beta, lB, np.atleast_2d(A), np.atleast_1d(sigma), np.atleast_1d(a))


def _elec_total(oracle, pos, typ, z, p, kmax, images=False):
    if images:
        rs = oracle.real_space_images(pos, typ, z, p)
    else:
        rs = oracle.real_space(pos, typ, z, p, use_cells=False)
    rec = oracle.ewald_recip(pos, z, p.box, p.beta, p.lB, kmax)
    c = oracle.constants(typ, z, p)
    return rs["E_real"] + rec["E_recip"] + c["E_corr"] + c["E_self"], rs, rec, c


@pytest.mark.parametrize("lattice", ["NaCl", "CsCl"])
def test_madelung_point_charge_limit(oracle, lattice):
    with open(os.path.join(GOLDEN, "madelung.json")) as f:
        gold = json.load(f)
    if lattice == "NaCl":
        pos, z, box = W.rock_salt(2, r0=1.0)
        r0 = 1.0
    else:
        pos, z, box = W.cesium_chloride(3, a0=1.0)
        r0 = math.sqrt(3) / 2
    M = gold[lattice]["M"]
    N = len(z)
    a = 0.05 * r0
    typ = np.zeros(N, np.int32)
    beta = 6.0 / (box[0] / 2)       # erfc(beta L/2) ~ 2e-17
    kmax = 2 * beta * 6.2           # exp(-k^2/4beta^2) ~ 2e-17
    p = _P(box, box[0] / 2, beta, 1.0, [[0.0]], [0.5], [a])
    E, rs, rec, c = _elec_total(oracle, pos, typ, z, p, kmax)
    assert E - c["E_self"] == pytest.approx(-M * N / (2 * r0), rel=1e-9)


def test_dipole_in_cubic_box(oracle):
    # residual = E_ewald + 2 pi lB r^2/(3 L^3) - u_elec(r) - U_self = O(r^4/L^5)
    a = 0.5
    res = []
    for L in (8.0, 16.0, 32.0):
        pos = np.array([[1.0, 1.2, 0.9], [1.0 + 0.6, 1.2 + 0.5, 0.9 + 0.3]])
        r = np.linalg.norm(pos[1] - pos[0])
        z = np.array([1, -1])
        typ = np.zeros(2, np.int32)
        beta = 6.0 / (L / 2)
        p = _P((L, L, L), L / 2, beta, 1.0, [[0.0]], [0.5], [a])
        E, _, _, c = _elec_total(oracle, pos, typ, z, p, 2 * beta * 6.2)
        u = oracle.u_elec(r, 1.0, -1.0, math.sqrt(2) * a)
        res.append(E + 2 * math.pi * r * r / (3 * L ** 3) - u - c["E_self"])
    # each doubling of L must shrink the residual by ~2^5
    assert abs(res[0]) < 1e-3
    assert 20 < abs(res[0] / res[1]) < 50
    assert 20 < abs(res[1] / res[2]) < 50


def test_beta_invariance_and_all_reciprocal_limit(oracle):
    w = W.small_bulk(N=60, seed=5, charged_frac=1.0, a_types=(0.5,), box=(5.0, 5.0, 5.0), rc=2.5)
    a = 0.5
    alpha = math.sqrt(math.pi / 2) / (math.sqrt(2) * a)
    totals = []
    for beta in (0.8, 1.0, 1.2, alpha):
        rc = 6.2 / beta            # erfc(beta rc) ~ 1e-18, beyond L/2: image sum
        p = _P(w.box, rc, beta, 1.0, w.A, w.sigma, w.a)
        E, rs, rec, c = _elec_total(oracle, w.pos, w.type, w.z, p, 2 * beta * 6.2, images=True)
        totals.append(E)
        if beta == alpha:
            # G = a_ij/sqrt(pi): the real-space bracket vanishes identically
            assert abs(rs["E_real"]) < 1e-12 * abs(E)
    np.testing.assert_allclose(totals, totals[0], rtol=1e-11)


def test_ewald_forces_and_virial_are_derivatives(oracle):
    w = W.small_bulk(N=90, seed=8, charged_frac=0.6, box=(6.0, 6.5, 5.5), rc=2.5)
    kmax = 9.0
    rec = oracle.ewald_recip(w.pos, w.z, w.box, w.beta, w.lB, kmax)
    h = 1e-5
    rng = np.random.default_rng(2)
    for i in rng.choice(np.nonzero(w.z)[0], 5, replace=False):
        for k in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[i, k] += h
            pm[i, k] -= h
            fd = -(oracle.ewald_recip(pp, w.z, w.box, w.beta, w.lB, kmax)["E_recip"]
                   - oracle.ewald_recip(pm, w.z, w.box, w.beta, w.lB, kmax)["E_recip"]) / (2 * h)
            assert rec["F"][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    np.testing.assert_allclose(rec["F"].sum(0), 0.0, atol=1e-10)
    # virial: the k-set must not change under the strain, so scale kmax too
    for k in range(3):
        es = []
        for s in (+h, -h):
            sc = np.ones(3)
            sc[k] += s
            box = tuple(np.asarray(w.box) * sc)
            # k-vectors are n/L: keep the same integer set by enumerating with
            # the strained box and a kmax large enough to hold it unchanged
            es.append(oracle.ewald_recip(w.pos * sc, w.z, box, w.beta, w.lB, 60.0)["E_recip"])
        full = oracle.ewald_recip(w.pos, w.z, w.box, w.beta, w.lB, 60.0)
        assert full["W"][k] == pytest.approx(-(es[0] - es[1]) / (2 * h), rel=1e-6)


@pytest.mark.parametrize("n", [2, 3, 8, 12, 16, 18, 27, 30, 64, 96, 100, 243, 256])
def test_fft_matches_numpy(oracle, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    np.testing.assert_allclose(oracle.fft(x, -1), np.fft.fft(x), rtol=1e-12, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.fft(x, +1), np.fft.ifft(x) * n, rtol=1e-12, atol=1e-12 * n)


@pytest.mark.parametrize("p", [3, 4, 5, 6, 8])
def test_bspline_properties(oracle, p):
    from scipy import integrate
    for t in (0.0, 0.13, 0.5, 0.77, 0.999):
        assert sum(oracle.bspline(p, t + j) for j in range(p)) == pytest.approx(1.0, abs=1e-14)
        # symmetric about p/2
        assert oracle.bspline(p, t + 1) == pytest.approx(oracle.bspline(p, p - t - 1), abs=1e-14)
    val, _ = integrate.quad(lambda x: oracle.bspline(p, x), 0, p, points=list(range(1, p)))
    assert val == pytest.approx(1.0, abs=1e-12)
    # moduli = |DFT of the spline samples M_p(1..p-1)|^2 (numpy's FFT)
    K = 24
    samples = np.zeros(K)
    for k in range(p - 1):
        samples[k] = oracle.bspline(p, k + 1)
    ref = np.abs(np.fft.fft(samples)) ** 2
    got = oracle.bspline_moduli(K, p)
    mask = ref > 1e-7
    np.testing.assert_allclose(got[mask], ref[mask], rtol=1e-12)
    if p % 2 == 1:
        # odd order: the modulus vanishes at the Nyquist index and is replaced
        # by the mean of its neighbours
        assert ref[K // 2] < 1e-20
        assert got[K // 2] == pytest.approx(0.5 * (ref[K // 2 - 1] + ref[K // 2 + 1]))


def test_spme_converges_to_exact_sum(oracle):
    w = W.small_bulk(N=400, seed=9, charged_frac=0.5, box=(7.0, 7.5, 8.0), rc=3.0, beta=1.0)
    ex = oracle.ewald_recip(w.pos, w.z, w.box, w.beta, w.lB, 12.4)
    errsE, errsF = [], []
    for K in (16, 32, 64):
        sp = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, (K, K, K), 6)
        errsE.append(abs(sp["E_recip"] - ex["E_recip"]) / abs(ex["E_recip"]))
        errsF.append(np.linalg.norm(sp["F"] - ex["F"]) / np.linalg.norm(ex["F"]))
    assert errsE[2] < 1e-7 and errsF[2] < 1e-6
    assert errsF[0] > errsF[1] > errsF[2]
    # higher order at fixed mesh also converges
    e4 = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, (24, 24, 24), 4)
    e8 = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, (24, 24, 24), 8)
    assert np.linalg.norm(e8["F"] - ex["F"]) < 0.2 * np.linalg.norm(e4["F"] - ex["F"])
    # the SPME virial tends to the exact one
    sp = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, (64, 64, 64), 6)
    np.testing.assert_allclose(sp["W"], ex["W"], rtol=1e-6, atol=1e-6 * abs(ex["E_recip"]))


def test_spme_forces_and_virial_are_derivatives(oracle):
    w = W.small_bulk(N=150, seed=12, charged_frac=0.6, box=(6.0, 6.2, 5.8), rc=2.5)
    K, p = (20, 18, 24), 5
    sp = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, K, p)
    h = 1e-5
    for i in np.nonzero(w.z)[0][:4]:
        for k in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[i, k] += h
            pm[i, k] -= h
            fd = -(oracle.spme_recip(pp, w.z, w.box, w.beta, w.lB, K, p)["E_recip"]
                   - oracle.spme_recip(pm, w.z, w.box, w.beta, w.lB, K, p)["E_recip"]) / (2 * h)
            assert sp["F"][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for k in range(3):
        es = []
        for s in (+h, -h):
            sc = np.ones(3)
            sc[k] += s
            es.append(oracle.spme_recip(w.pos * sc, w.z, tuple(np.asarray(w.box) * sc), w.beta, w.lB, K, p)[
                "E_recip"])
        assert sp["W"][k] == pytest.approx(-(es[0] - es[1]) / (2 * h), rel=1e-6)


def test_config1_exact_vs_spme_method_error(oracle):
    # the GPU uses SPME 32^3 order 5 for the first configuration; the
    # oracle's own SPME-vs-exact difference there is the method error
    w = W.config1()
    ex = oracle.ewald_recip(w.pos, w.z, w.box, w.beta, w.lB, w.kmax)
    sp = oracle.spme_recip(w.pos, w.z, w.box, w.beta, w.lB, w.grid, w.order)
    assert ex["n_kvec_half"] == 2688      # 5376 wave vectors with |k| <= 8
    assert abs(sp["E_recip"] - ex["E_recip"]) / abs(ex["E_recip"]) < 1e-4
    assert np.linalg.norm(sp["F"] - ex["F"]) / np.linalg.norm(ex["F"]) < 1e-3
