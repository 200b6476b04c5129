"""Pins of the oracle's pair terms against facts fixed by the paper and by
mathematics, independent of the oracle's own formulas:

* eq. u_ex is the overlap integral A * int rho_i rho_j of two normalised
  Gaussian mass densities (eq. mass_distribution; SI derivation): checked by
  numerical quadrature of that overlap, and by int u_ex d^3r = A.
* eq. u_elec is the Coulomb energy of two Gaussian charge clouds
  (eq. charge_distribution); the SI derivation reduces it to a 1D Fourier
  integral, evaluated here by quadrature.  Limits r -> 0, r -> inf, and the
  Born self energy (SI "Limits", eq. self_energy) are the paper's statements.
* real-space sums: cell list == brute force; forces == -grad E (central
  differences); virial diagonal == -dE/d(strain); zero net force.
* parameter derivatives: dE/dA * A == E per type pair (E is linear in A);
  dE/dsigma, dE/da by central differences.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import gcme_workloads as W


def test_u_ex_is_overlap_of_gaussian_mass_densities(oracle):
    # u_ex(r) = A int rho_i(x) rho_j(x - r) d^3x with rho the normalised
    # Gaussian (3/(2 pi s^2))^{3/2} exp(-3 x^2/(2 s^2)).  In cylindrical
    # coordinates around the axis through both centres this is a 2D integral.
    A = 25.0
    for si, sj, r in [(0.5, 0.5, 0.0), (0.5, 0.5, 0.7), (0.3, 0.7, 1.1), (0.4, 0.6, 2.0)]:
        def rho(s, d2):
            return (3.0 / (2 * math.pi * s * s)) ** 1.5 * math.exp(-3.0 * d2 / (2 * s * s))

        def integrand(rho_c, zc):
            return 2 * math.pi * rho_c * rho(si, rho_c ** 2 + zc ** 2) * rho(sj, rho_c ** 2 + (zc - r) ** 2)

        val, _ = integrate.dblquad(integrand, -8, 8 + r, 0, 8, epsabs=1e-13, epsrel=1e-11)
        assert oracle.u_ex(r, A, si * si + sj * sj) == pytest.approx(A * val, rel=1e-8)


def test_u_ex_integrates_to_A(oracle):
    for A, s2 in [(25.0, 0.5), (15.0, 0.18), (35.0, 0.98)]:
        val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.u_ex(r, A, s2), 0, 40,
                                epsabs=1e-13, epsrel=1e-12)
        assert val == pytest.approx(A, rel=1e-10)


def test_u_elec_matches_fourier_integral(oracle):
    # SI derivation: u = (2 lB zz / (pi r)) int_0^inf sin(k r)/k exp(-a^2 k^2/(2 pi)) dk
    lB = 1.3
    for aij, r, zz in [(0.707, 0.3, 1.0), (0.5, 1.0, -1.0), (0.9, 2.5, 1.0), (0.42, 0.05, -1.0)]:
        f = lambda k: math.exp(-aij * aij * k * k / (2 * math.pi)) / k if k > 0 else r
        val, _ = integrate.quad(f, 0, 200, weight="sin", wvar=r, limit=500)
        expect = 2 * lB * zz / (math.pi * r) * val
        assert oracle.u_elec(r, lB, zz, aij) == pytest.approx(expect, rel=1e-9)


def test_u_elec_limits(oracle):
    lB, aij = 0.8, 0.6
    # contact value lB zz sqrt(2)/a_ij, i.e. z z e^2 /(2^{3/2} pi eps a_ij)
    assert oracle.u_elec(0.0, lB, 1.0, aij) == pytest.approx(lB * math.sqrt(2) / aij, rel=1e-14)
    assert oracle.u_elec(1e-7, lB, 1.0, aij) == pytest.approx(lB * math.sqrt(2) / aij, rel=1e-10)
    # far field and point-charge limit: Coulomb lB zz / r
    assert oracle.u_elec(30.0, lB, -1.0, aij) == pytest.approx(-lB / 30.0, rel=1e-14)
    assert oracle.u_elec(1.0, lB, 1.0, 1e-4) == pytest.approx(lB, rel=1e-14)
    # Born self energy z^2 lB/(2 a) = 1/2 u_elec(r -> 0) with a_ii = sqrt(2) a
    a = 0.45
    assert 0.5 * oracle.u_elec(0.0, lB, 1.0, math.sqrt(2) * a) == pytest.approx(lB / (2 * a), rel=1e-14)


def test_real_bracket_is_difference_of_two_smeared_couplings(oracle):
    # The real-space bracket of eq. ewald pairs the smeared charge (width a_ij)
    # against a Gaussian screening cloud: with G = 1/(sqrt2 beta) the second
    # erf is u_elec at an effective width a = sqrt(pi/2)/beta.
    alpha, beta = 1.7725, 1.1
    a_eff = math.sqrt(math.pi / 2) / beta
    a_ij = math.sqrt(math.pi / 2) / alpha
    for r in [0.01, 0.3, 1.0, 2.7]:
        expect = oracle.u_elec(r, 1.0, 1.0, a_ij) - oracle.u_elec(r, 1.0, 1.0, a_eff)
        assert oracle.phi_real(r, alpha, beta) == pytest.approx(expect, rel=1e-12, abs=1e-15)
    # r -> 0 limit: (2/sqrt(pi)) (alpha - beta)
    assert oracle.phi_real(0.0, alpha, beta) == pytest.approx(2 / math.sqrt(math.pi) * (alpha - beta))


def _params(w, rc=None, beta=None):
    from oracle.oracle import Params
    return Params(w.box, w.rc if rc is None else rc, w.beta if beta is None else beta, w.lB,
                  w.A, w.sigma, w.a)


def test_cells_equal_brute_force(oracle):
    w = W.small_bulk(N=700, seed=3, box=(8.2, 9.0, 7.6), rc=2.5)
    p = _params(w)
    b = oracle.real_space(w.pos, w.type, w.z, p, use_cells=False, adjoint=True)
    c = oracle.real_space(w.pos, w.type, w.z, p, use_cells=True, adjoint=True)
    np.testing.assert_allclose(c["F"], b["F"], rtol=1e-12, atol=1e-12)
    assert c["E_ex"] == pytest.approx(b["E_ex"], rel=1e-13)
    assert c["E_real"] == pytest.approx(b["E_real"], rel=1e-12)
    np.testing.assert_allclose(c["W"], b["W"], rtol=1e-12, atol=1e-10)
    sample = np.array([5, 17, 3, 699, 0])
    s = oracle.real_space(w.pos, w.type, w.z, p, use_cells=True, sample=sample)
    np.testing.assert_allclose(s["F"], b["F"][sample], rtol=1e-13, atol=1e-13)


def test_two_beads_closed_form(oracle):
    # two beads in a large box: E_ex = u_ex(r), E_real = lB zz bracket(r);
    # force along the separation with magnitude -dU/dr (central difference
    # of the scalar functions, not of the sum).
    from oracle.oracle import Params
    A = np.array([[20.0, 27.0], [27.0, 31.0]])
    sig = np.array([0.4, 0.6])
    p = Params((20.0, 20.0, 20.0), 6.0, 1.1, 0.9, A, sig, sig)
    pos = np.array([[3.0, 4.0, 5.0], [3.8, 4.3, 4.1]])
    typ = np.array([0, 1])
    z = np.array([1, -1])
    out = oracle.real_space(pos, typ, z, p, use_cells=False)
    d = pos[0] - pos[1]
    r = np.linalg.norm(d)
    s2 = 0.16 + 0.36
    aij = math.sqrt(0.16 + 0.36)
    alpha = math.sqrt(math.pi / 2) / aij
    assert out["E_ex"] == pytest.approx(oracle.u_ex(r, 27.0, s2), rel=1e-14)
    assert out["E_real"] == pytest.approx(-0.9 * oracle.phi_real(r, alpha, 1.1), rel=1e-14)
    h = 1e-6
    U = lambda rr: oracle.u_ex(rr, 27.0, s2) - 0.9 * oracle.phi_real(rr, alpha, 1.1)
    dUdr = (U(r + h) - U(r - h)) / (2 * h)
    np.testing.assert_allclose(out["F"][0], -dUdr * d / r, rtol=1e-8)
    np.testing.assert_allclose(out["F"][1], dUdr * d / r, rtol=1e-8)


@pytest.fixture(scope="module")
def fd_system():
    return W.small_bulk(N=160, seed=21, charged_frac=0.5, box=(6.5, 7.0, 6.0), rc=2.4)


def test_forces_are_minus_gradient(oracle, fd_system):
    w = fd_system
    p = _params(w)
    ref = oracle.real_space(w.pos, w.type, w.z, p, use_cells=False)
    h = 1e-5
    rng = np.random.default_rng(0)
    for i in rng.choice(w.N, 8, replace=False):
        for k in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[i, k] += h
            pm[i, k] -= h
            ep = oracle.real_space(pp, w.type, w.z, p, use_cells=False)
            em = oracle.real_space(pm, w.type, w.z, p, use_cells=False)
            fd = -((ep["E_ex"] + ep["E_real"]) - (em["E_ex"] + em["E_real"])) / (2 * h)
            assert ref["F"][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    np.testing.assert_allclose(ref["F"].sum(0), 0.0, atol=1e-9)


def test_virial_is_minus_strain_derivative(oracle, fd_system):
    w = fd_system
    ref = oracle.real_space(w.pos, w.type, w.z, _params(w), use_cells=False)
    h = 1e-6
    for k in range(3):
        es = []
        for s in (+h, -h):
            scale = np.ones(3)
            scale[k] += s
            box = tuple(np.asarray(w.box) * scale)
            from oracle.oracle import Params
            p = Params(box, w.rc, w.beta, w.lB, w.A, w.sigma, w.a)
            o = oracle.real_space(w.pos * scale, w.type, w.z, p, use_cells=False)
            es.append(o["E_ex"] + o["E_real"])
        assert ref["W"][k] == pytest.approx(-(es[0] - es[1]) / (2 * h), rel=1e-6)


def test_parameter_derivatives(oracle, fd_system):
    from oracle.oracle import Params
    w = fd_system
    out = oracle.real_space(w.pos, w.type, w.z, _params(w), use_cells=False, adjoint=True)
    nt = w.nt
    # E_ex is linear in A: dE/dA_tt' = E_ex{t,t'} / A_tt'
    h = 1e-4
    for t in range(nt):
        for u in range(t, nt):
            Ap, Am = w.A.copy(), w.A.copy()
            Ap[t, u] += h; Ap[u, t] = Ap[t, u]
            Am[t, u] -= h; Am[u, t] = Am[t, u]
            ep = oracle.real_space(w.pos, w.type, w.z, Params(w.box, w.rc, w.beta, w.lB, Ap, w.sigma, w.a))
            em = oracle.real_space(w.pos, w.type, w.z, Params(w.box, w.rc, w.beta, w.lB, Am, w.sigma, w.a))
            fd = (ep["E_ex"] - em["E_ex"]) / (2 * h)
            assert out["Eex_tt"][t, u] / w.A[t, u] == pytest.approx(fd, rel=1e-9)
    h = 1e-6
    for t in range(nt):
        for which in ("sigma", "a"):
            vals = []
            for s in (+h, -h):
                sg, aa = w.sigma.copy(), w.a.copy()
                (sg if which == "sigma" else aa)[t] += s
                o = oracle.real_space(w.pos, w.type, w.z, Params(w.box, w.rc, w.beta, w.lB, w.A, sg, aa))
                vals.append(o["E_ex"] + o["E_real"])
            fd = (vals[0] - vals[1]) / (2 * h)
            got = out["dE_dsigma"][t] if which == "sigma" else out["dE_da"][t]
            assert got == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # self-energy derivative: U_self = lB/2 sum z^2 / a
    c = oracle.constants(w.type, w.z, _params(w))
    for t in range(nt):
        aa = w.a.copy(); aa[t] += h
        cp = oracle.constants(w.type, w.z, Params(w.box, w.rc, w.beta, w.lB, w.A, w.sigma, aa))
        aa[t] -= 2 * h
        cm = oracle.constants(w.type, w.z, Params(w.box, w.rc, w.beta, w.lB, w.A, w.sigma, aa))
        assert c["dE_da_self"][t] == pytest.approx((cp["E_self"] - cm["E_self"]) / (2 * h), rel=1e-7)


def test_gcm_mean_energy_uniform_positions(oracle):
    # For uniform random positions the expected GCM energy is
    # N(N-1)/(2V) * A * P(r < rc) with P = erf(x) - (2x/sqrt(pi)) exp(-x^2),
    # x = rc sqrt(3/2)/s (the Gaussian's mass inside rc).  Check within 4 s.d.
    # of the sample-to-sample spread measured over several seeds.
    vals = []
    for seed in range(6):
        w = W.bulk("m", 1200, 100 + seed, 0.0, [0.5], [[25.0]], 2.0, 1.0, (8, 8, 8))
        vals.append(oracle.real_space(w.pos, w.type, w.z, _params(w))["E_ex"])
    s = math.sqrt(0.5)
    x = 2.0 * math.sqrt(1.5) / s
    P = math.erf(x) - 2 * x / math.sqrt(math.pi) * math.exp(-x * x)
    V = w.box[0] ** 3
    expect = 1200 * 1199 / (2 * V) * 25.0 * P
    mean, sd = np.mean(vals), np.std(vals, ddof=1)
    assert abs(mean - expect) < 4 * sd / math.sqrt(len(vals)) + 1e-9 * expect
