"""Pins of the oracle's slab correction, harmonic bonds and fixed (infinite
mass) bead types, the terms of the slab systems in the section on
polyelectrolyte adsorption at electrodes.

- Slab correction: physics, not the formula.  A neutral slab confined to
  0 < z < h in a box with a vacuum gap along z: the tin-foil Ewald sum of
  eq. ewald (exact k-sum) changes with the gap (the slabs of the periodic
  stack see each other's dipoles), while that sum plus the correction
  converges to the gap-independent slab value; the forces converge too.
  Also: force = -dE/dz (central differences), zero net force, virial =
  -dE/d strain.
- Bonds: worked values of a stretched bond (also across the periodic
  boundary), zero at the rest length, force = -grad E, Newton's third law,
  virial = -dE/d strain.
- Fixed types: beads of infinite mass keep their positions bit for bit over
  Langevin steps while feeling forces; the kinetic energy stays finite.
- Image charges (metal electrodes): a charge near the conducting plane feels
  its image's pull -lB/(2d)^2, approached as the periodic box grows; images
  stay the exact reflections of their sources through MD steps.
"""
import numpy as np
import pytest

import oracle.oracle as O


def _slab_system(seed=7, N=24, h=4.0, Lx=6.0):
    rng = np.random.default_rng(seed)
    pos = np.c_[rng.uniform(0, Lx, N), rng.uniform(0, Lx, N), rng.uniform(0.3, h - 0.3, N)]
    z = np.array([1, -1] * (N // 2), dtype=np.int32)
    t = np.zeros(N, dtype=np.int32)
    return pos, t, z


def _params(box, A=0.0):
    return O.Params(box=box, rc=3.0, beta=1.0, lB=1.0, A=np.full((1, 1), A), sigma=np.array([0.5]),
                    a=np.array([0.5]))


def test_slab_correction_removes_the_gap_dependence():
    h, Lx = 4.0, 6.0
    pos, t, z = _slab_system(h=h, Lx=Lx)
    plain, corr, forces = [], [], []
    for Lz in (3 * h, 6 * h, 9 * h):
        p = _params((Lx, Lx, Lz))
        ex = O.Extra(slab=True)
        r = O.forces_ext(pos, t, z, p, ex, recip_mode=O.RECIP_EWALD, kmax=10.0)
        plain.append(r["E"][:5].sum())
        corr.append(r["E"].sum())
        forces.append(r["F"])
    scale = abs(corr[-1])
    # without the correction the energy moves by several percent ...
    assert abs(plain[0] - plain[2]) > 0.02 * scale
    # ... with it, it has converged already at a gap of twice the slab width
    assert abs(corr[0] - corr[2]) < 1e-5 * scale
    assert abs(corr[1] - corr[2]) < 1e-9 * scale
    fs = np.linalg.norm(forces[2])
    assert np.linalg.norm(forces[1] - forces[2]) < 1e-7 * fs
    assert np.linalg.norm(forces[0] - forces[2]) < 1e-3 * fs


def test_slab_force_is_minus_gradient_and_net_zero():
    pos, t, z = _slab_system(seed=3)
    box = (6.0, 6.0, 12.0)
    s = O.slab(pos, z, box, 1.0)
    assert abs(s["F"].sum(axis=0)).max() < 1e-12 * np.abs(s["F"]).max()
    assert np.all(s["F"][:, :2] == 0.0)
    h = 1e-5
    for i in (0, 5, 17):
        pp, pm = pos.copy(), pos.copy()
        pp[i, 2] += h
        pm[i, 2] -= h
        fd = -(O.slab(pp, z, box, 1.0)["E"] - O.slab(pm, z, box, 1.0)["E"]) / (2 * h)
        assert s["F"][i, 2] == pytest.approx(fd, rel=1e-7)


def test_slab_virial_is_minus_strain_derivative():
    pos, t, z = _slab_system(seed=4)
    box = np.array([6.0, 6.0, 12.0])
    s = O.slab(pos, z, box, 1.0)
    h = 1e-6
    for a in range(3):
        es = []
        for e in (h, -h):
            sc = np.ones(3)
            sc[a] += e
            es.append(O.slab(pos * sc, z, box * sc, 1.0)["E"])
        assert s["W"][a] == pytest.approx(-(es[0] - es[1]) / (2 * h), rel=1e-6)
    assert np.all(s["W"][3:] == 0.0)


def test_bond_worked_values():
    # two beads 1.0 apart along x, k = 100, b = 0.8: E = 100/2 * 0.2^2 = 2,
    # |F| = 100 * 0.2 = 20, pulling the beads together
    pos = np.array([[1.0, 2.0, 3.0], [2.0, 2.0, 3.0]])
    r = O.bonds(pos, (10.0, 10.0, 10.0), [[0, 1]], 100.0, 0.8)
    assert r["E"] == pytest.approx(2.0, rel=1e-14)
    np.testing.assert_allclose(r["F"], [[20.0, 0, 0], [-20.0, 0, 0]], rtol=1e-13, atol=1e-13)
    # the same bond across the periodic boundary
    pos2 = np.array([[9.6, 2.0, 3.0], [0.6, 2.0, 3.0]])
    r2 = O.bonds(pos2, (10.0, 10.0, 10.0), [[0, 1]], 100.0, 0.8)
    assert r2["E"] == pytest.approx(2.0, rel=1e-12)
    np.testing.assert_allclose(r2["F"], r["F"], rtol=1e-11, atol=1e-11)
    # compressed to 0.5: E = 50 * 0.09 = 4.5, pushing apart with |F| = 30
    pos3 = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.5]])
    r3 = O.bonds(pos3, (10.0, 10.0, 10.0), [[0, 1]], 100.0, 0.8)
    assert r3["E"] == pytest.approx(4.5, rel=1e-13)
    np.testing.assert_allclose(r3["F"], [[0, 0, -30.0], [0, 0, 30.0]], rtol=1e-13, atol=1e-12)
    # at the rest length
    pos4 = np.array([[1.0, 2.0, 3.0], [1.0, 2.8, 3.0]])
    assert O.bonds(pos4, (10.0, 10.0, 10.0), [[0, 1]], 100.0, 0.8)["E"] == pytest.approx(0.0, abs=1e-25)


def _chain(seed=5, n=12, L=5.0):
    rng = np.random.default_rng(seed)
    steps = rng.normal(size=(n - 1, 3))
    steps *= (0.8 + 0.2 * rng.uniform(-1, 1, (n - 1, 1))) / np.linalg.norm(steps, axis=1, keepdims=True)
    pos = np.vstack([np.zeros(3), np.cumsum(steps, axis=0)]) + 2.0
    pos %= L  # chains cross the periodic boundary
    pairs = np.c_[np.arange(n - 1), np.arange(1, n)]
    return pos, pairs, (L, L, L)


def test_bond_force_gradient_newton_virial():
    pos, pairs, box = _chain()
    r = O.bonds(pos, box, pairs, 100.0, 0.8)
    assert np.abs(r["F"].sum(axis=0)).max() < 1e-12 * np.abs(r["F"]).max()
    h = 1e-6
    for i in (0, 4, 11):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = -(O.bonds(pp, box, pairs, 100.0, 0.8)["E"] - O.bonds(pm, box, pairs, 100.0, 0.8)["E"]) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    # -dE/d strain with the bonds' own (unwrapped) geometry: strain the
    # minimum-image separations about bead 0
    un = np.vstack([pos[0], pos[0] + np.cumsum(
        [(pos[j] - pos[i]) - np.asarray(box) * np.round((pos[j] - pos[i]) / np.asarray(box)) for i, j in pairs],
        axis=0)])
    big = (100.0, 100.0, 100.0)
    for a in range(3):
        es = []
        for e in (h, -h):
            sc = np.ones(3)
            sc[a] += e
            es.append(O.bonds(un * sc, big, pairs, 100.0, 0.8)["E"])
        assert r["W"][a] == pytest.approx(-(es[0] - es[1]) / (2 * h), rel=1e-6)


def test_infinite_mass_type_stays_fixed():
    rng = np.random.default_rng(11)
    N, L = 200, 5.0
    pos = rng.uniform(0, L, (N, 3))
    t = (np.arange(N) % 2).astype(np.int32)  # type 1 fixed
    z = np.zeros(N, dtype=np.int32)
    p = O.Params(box=(L, L, L), rc=2.5, beta=1.0, lB=1.0, A=np.full((2, 2), 25.0),
                 sigma=np.array([0.5, 0.5]), a=np.array([0.5, 0.5]))
    vel = rng.normal(size=(N, 3))
    vel[t == 1] = 0.0
    mass = np.array([1.0, np.inf])
    f0 = O.forces(pos, t, z, p, recip_mode=O.RECIP_NONE)["F"]
    assert np.abs(f0[t == 1]).max() > 1.0  # they are pushed ...
    p1, v1, F1, Elog = O.md(pos, vel, t, z, np.arange(N), p, mass, 0.02, 1.0, 1.0, 9, 0, 0, 10,
                            recip_mode=O.RECIP_NONE)
    np.testing.assert_array_equal(p1[t == 1], pos[t == 1])  # ... and do not move
    assert np.all(v1[t == 1] == 0.0)
    assert np.abs(p1[t == 0] - pos[t == 0]).max() > 1e-3
    assert np.all(np.isfinite(Elog))
    # the kinetic energy is that of the mobile beads only
    assert Elog[-1, 1] == pytest.approx(0.5 * (v1[t == 0] ** 2).sum(), rel=1e-12)


def test_image_charge_attracts_to_the_electrode():
    """Method of image charges: a charge at height d over a perfectly
    conducting plane is pulled toward it by its image, F = -lB q^2/(2d)^2
    (the smeared charges act as points at 2d >= 1.5 to 1e-3); the periodic
    copies' share falls as the box grows."""
    ratios = {}
    for L in (16.0, 32.0):
        for d in (1.0, 1.5):
            pos = np.array([[L / 2, L / 2, d], [0.0, 0.0, 0.0]])
            pos = O.mirror_images(pos, (L, L, L), [[1, 0]])
            assert pos[1, 2] == L - d and pos[1, 0] == pos[0, 0] and pos[1, 1] == pos[0, 1]
            p = O.Params(box=(L, L, L), rc=4.0, beta=1.0, lB=1.0, A=np.zeros((2, 2)), sigma=np.array([0.5, 0.5]),
                         a=np.array([0.5, 0.5]))
            F = O.forces(pos, np.array([0, 1]), np.array([1, -1]), p, recip_mode=O.RECIP_EWALD, kmax=9.5)["F"]
            assert abs(F[0, 0]) < 1e-12 and abs(F[0, 1]) < 1e-12
            ratios[(L, d)] = F[0, 2] / (-1.0 / (2 * d) ** 2)
    assert abs(ratios[(32.0, 1.0)] - 1.0) < 2e-3
    assert abs(ratios[(32.0, 1.5)] - 1.0) < 6e-3
    for d in (1.0, 1.5):
        assert abs(ratios[(32.0, d)] - 1.0) < abs(ratios[(16.0, d)] - 1.0)


def test_images_follow_their_sources_in_md():
    rng = np.random.default_rng(12)
    L, H = 6.0, 5.0
    n = 60
    pos = np.c_[rng.uniform(0, L, n), rng.uniform(0, L, n), rng.uniform(0.5, H - 0.5, n)]
    z = np.array([1, -1] * (n // 2), dtype=np.int32)
    # images of every charged bead, type 1 (no excluded volume, infinite mass)
    img = np.c_[np.arange(n, 2 * n), np.arange(n)]
    pos = O.mirror_images(np.vstack([pos, np.zeros((n, 3))]), (L, L, 2 * H), img)
    t = np.r_[np.zeros(n), np.ones(n)].astype(np.int32)
    zz = np.r_[z, -z].astype(np.int32)
    A = np.array([[25.0, 0.0], [0.0, 0.0]])
    p = O.Params(box=(L, L, 2 * H), rc=2.5, beta=1.2, lB=1.0, A=A, sigma=np.array([0.5, 0.5]), a=np.array([0.5, 0.5]))
    vel = np.r_[rng.normal(size=(n, 3)), np.zeros((n, 3))]
    ex = O.Extra(images=img)
    p1, v1, F1, _ = O.md(pos, vel, t, zz, np.arange(2 * n), p, np.array([1.0, np.inf]), 0.02, 1.0, 1.0, 3, 0, 0, 5,
                         recip_mode=O.RECIP_EWALD, kmax=6.0, extra=ex)
    np.testing.assert_array_equal(p1[n:], O.mirror_images(p1, (L, L, 2 * H), img)[n:])
    assert np.abs(p1[:n] - pos[:n]).max() > 1e-3
    assert np.all(v1[n:] == 0.0)
