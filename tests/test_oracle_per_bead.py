"""Pins of the oracle's per-bead radius derivatives dE/dsigma_i, dE/da_i and
of the forces' vector-Jacobian product (force matching).

A bead given a type of its own (with its old type's parameters, so the
energy is unchanged) has a per-type derivative equal to its per-bead one:
central differences of the oracle's energy over that type's radius pin the
per-bead values independently of their formula.  Summed over a type they
equal the per-type derivatives; an uncharged bead has dE/da_i = 0.
"""
import numpy as np
import pytest

import oracle.oracle as O


def _system(seed=3, N=220, L=5.2):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (N, 3))
    t = (np.arange(N) % 2).astype(np.int32)
    z = np.zeros(N, dtype=np.int32)
    z[:40] = np.array([1, -1] * 20)
    A = np.array([[22.0, 25.0], [25.0, 28.0]])
    p = O.Params(box=(L, L, L), rc=2.4, beta=1.1, lB=1.0, A=A, sigma=np.array([0.45, 0.55]), a=np.array([0.4, 0.6]))
    return pos, t, z, p


def _own_type(t, p, k):
    """Parameters with bead k moved to a third type identical to its own."""
    tk = t[k]
    nt = 3
    A = np.zeros((nt, nt))
    A[:2, :2] = p.A
    A[2, :2] = A[:2, 2] = p.A[tk]
    A[2, 2] = p.A[tk, tk]
    t2 = t.copy()
    t2[k] = 2
    return t2, O.Params(box=p.box, rc=p.rc, beta=p.beta, lB=p.lB, A=A, sigma=np.r_[p.sigma, p.sigma[tk]],
                        a=np.r_[p.a, p.a[tk]])


def _energy(pos, t, z, p):
    E = O.forces(pos, t, z, p, recip_mode=O.RECIP_NONE)["E"]
    return E[0] + E[1] + E[4]  # the terms that depend on the radii


@pytest.mark.parametrize("k", [0, 7, 150])
def test_per_bead_matches_finite_differences_of_an_own_type(k):
    pos, t, z, p = _system()
    pb = O.per_bead_adjoint(pos, t, z, p)
    t2, p2 = _own_type(t, p, k)
    assert _energy(pos, t2, z, p2) == pytest.approx(_energy(pos, t, z, p), rel=1e-13)
    h = 1e-5
    for name, attr in (("dE_dsigma", "sigma"), ("dE_da", "a")):
        es = []
        for e in (h, -h):
            v = getattr(p2, attr).copy()
            v[2] += e
            q = O.Params(box=p2.box, rc=p2.rc, beta=p2.beta, lB=p2.lB, A=p2.A,
                         sigma=v if attr == "sigma" else p2.sigma, a=v if attr == "a" else p2.a)
            es.append(_energy(pos, t2, z, q))
        fd = (es[0] - es[1]) / (2 * h)
        assert pb[name][k] == pytest.approx(fd, rel=1e-6, abs=1e-8), name
    if z[k] == 0:
        assert pb["dE_da"][k] == 0.0


def test_per_bead_sums_to_per_type():
    pos, t, z, p = _system(seed=4)
    pb = O.per_bead_adjoint(pos, t, z, p)
    rs = O.real_space(pos, t, z, p, adjoint=True)
    c = O.constants(t, z, p)
    for ty in range(2):
        assert pb["dE_dsigma"][t == ty].sum() == pytest.approx(rs["dE_dsigma"][ty], rel=1e-11)
        assert pb["dE_da"][t == ty].sum() == pytest.approx(rs["dE_da"][ty] + c["dE_da_self"][ty], rel=1e-11)


def test_force_vjp_matches_finite_differences():
    """sum_i v_i . dF_i/dtheta against central differences of sum_i v_i . F_i
    over each parameter (forces from the oracle's evaluation; the
    reciprocal forces do not depend on these parameters)."""
    pos, t, z, p = _system(seed=5, N=160)
    rng = np.random.default_rng(9)
    v = rng.normal(size=(len(pos), 3))
    vj = O.force_vjp(pos, t, z, p, v)

    def vF(q):
        return float((v * O.forces(pos, t, z, q, recip_mode=O.RECIP_NONE)["F"]).sum())

    def with_(A=None, sigma=None, a=None):
        return O.Params(box=p.box, rc=p.rc, beta=p.beta, lB=p.lB, A=p.A if A is None else A,
                        sigma=p.sigma if sigma is None else sigma, a=p.a if a is None else a)

    h = 1e-5
    for (ti, tu) in ((0, 0), (0, 1), (1, 1)):
        Ap, Am = p.A.copy(), p.A.copy()
        Ap[ti, tu] += h
        Am[ti, tu] -= h
        if ti != tu:
            Ap[tu, ti] += h
            Am[tu, ti] -= h
        fd = (vF(with_(A=Ap)) - vF(with_(A=Am))) / (2 * h)
        assert vj["dA"][ti, tu] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for ty in range(2):
        for name, key in (("sigma", "dsigma"), ("a", "da")):
            vp, vm = getattr(p, name).copy(), getattr(p, name).copy()
            vp[ty] += h
            vm[ty] -= h
            fd = (vF(with_(**{name: vp})) - vF(with_(**{name: vm}))) / (2 * h)
            assert vj[key][ty] == pytest.approx(fd, rel=1e-6, abs=1e-8), (name, ty)
