"""GPU edge cases and the remaining paths against the FP64 oracle:
boxes smaller than the pair kernels' neighbourhood (periodic images staged
more than once), batched replicas of uneven size and parameters, replicas
without charges, the smallest system (two beads), pair counts, integrator
trajectories, the parameter adjoint, and argument validation."""
import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import energy_errors, gpu_eval, make_engine, oracle_eval, rel, rel_rms

pytestmark = pytest.mark.gpu


def _cmp(got_F, got_E, got_W, ref, ftol, etol):
    ferr = rel_rms(got_F, ref["F"])
    eerr = energy_errors(got_E[:5], ref["E"])
    # the virial tensor is a sum of cancelling pair and mesh parts: measure
    # its error on the scale of the energies that make it up
    wscale = np.linalg.norm(ref["W"]) + np.abs(ref["E"][:3]).sum()
    werr = np.linalg.norm(got_W - ref["W"]) / wscale
    print(f"  force {ferr:.2e} energy {np.array2string(eerr, precision=2)} virial {werr:.2e}", flush=True)
    assert ferr < ftol
    assert np.all(eerr < etol), eerr
    assert werr < 10 * max(ftol, etol)


@pytest.mark.parametrize("direct", [0, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_box_images(precision, direct):
    # L = 5.2 with rc = 2.5: the cell stencil wraps onto itself
    w = W.small_bulk(N=350, seed=13, charged_frac=0.4, box=(5.2, 5.3, 5.05), rc=2.5, grid=(16, 16, 16))
    print(f"case small box {w.box} prec={precision} direct_pairs={direct}", flush=True)
    eng = make_engine([w], precision, tuning=dict(cells_per_cutoff=3, direct_pairs=direct))
    got = gpu_eval(eng)
    eng.close()
    tol = (1e-9, 1e-10) if precision == "fp64" else (1e-5, 1e-6)
    _cmp(got["force"], got["energy"][0], got["virial"][0], oracle_eval(w), *tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_replicas(precision):
    ws = W.config5(n_replicas=6, seed=77)
    ws.append(W.small_bulk(N=257, seed=3, charged_frac=0.0, box=(5.5, 5.5, 5.5), rc=2.5, grid=(16, 16, 16)))
    ws[2] = W.small_bulk(N=901, seed=5, charged_frac=0.3, a_types=(0.35, 0.55, 0.65), box=(7.1, 8.2, 6.3),
                         rc=2.5, grid=(24, 32, 18))
    print("case batched replicas", [w.N for w in ws], [w.grid for w in ws], flush=True)
    eng = make_engine(ws, precision)
    got = gpu_eval(eng)
    eng.close()
    tol = (1e-9, 1e-10) if precision == "fp64" else (1e-5, 1e-6)
    off = 0
    for r, w in enumerate(ws):
        ref = oracle_eval(w)
        sl = slice(off, off + w.N)
        off += w.N
        print(f" replica {r} N={w.N}", flush=True)
        _cmp(got["force"][sl], got["energy"][r], got["virial"][r], ref, *tol)


def test_batched_equals_single():
    ws = W.config5(n_replicas=3, seed=11)
    eng = make_engine(ws, "fp64")
    allr = gpu_eval(eng)
    eng.close()
    off = 0
    for r, w in enumerate(ws):
        e1 = make_engine([w], "fp64")
        one = gpu_eval(e1)
        e1.close()
        np.testing.assert_allclose(allr["force"][off:off + w.N], one["force"], rtol=0, atol=1e-11)
        np.testing.assert_allclose(allr["energy"][r], one["energy"][0], rtol=1e-12)
        off += w.N


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_list_free_equals_lists(precision):
    # Both pair paths visit the same pairs with the same cutoff test; only the
    # order of the per-bead sums differs.
    w = W.config2()
    print(f"case list vs list-free {w.name} N={w.N} prec={precision}", flush=True)
    got = {}
    for d in (0, 3):
        eng = make_engine([w], precision, tuning=dict(cells_per_cutoff=3, beads_per_cluster=4,
                                                       charges_per_cluster=4, direct_pairs=d))
        got[d] = gpu_eval(eng)
        if precision == "mixed":
            got[d]["pairs"] = eng.count_pairs()
        eng.close()
    ftol = 1e-12 if precision == "fp64" else 1e-6
    ferr = rel_rms(got[3]["force"], got[0]["force"])
    eerr = np.abs(got[3]["energy"][0, :5] - got[0]["energy"][0, :5]) / np.abs(got[0]["energy"][0, :5]).max()
    print(f"  list-free vs list: force {ferr:.2e} energy {eerr.max():.2e}", flush=True)
    assert ferr < ftol
    assert eerr.max() < ftol
    if precision == "mixed":
        assert got[3]["pairs"] == got[0]["pairs"]


def test_two_beads():
    w = W.small_bulk(N=2, seed=1, charged_frac=1.0, a_types=(0.5,), box=(6.0, 6.0, 6.0), rc=2.9,
                     grid=(16, 16, 16))
    w.pos[:] = W.lattice_positions(np.array([[0.1, 0.2, 0.3], [0.15, 0.22, 0.31]]), w.box)
    eng = make_engine([w], "fp64")
    got = gpu_eval(eng)
    eng.close()
    _cmp(got["force"], got["energy"][0], got["virial"][0], oracle_eval(w), 1e-9, 1e-10)


@pytest.mark.parametrize("direct", [0, 1])
def test_pair_count_matches_kdtree(direct):
    from scipy.spatial import cKDTree
    w = W.small_bulk(N=3000, seed=21, charged_frac=0.2, box=(10.6, 10.6, 10.7), rc=2.7, grid=(32, 32, 32))
    print(f"case pair count direct_pairs={direct}", flush=True)
    eng = make_engine([w], "mixed", tuning=dict(direct_pairs=direct))
    n = eng.count_pairs()
    eng.close()
    tree = cKDTree(np.mod(w.pos, w.box), boxsize=w.box)
    ref = len(tree.query_pairs(w.rc))
    # ties at exactly rc have measure zero for random inputs
    assert n == ref


def test_velocity_verlet_trajectory_fp64():
    # The engine keeps positions on a 2^-32 L lattice, the oracle in FP64, so
    # the trajectories separate at the rate chaos amplifies a ~1e-9 rounding:
    # after one step they agree to that rounding, and the energy drift of the
    # whole 100-step run matches the oracle's.
    from oracle import oracle as O
    from tests.gpu_common import oracle_params
    w = W.config1()
    p = oracle_params(w)
    eng = make_engine([w], "fp64")
    errs, gtot = {}, {}
    done = 0
    for n in (1, 9, 90):
        obs = eng.step(n, observe=True)
        eng.sync()
        done += n
        pos, vel, step = eng.get_state()
        assert step == done
        opos, ovel, oF, Elog = O.md(w.pos, w.vel, w.type, w.z, np.arange(w.N, dtype=np.int32), p, w.mass, w.dt,
                                    0.0, w.kT, 0, 0, 0, done, recip_mode=O.RECIP_SPME, K=w.grid, order=w.order)
        d = pos.cpu().numpy().T - opos
        d -= np.asarray(w.box) * np.round(d / np.asarray(w.box))
        errs[done] = np.sqrt((d ** 2).mean())
        E = obs["energy"].cpu().numpy()[0]
        gtot[done] = E[5] + E[6]
        if done == 1:
            assert gtot[1] == pytest.approx(Elog[0, 0] + Elog[0, 1], rel=1e-10)
    eng.close()
    ora_drift = abs((Elog[-1, 0] + Elog[-1, 1]) - (Elog[0, 0] + Elog[0, 1]))
    gpu_drift = abs(gtot[100] - gtot[1])
    print(f"  VV rms position difference by step: {errs}; energy drift gpu {gpu_drift:.3e} "
          f"oracle {ora_drift:.3e}", flush=True)
    assert errs[1] < 1e-8
    assert errs[10] < 1e-6
    assert gpu_drift < 2.0 * ora_drift + 1e-9 * abs(gtot[1])


@pytest.mark.parametrize("layout", [0, 2])
@pytest.mark.parametrize("gamma", [0.0, 1.0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_steps_equal_single_steps(precision, gamma, layout):
    # A run of n steps fuses each step's second half kick with the next
    # step's first half and binning; n runs of one step do not.  The
    # arithmetic is the same, so the trajectories agree bit for bit.
    w = W.small_bulk(N=900, seed=8, charged_frac=0.3, box=(7.1, 7.3, 6.9), rc=2.5, grid=(24, 24, 24))
    w.gamma = gamma
    print(f"case fused steps prec={precision} gamma={gamma} layout={layout}", flush=True)
    runs = []
    for split in (False, True):
        eng = make_engine([w], precision, seed=5, tuning=dict(stream_layout=layout))
        if split:
            for _ in range(12):
                eng.step(1)
        else:
            eng.step(12)
        obs = eng.step(1, observe=True)
        eng.sync()
        pos, vel, step = eng.get_state()
        runs.append((pos.cpu().numpy(), vel.cpu().numpy(), step, obs["energy"].cpu().numpy()))
        eng.close()
    assert runs[0][2] == runs[1][2] == 13
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    np.testing.assert_array_equal(runs[0][3], runs[1][3])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_leaves_state_unchanged(precision):
    # The autotuner times whole steps from the current state and restores
    # it (order, positions, velocities, forces, step counter): a run after
    # it equals, bit for bit, the same run of an engine switched to the
    # tuning it picked at that point.
    w = W.small_bulk(N=900, seed=9, charged_frac=0.3, box=(7.1, 7.3, 6.9), rc=2.5, grid=(24, 24, 24))
    print(f"case autotune restore prec={precision}", flush=True)
    eng = make_engine([w], precision, seed=5)
    eng.step(3)
    eng.sync()
    before = [x.cpu().numpy() for x in eng.get_state()[:2]] + [eng.get_state()[2]]
    tun = eng.autotune()
    after = [x.cpu().numpy() for x in eng.get_state()[:2]] + [eng.get_state()[2]]
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    assert before[2] == after[2] == 3
    runs = []
    for e in (eng, None):
        if e is None:
            e = make_engine([w], precision, seed=5)
            e.step(3)
            e.set_tuning(**tun)
        e.step(7)
        obs = e.step(1, observe=True)
        e.sync()
        pos, vel, step = e.get_state()
        runs.append((pos.cpu().numpy(), vel.cpu().numpy(), step, obs["energy"].cpu().numpy(),
                     obs["force"].cpu().numpy()))
        e.close()
    assert runs[0][2] == runs[1][2] == 11
    for k in (0, 1, 3, 4):
        np.testing.assert_array_equal(runs[0][k], runs[1][k])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_langevin_trajectory_short(precision):
    from oracle import oracle as O
    from tests.gpu_common import oracle_params
    w = W.small_bulk(N=800, seed=41, charged_frac=0.3, box=(6.9, 6.9, 6.8), rc=2.5, grid=(24, 24, 24))
    eng = make_engine([w], precision, seed=99)
    eng.step(10)
    eng.sync()
    pos, vel, _ = eng.get_state()
    eng.close()
    p = oracle_params(w)
    opos, ovel, _, _ = O.md(w.pos, w.vel, w.type, w.z, np.arange(w.N, dtype=np.int32), p, w.mass, w.dt, w.gamma,
                            w.kT, 99, 0, 0, 10, recip_mode=O.RECIP_SPME, K=w.grid, order=w.order)
    dv = rel_rms(vel.cpu().numpy().T, ovel)
    print(f"  BAOAB 10 steps velocity rel diff {dv:.2e}", flush=True)
    # same noise on both sides; the residual is the 2^-32 position lattice
    # (fp64) or float32 forces (mixed), grown over 10 steps
    assert dv < (1e-7 if precision == "fp64" else 1e-4)


def test_langevin_temperature():
    w = W.small_bulk(N=4000, seed=42, charged_frac=0.2, box=(11.7, 11.7, 11.7), rc=2.5, grid=(32, 32, 32))
    eng = make_engine([w], "mixed", seed=5)
    eng.step(400)
    Ts = []
    for _ in range(20):
        o = eng.step(20, observe=True)
        eng.sync()
        Ts.append(2 * o["energy"][0, 6].item() / (3 * w.N))
    eng.close()
    print(f"  <T> = {np.mean(Ts):.4f} +- {np.std(Ts) / np.sqrt(len(Ts)):.4f}", flush=True)
    assert abs(np.mean(Ts) - 1.0) < 0.02


@pytest.mark.parametrize("direct", [0, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_matches_oracle(precision, direct):
    w = W.small_bulk(N=900, seed=7, charged_frac=0.3, a_types=(0.35, 0.55, 0.65), box=(7.1, 7.3, 6.9),
                     rc=2.5, grid=(24, 24, 24))
    print(f"case adjoint prec={precision} direct_pairs={direct}", flush=True)
    eng = make_engine([w], precision, tuning=dict(direct_pairs=direct))
    got = gpu_eval(eng, adjoint=True)
    eng.close()
    ref = oracle_eval(w, adjoint=True)
    nt = w.nt
    ett = ref["Eex_tt"]
    dA_ref = ett / w.A
    tol = 1e-10 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(got["dE_dA"][0][:nt, :nt], dA_ref, rtol=tol)
    np.testing.assert_allclose(got["dE_dsigma"][0][:nt], ref["dE_dsigma"], rtol=tol)
    np.testing.assert_allclose(got["dE_da"][0][:nt], ref["dE_da"], rtol=tol)


def test_validation_errors():
    from paper_2403_08148_amd import GCMe, GCMeError, params_from_workload
    from paper_2403_08148_amd import _binding as B
    w = W.small_bulk(N=300, seed=1, box=(5.0, 5.0, 5.0), rc=2.4)
    eng = GCMe([w.N], precision="mixed")
    with pytest.raises(GCMeError) as e:
        eng.forces_energy()
    assert e.value.status == B.GCME_ESTATE
    for bad, code in [(dict(cutoff=2.6), B.GCME_EGEOMETRY), (dict(grid=(20, 20, 20)), B.GCME_EUNSUPPORTED),
                      (dict(order=9), B.GCME_EUNSUPPORTED), (dict(box=(5.0, -1.0, 5.0)), B.GCME_EGEOMETRY),
                      (dict(beta=0.0), B.GCME_EINVAL)]:
        with pytest.raises(GCMeError) as e:
            eng.set_params(params_from_workload(w, **bad))
        assert e.value.status == code, bad
    eng.set_params(params_from_workload(w))
    z = w.z.copy()
    z[np.nonzero(z)[0][0]] = 0
    with pytest.raises(GCMeError) as e:
        eng.set_state(w.pos, w.type, z, w.vel)
    assert e.value.status == B.GCME_ENONNEUTRAL
    t = w.type.copy()
    t[0] = 7
    with pytest.raises(GCMeError) as e:
        eng.set_state(w.pos, t, w.z, w.vel)
    assert e.value.status == B.GCME_EINVAL
    # strict no-collapse check: tiny A with large lB violates it
    with pytest.raises(GCMeError):
        eng.set_params(params_from_workload(w, A=w.A * 1e-3, lB=5.0, flags=B.GCME_FLAG_STRICT_CONTACT))
    eng.close()
