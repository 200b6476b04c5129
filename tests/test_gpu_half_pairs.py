"""GPU parity of the column-cluster pair kernels (tuning half_pairs, two bits
per pair type: bits 0-1 the excluded volume, 2-3 the real-space
electrostatics; 1 = half shell: each unordered pair within rc evaluated once,
by the column cluster that owns it, both beads receiving its force; 2 = both
ends: every pair from both of its beads' clusters).

The bars are those of test_gpu_parity.py (FP64: 1e-9 force RMS, 1e-10 per
energy term; mixed: 1e-5 and 1e-6; per bead ten times the RMS bar), against
the FP64 oracle on the same inputs:
* every cell size (1 to 4 cells per cutoff, which takes the enumeration from
  whole axes to narrow stencils), both cluster sizes, ragged boxes with three
  types and charged beads;
* boxes with two cells along an axis, where a column is exactly half the
  axis ahead of another (the tie the ownership rule breaks by index), and
  with one cell;
* the bulk electrolyte at full size, on and off the position lattice;
* batched replicas, the slab systems (sparse image halves: clusters spread
  over several cells), runs of steps (a run of n steps equals n runs of one
  step), bit-identical reruns, and the paths that fall back to the cluster
  kernels (parameter derivatives, pair counting).
"""
import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import energy_errors, gpu_eval, make_engine, oracle_eval, per_bead_err, rel_rms
from tests.test_gpu_parity import _check

pytestmark = pytest.mark.gpu

HALF = dict(half_pairs=5)  # both pair types half shell


def _t(**kw):
    d = dict(HALF)
    d.update(kw)
    return d


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tuning", [_t(cells_per_cutoff=1, beads_per_cluster=8, charges_per_cluster=4, direct_pairs=3),
                                    _t(cells_per_cutoff=2, beads_per_cluster=4, charges_per_cluster=8, direct_pairs=3),
                                    _t(cells_per_cutoff=2, beads_per_cluster=8, direct_pairs=1, stream_layout=1,
                                       half_pairs=1),
                                    _t(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=2, direct_pairs=2,
                                       stream_layout=0, half_pairs=4),
                                    _t(cells_per_cutoff=3, beads_per_cluster=2, charges_per_cluster=8, direct_pairs=3,
                                       stream_layout=2),
                                    _t(cells_per_cutoff=4, beads_per_cluster=4, charges_per_cluster=4, direct_pairs=3,
                                       stream_layout=4),
                                    _t(cells_per_cutoff=1, beads_per_cluster=8, charges_per_cluster=4, direct_pairs=3,
                                       half_pairs=10),
                                    _t(cells_per_cutoff=2, beads_per_cluster=4, charges_per_cluster=8, direct_pairs=3,
                                       half_pairs=6),
                                    _t(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=4, direct_pairs=3,
                                       half_pairs=9),
                                    _t(cells_per_cutoff=4, beads_per_cluster=8, charges_per_cluster=8, direct_pairs=3,
                                       half_pairs=10, stream_layout=1)])
def test_half_tunings_parity(precision, tuning):
    w = W.small_bulk(N=1001, seed=4, charged_frac=0.25, a_types=(0.3, 0.5, 0.7), box=(7.7, 8.3, 6.5),
                     rc=2.6, grid=(27, 36, 24), order=4)
    _check(w, precision, tuning)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("cpc", [1, 2])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_two_cells_per_axis(precision, cpc, mode):
    # 5.3 / 2.5: two cells per axis at one cell per cutoff (every column of
    # the other half-axis is exactly half the axis away), four at two
    # (whole axes)
    w = W.small_bulk(N=360, seed=8, charged_frac=0.3, box=(5.3, 5.6, 5.2), rc=2.5, grid=(18, 18, 18))
    _check(w, precision, _t(cells_per_cutoff=cpc, beads_per_cluster=8, half_pairs=mode))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_one_cell_across(precision, mode):
    # 3.0 wide at rc = 1.45: one cell along x at one cell per cutoff
    w = W.small_bulk(N=180, seed=9, charged_frac=0.2, box=(3.0, 6.2, 5.9), rc=1.45, grid=(16, 24, 24))
    _check(w, precision, _t(cells_per_cutoff=1, beads_per_cluster=4, half_pairs=mode))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("on_lattice", [True, False])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_config2_full_size(precision, on_lattice, mode):
    w = W.config2(on_lattice=on_lattice)
    print(f"case config2 N={w.N} prec={precision} on_lattice={on_lattice} mode={mode}", flush=True)
    eng = make_engine([w], precision, tuning=_t(cells_per_cutoff=2, beads_per_cluster=8, half_pairs=mode))
    got = gpu_eval(eng)
    eng.close()
    ref = oracle_eval(w)
    ferr = rel_rms(got["force"], ref["F"])
    fb = per_bead_err(got["force"], ref["F"])
    eerr = energy_errors(got["energy"][0, :5], ref["E"])
    werr = rel_rms(got["virial"][0], ref["W"])
    print(f"  force {ferr:.2e} per-bead {fb:.2e} energy {np.array2string(eerr, precision=2)} virial {werr:.2e}",
          flush=True)
    if precision == "mixed":
        assert ferr < 1e-5 and fb < 1e-4 and np.all(eerr < 1e-6) and werr < 1e-5
    elif on_lattice:
        assert ferr < 1e-9 and fb < 1e-8 and np.all(eerr < 1e-10) and werr < 1e-8
    else:
        # off the lattice the FP64 engine computes the forces of the stored
        # (rounded) positions: test_gpu_general_inputs.py derives that bar;
        # here, the same pairs as the cluster kernels at the same positions
        eng = make_engine([w], precision, tuning=dict(cells_per_cutoff=2, beads_per_cluster=8, direct_pairs=3))
        full = gpu_eval(eng)
        eng.close()
        d = rel_rms(got["force"], full["force"])
        print(f"  against the cluster kernels: force {d:.2e}", flush=True)
        assert d < 1e-12
        assert np.all(np.abs(got["energy"][0, :5] - full["energy"][0, :5])
                      <= 1e-12 * np.abs(full["energy"][0, :5]) + 1e-9)


@pytest.mark.parametrize("mode", [5, 10])
def test_half_reruns_bit_identical(mode):
    w = W.small_bulk(N=2000, seed=12, charged_frac=0.2, box=(9.3, 9.1, 9.5), rc=2.5, grid=(24, 24, 24))
    eng = make_engine([w], "mixed", tuning=_t(cells_per_cutoff=2, beads_per_cluster=8, half_pairs=mode))
    a = gpu_eval(eng)
    b = gpu_eval(eng)
    eng.close()
    assert np.array_equal(a["force"], b["force"])
    assert np.array_equal(a["energy"], b["energy"])
    assert np.array_equal(a["virial"], b["virial"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_batched_replicas(precision, mode):
    ws = W.config5(n_replicas=6, seed=7)
    tun = _t(cells_per_cutoff=2, beads_per_cluster=8, half_pairs=mode)
    eng = make_engine(ws, precision, tuning=tun)
    got = gpu_eval(eng)
    eng.close()
    off = 0
    ftol, etol = (1e-9, 1e-10) if precision == "fp64" else (1e-5, 1e-6)
    for r, w in enumerate(ws):
        ref = oracle_eval(w)
        F = got["force"][off:off + w.N]
        ferr = rel_rms(F, ref["F"])
        eerr = energy_errors(got["energy"][r, :5], ref["E"])
        print(f"replica {r} N={w.N}: force {ferr:.2e} energy {np.array2string(eerr, precision=2)}", flush=True)
        assert ferr < ftol
        assert np.all(eerr < etol)
        off += w.N


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("metal", [False, True])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_slab(precision, metal, mode):
    from tests.test_gpu_slab import _compare, _engine, _oracle
    w = W.slab_system(metal=metal)
    print(f"case slab_system metal={metal} N={w.N} prec={precision} mode={mode}", flush=True)
    eng = _engine([w], precision, tuning=_t(cells_per_cutoff=2, beads_per_cluster=8, half_pairs=mode))
    got = gpu_eval(eng)
    eng.close()
    _compare(got["energy"][0], got["force"], got["virial"][0], _oracle(w), precision, "half")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gamma", [0.0, 1.0])
@pytest.mark.parametrize("mode", [5, 10])
def test_half_fused_steps_equal_single_steps(precision, gamma, mode):
    w = W.small_bulk(N=900, seed=13, charged_frac=0.2, box=(7.0, 7.3, 7.1), rc=2.5, grid=(24, 24, 24))
    w.gamma = gamma
    print(f"case half fused steps prec={precision} gamma={gamma}", flush=True)
    runs = []
    for split in (False, True):
        eng = make_engine([w], precision, seed=5, tuning=_t(cells_per_cutoff=2, beads_per_cluster=8, half_pairs=mode))
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


def test_half_falls_back_for_derivatives_and_counts():
    w = W.small_bulk(N=700, seed=3, charged_frac=0.3, box=(7.1, 6.6, 6.3), rc=2.5, grid=(24, 24, 24))
    eng = make_engine([w], "fp64", tuning=_t(cells_per_cutoff=2, beads_per_cluster=8))
    got = gpu_eval(eng, adjoint=True)
    n_half = eng.count_pairs()
    eng.set_tuning(half_pairs=0)
    ref_gpu = gpu_eval(eng, adjoint=True)
    n_full = eng.count_pairs()
    eng.close()
    assert n_half == n_full
    ref = oracle_eval(w, adjoint=True)
    assert rel_rms(got["force"], ref["F"]) < 1e-9
    for k in ("dE_dA", "dE_dsigma", "dE_da"):
        np.testing.assert_allclose(got[k], ref_gpu[k], rtol=1e-12, atol=1e-12)
