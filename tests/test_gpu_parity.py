"""GPU parity: the HIP engine against the FP64 oracle on the same seeded
inputs (oracle in SPME-matched mode: same mesh and order).

Tolerances: FP64 engine -- 1e-9 relative RMS force error and 1e-10 relative
energy error per term (fixed-point forces at 2^-40, everything else FP64).
Mixed engine -- the target of the method: 1e-5 relative RMS force error and
1e-6 relative energy error per term against the FP64 oracle.  Per bead,
max_i |dF_i| / max(|F_i|, F_rms) is held to ten times the RMS tolerance.
These inputs lie on the engine's 2^-32 L position lattice; the same checks on
general positions are in test_gpu_general_inputs.py.
"""
import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import energy_errors, gpu_eval, make_engine, oracle_eval, per_bead_err, rel, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-9, 1e-10), "mixed": (1e-5, 1e-6)}


def _check(w, precision, tuning=None, etol=None):
    print(f"case {w.name} N={w.N} grid={w.grid} box={w.box} prec={precision} tuning={tuning}", flush=True)
    eng = make_engine([w], precision, tuning=tuning)
    got = gpu_eval(eng)
    eng.close()
    ref = oracle_eval(w)
    ftol, et = TOL[precision]
    if etol is not None:
        et = etol
    ferr = rel_rms(got["force"], ref["F"])
    fb = per_bead_err(got["force"], ref["F"])
    eerr = energy_errors(got["energy"][0, :5], ref["E"])
    werr = rel_rms(got["virial"][0], ref["W"])
    print(f"  force {ferr:.2e} per-bead {fb:.2e} energy {np.array2string(eerr, precision=2)} virial {werr:.2e}",
          flush=True)
    assert ferr < ftol
    assert fb < 10 * ftol
    assert np.all(eerr < et), eerr
    assert werr < max(ftol, et) * 10
    assert got["energy"][0, 5] == pytest.approx(got["energy"][0, :5].sum(), rel=1e-14)
    return got, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_box_parity(precision):
    w = W.small_bulk(N=700, seed=3, charged_frac=0.3, box=(7.1, 6.6, 6.3), rc=2.5, grid=(24, 24, 24))
    _check(w, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tuning", [dict(cells_per_cutoff=1, beads_per_cluster=2, charges_per_cluster=8,
                                         direct_pairs=0, stream_layout=0),
                                    dict(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=2,
                                         direct_pairs=0, stream_layout=0),
                                    dict(cells_per_cutoff=4, beads_per_cluster=4, charges_per_cluster=4,
                                         direct_pairs=0, stream_layout=0),
                                    dict(cells_per_cutoff=1, beads_per_cluster=8, charges_per_cluster=2,
                                         direct_pairs=3),
                                    dict(cells_per_cutoff=2, beads_per_cluster=2, charges_per_cluster=4,
                                         direct_pairs=1),
                                    dict(cells_per_cutoff=4, beads_per_cluster=4, charges_per_cluster=8,
                                         direct_pairs=2),
                                    dict(cells_per_cutoff=3, beads_per_cluster=4, charges_per_cluster=2,
                                         direct_pairs=3, stream_layout=1),
                                    dict(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=4,
                                         direct_pairs=1, stream_layout=2),
                                    dict(cells_per_cutoff=2, beads_per_cluster=4, charges_per_cluster=4,
                                         direct_pairs=0, stream_layout=3),
                                    dict(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=2,
                                         direct_pairs=2, stream_layout=4),
                                    dict(cells_per_cutoff=4, beads_per_cluster=2, charges_per_cluster=4,
                                         direct_pairs=3, stream_layout=5)])
def test_tunings_parity(precision, tuning):
    w = W.small_bulk(N=1001, seed=4, charged_frac=0.25, a_types=(0.3, 0.5, 0.7), box=(7.7, 8.3, 6.5),
                     rc=2.6, grid=(27, 36, 24), order=4)
    _check(w, precision, tuning)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tile", [(8, 8, 0, 0), (16, 4, 2, 2), (2, 8, 16, 16), (16, 16, 1, 1), (1, 1, 8, 4)])
def test_mesh_tile_shapes(precision, tile):
    # the fused spread and gather passes with other z-line tiles (spread x,
    # y, gather x, y; 0 = the spread's), ragged at the mesh edges (27 and
    # 36 lines are not multiples of 8 or 16)
    w = W.small_bulk(N=1001, seed=4, charged_frac=0.25, a_types=(0.3, 0.5, 0.7), box=(7.7, 8.3, 6.5),
                     rc=2.6, grid=(27, 36, 24), order=4)
    _check(w, precision, dict(mesh_tile_x=tile[0], mesh_tile_y=tile[1], gather_tile_x=tile[2],
                              gather_tile_y=tile[3]))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("grid", [(128, 128, 24), (128, 128, 27), (96, 128, 24)])
def test_line_batched_mesh_passes(precision, grid):
    # planes too large for the fused y/x pass: the line-batched y and x
    # passes, with the transforms fixed at compile time when K0 = K1 = 128
    # (both precisions), at run time otherwise; odd and even z lengths
    w = W.small_bulk(N=800, seed=21, charged_frac=0.4, box=(7.4, 7.9, 6.8), rc=2.5, grid=grid)
    _check(w, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order,tile", [(3, (2, 4)), (8, (4, 2)), (6, (3, 5))])
def test_line_layout_orders_and_gather_tiles(precision, order, tile):
    # a mesh in line layout (its plane does not fit LDS) with other orders,
    # an odd z length and gather tiles ragged at the mesh edges
    w = W.small_bulk(N=700, seed=23, charged_frac=0.4, box=(7.4, 7.9, 6.8), rc=2.5, grid=(96, 128, 27),
                     order=order)
    _check(w, precision, dict(gather_tile_x=tile[0], gather_tile_y=tile[1]))


@pytest.mark.parametrize("order", [3, 6, 8])
def test_orders_and_odd_mesh(order):
    w = W.small_bulk(N=512, seed=5, charged_frac=0.5, a_types=(0.45,), box=(6.0, 6.0, 6.0), rc=2.5,
                     grid=(18, 27, 32), order=order)
    _check(w, "fp64")


def test_config1_fp64_and_method_error():
    w = W.config1()
    got, ref = _check(w, "fp64")
    # method error of SPME 32^3 order 5 against the exact k-sum |k| <= 8
    ex = oracle_exact(w)
    ferr = rel_rms(got["force"], ex["F"])
    print(f"  config1 method error vs exact Ewald: force {ferr:.2e}", flush=True)
    assert ferr < 1e-3


def oracle_exact(w):
    from oracle import oracle as O
    from tests.gpu_common import oracle_params
    return O.forces(w.pos, w.type, w.z, oracle_params(w), recip_mode=O.RECIP_EWALD, kmax=w.kmax)


def test_config2_mixed_full_size():
    w = W.config2()
    _check(w, "mixed")


def test_deterministic_reruns():
    w = W.small_bulk(N=900, seed=6, charged_frac=0.3, box=(7.0, 7.0, 7.2), rc=2.4, grid=(24, 24, 24))
    eng = make_engine([w], "mixed")
    a = gpu_eval(eng)
    b = gpu_eval(eng)
    eng.close()
    np.testing.assert_array_equal(a["force"], b["force"])
    np.testing.assert_array_equal(a["energy"], b["energy"])
    np.testing.assert_array_equal(a["virial"], b["virial"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tuning", [dict(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=4, direct_pairs=3),
                                    dict(cells_per_cutoff=2, beads_per_cluster=4, charges_per_cluster=2, direct_pairs=3),
                                    dict(cells_per_cutoff=3, beads_per_cluster=8, charges_per_cluster=4, direct_pairs=0)])
def test_forces_only_pass_parity(precision, tuning):
    # The pass a step runs (forces, no energy or virial) has kernels of its
    # own (no per-pair validity test in the list-free excluded-volume kernel,
    # a padded final drain): its forces against the oracle at full size.
    w = W.config2()
    print(f"case forces-only {w.name} prec={precision} tuning={tuning}", flush=True)
    eng = make_engine([w], precision, tuning=tuning)
    F = eng.forces_energy(energy=False, virial=False)["force"]
    eng.sync()
    F = F.cpu().numpy().T
    eng.close()
    ref = oracle_eval(w)
    ferr = rel_rms(F, ref["F"])
    fb = per_bead_err(F, ref["F"])
    print(f"  force {ferr:.2e} per-bead {fb:.2e}", flush=True)
    assert ferr < TOL[precision][0]
    assert fb < 10 * TOL[precision][0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_forces_only_small_boxes(precision):
    # clusters outside the first-bead frame (boxes near 2 rc) in the forces-only pass
    for w in (W.small_bulk(N=350, seed=13, charged_frac=0.4, box=(5.2, 5.3, 5.05), rc=2.5, grid=(16, 16, 16)),
              W.small_bulk(N=1001, seed=4, charged_frac=0.25, a_types=(0.3, 0.5, 0.7), box=(7.7, 8.3, 6.5),
                           rc=2.6, grid=(27, 36, 24), order=4)):
        for ci in (2, 4, 8):
            eng = make_engine([w], precision, tuning=dict(cells_per_cutoff=3, beads_per_cluster=ci, direct_pairs=3))
            F = eng.forces_energy(energy=False, virial=False)["force"]
            eng.sync()
            F = F.cpu().numpy().T
            eng.close()
            Fr = oracle_eval(w)["F"]
            ferr, fb = rel_rms(F, Fr), per_bead_err(F, Fr)
            print(f"case forces-only {w.name} box={w.box} CI={ci} prec={precision}: force {ferr:.2e} "
                  f"per-bead {fb:.2e}", flush=True)
            assert ferr < TOL[precision][0]
            assert fb < 10 * TOL[precision][0]
