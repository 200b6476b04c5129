"""GPU parity of the per-bead radius derivatives dE/dsigma_i and dE/da_i
(the derivative with respect to each bead's own radii at the per-type
values) against the FP64 oracle, through both pair paths."""
import numpy as np
import pytest

import gcme_workloads as W
from oracle import oracle as O
from tests.gpu_common import make_engine, oracle_params, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _check(w, precision, tuning=None, tag=""):
    eng = make_engine([w], precision, tuning=tuning)
    out = eng.forces_energy(adjoint=True, per_bead=True)
    eng.sync()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    eng.close()
    ref = O.per_bead_adjoint(w.pos, w.type, w.z, oracle_params(w))
    es = rel_rms(got["dE_dsigma_bead"], ref["dE_dsigma"])
    ea = rel_rms(got["dE_da_bead"], ref["dE_da"])
    print(f"  {tag}: dE/dsigma_i {es:.2e}  dE/da_i {ea:.2e}", flush=True)
    assert es < TOL[precision] and ea < TOL[precision]
    assert np.all(got["dE_da_bead"][w.z == 0] == 0.0)
    # summed over a type: the engine's own per-type derivatives
    for t in range(w.nt):
        for pb, pt in (("dE_dsigma_bead", "dE_dsigma"), ("dE_da_bead", "dE_da")):
            s = got[pb][w.type == t].sum()
            assert s == pytest.approx(got[pt][0, t], rel=1e-11 if precision == "fp64" else 1e-5,
                                      abs=1e-9 * np.abs(got[pb]).sum())


@pytest.mark.parametrize("direct", [0, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_bead_small(precision, direct):
    w = W.small_bulk(N=900, seed=51, charged_frac=0.3, a_types=(0.35, 0.55, 0.65), box=(7.1, 7.3, 6.9), rc=2.5,
                     grid=(24, 24, 24))
    print(f"case per_bead N={w.N} prec={precision} direct={direct}", flush=True)
    _check(w, precision, tuning=dict(direct_pairs=direct), tag=f"{precision} direct={direct}")


def test_per_bead_bulk_N32768():
    w = W.config2()
    print(f"case per_bead N={w.N} mixed", flush=True)
    _check(w, "mixed", tag="N=32768 mixed")


def test_per_bead_refusals():
    from paper_2403_08148_amd import GCMe, params_from_workload
    from paper_2403_08148_amd._binding import GCMeError, GCME_FLAG_ALL_RECIPROCAL
    w = W.small_bulk(N=300, seed=52, charged_frac=0.2, a_types=(0.5,), box=(5.0, 5.0, 5.0), rc=2.0, grid=(16, 16, 16))
    print("case per_bead_refusals", flush=True)
    eng = make_engine([w], "fp64")
    with pytest.raises(GCMeError, match="EINVAL"):
        eng.step(2, observe=True, per_bead=True)
    eng.close()
    eng = GCMe([w.N], precision="fp64")
    eng.set_params(params_from_workload(w, flags=GCME_FLAG_ALL_RECIPROCAL, grid=(32, 32, 32)))
    eng.set_state(w.pos, w.type, w.z, w.vel)
    with pytest.raises(GCMeError, match="EUNSUPPORTED"):
        eng.forces_energy(per_bead=True)
    eng.close()
