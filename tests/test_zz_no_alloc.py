"""The entry point that allocates no device memory,
gcme_forces_energy_noalloc, called through the C ABI, against the existing
gcme_forces_energy of a context on the same inputs (same kernels and
tuning: forces summed exactly in fixed point, partial sums reduced in a
fixed order, so the outputs are bit-identical).  Two calls in a row, the
second on a smaller system, so that nothing of the first call's scratch
contents reaches the second; and a system too large for the scratch is
refused before any kernel runs."""
import ctypes as C

import numpy as np
import pytest

import gcme_workloads as W
from tests.gpu_common import make_engine

pytestmark = pytest.mark.gpu


def _noalloc(w, precision):
    import torch
    from paper_2403_08148_amd import _binding as B
    from paper_2403_08148_amd.engine import c_params
    from paper_2403_08148_amd import params_from_workload
    L = B.load()
    dev = torch.device("cuda", 0)
    pos = torch.tensor(np.ascontiguousarray(w.pos.T), dtype=torch.float64, device=dev)
    typ = torch.tensor(w.type, dtype=torch.int32, device=dev)
    z = torch.tensor(w.z, dtype=torch.int32, device=dev)
    F = torch.full((3, w.N), np.nan, dtype=torch.float64, device=dev)
    E = torch.full((B.GCME_N_TERMS,), np.nan, dtype=torch.float64, device=dev)
    V = torch.full((6,), np.nan, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    cp, keep = c_params(params_from_workload(w))
    prec = B.GCME_FP64 if precision == "fp64" else B.GCME_MIXED
    st = L.gcme_forces_energy_noalloc(C.byref(cp), w.N, prec, C.c_void_p(pos.data_ptr()),
                                      C.c_void_p(typ.data_ptr()), C.c_void_p(z.data_ptr()),
                                      C.c_void_p(F.data_ptr()), C.c_void_p(E.data_ptr()),
                                      C.c_void_p(V.data_ptr()), C.c_void_p(stream.cuda_stream))
    B.check(None, st)
    torch.cuda.current_stream(dev).wait_stream(stream)
    torch.cuda.synchronize()
    return F.cpu().numpy().T.copy(), E.cpu().numpy(), V.cpu().numpy()


def _context(w, precision):
    eng = make_engine([w], precision)
    out = eng.forces_energy()
    eng.sync()
    res = (out["force"].cpu().numpy().T.copy(), out["energy"].cpu().numpy()[0], out["virial"].cpu().numpy()[0])
    eng.close()
    return res


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_context_two_calls(precision):
    big = W.small_bulk(N=3000, seed=41, charged_frac=0.3, a_types=(0.4, 0.6), box=(10.6, 10.7, 10.8), rc=2.5,
                       grid=(32, 32, 32))
    small = W.small_bulk(N=700, seed=42, charged_frac=0.2, a_types=(0.5,), box=(6.6, 6.5, 6.7), rc=2.4,
                         grid=(24, 24, 24))
    for w in (big, small):
        print(f"case noalloc {w.name} N={w.N} prec={precision}", flush=True)
        F, E, V = _noalloc(w, precision)
        Fc, Ec, Vc = _context(w, precision)
        assert np.all(np.isfinite(F)) and np.all(np.isfinite(E)) and np.all(np.isfinite(V))
        np.testing.assert_array_equal(F, Fc)
        np.testing.assert_array_equal(E, Ec)
        np.testing.assert_array_equal(V, Vc)
        print(f"  bit-identical to the context's evaluation (|F|max {np.abs(F).max():.3e})", flush=True)


def test_noalloc_refuses_a_system_beyond_its_scratch():
    import torch
    from paper_2403_08148_amd import _binding as B
    from paper_2403_08148_amd.engine import c_params
    from paper_2403_08148_amd import params_from_workload
    L = B.load()
    # bead buffers alone exceed the scratch; nothing is launched
    n = B.GCME_NOALLOC_SCRATCH_BYTES // 64
    w = W.small_bulk(N=300, seed=43, box=(5.0, 5.0, 5.0), rc=2.4)
    cp, keep = c_params(params_from_workload(w))
    print(f"case noalloc too large N={n}", flush=True)
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = L.gcme_forces_energy_noalloc(C.byref(cp), n, B.GCME_MIXED, C.c_void_p(dummy.data_ptr()),
                                      C.c_void_p(dummy.data_ptr()), C.c_void_p(dummy.data_ptr()), None, None, None,
                                      None)
    assert st == B.GCME_ENOMEM
    msg = L.gcme_last_error(None).decode()
    print(f"  refused: {msg}", flush=True)
    assert "scratch" in msg
    torch.cuda.synchronize()
