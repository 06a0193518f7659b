"""The allocation-free entry point usp_residual_static: the FP64 true residual
computed with every temporary in the library's static device scratch.  Checked
against usp_residual of a prepared operator (same kernels, same launch shapes:
identical bits) on calls in a row with shrinking grids, and against the FP64
oracle's residual; a grid whose temporaries exceed the scratch is rejected
before any device work."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import oracle_helmholtz, to_np
from oracle import richardson as R
from paper_2207_14222_amd import media

pytestmark = pytest.mark.gpu

DPT = ct.POINTER(ct.c_double)


def _static(sym, dt, B, y, x):
    from paper_2207_14222_amd import _lib as L
    rel, rn, yn = np.zeros(1), np.zeros(1), np.zeros(1)
    stream = ct.c_void_p(torch.cuda.current_stream(B.device).cuda_stream)
    L.check(L.lib().usp_residual_static(ct.byref(sym), dt, ct.c_void_p(B.data_ptr()), ct.c_void_p(y.data_ptr()),
                                        ct.c_void_p(x.data_ptr()), rel.ctypes.data_as(DPT), rn.ctypes.data_as(DPT),
                                        yn.ctypes.data_as(DPT), stream))
    return float(rel[0]), float(rn[0]), float(yn[0])


@pytest.mark.parametrize("order", ["large_first", "small_first"])
def test_static_residual_equals_handle_residual(order):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14222_amd import _lib as L, solver
    cases = [((32, 64, 128), "c128"), ((16, 32), "c64"), ((256,), "c128")]
    if order == "small_first":
        cases = cases[::-1]
    for shape, dt in cases:
        print(f"[gpu-case] static residual {shape} {dt}", flush=True)
        if len(shape) == 1:
            p = media.helmholtz_1d(n=shape[0])
        else:
            p = media.helmholtz_spheres(shape=shape, count=4, width=2, w0=2.0, plane=1, seed=31)
        tdt = torch.complex128 if dt == "c128" else torch.complex64
        can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=tdt)
        op = solver.Operator(can.symbol, can.B)
        x, _ = op.iterate(can.y, alpha=0.8, K=5)
        ref = op.residual(can.y, x)
        got = _static(can.symbol, L.USP_C128 if dt == "c128" else L.USP_C64, can.B, can.y, x)
        assert got == ref, (shape, dt, got, ref)
        if dt == "c128":
            cp, op_o = oracle_helmholtz(p)
            rho_o = R.relative_residual(op_o, to_np(x), cp.y)
            assert abs(got[0] - rho_o) < 1e-10 * rho_o


def test_static_residual_rejects_grids_beyond_the_scratch():
    from paper_2207_14222_amd import _lib as L, solver
    sym = solver.make_symbol((256, 256, 256), (0.25,) * 3, s=1j, a0=2.0, a2=-1.0)
    rel = np.zeros(1)
    # rejected from the sizes alone: the (never dereferenced) pointers are placeholders
    rc = L.lib().usp_residual_static(ct.byref(sym), L.USP_C128, ct.c_void_p(256), ct.c_void_p(256),
                                     ct.c_void_p(256), rel.ctypes.data_as(DPT), None, None, None)
    assert rc == L.USP_ERR_WORKSPACE
    assert "static scratch" in L.last_error()
