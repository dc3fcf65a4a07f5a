"""The allocation-free entry point p2o_apply_F_noalloc through the C ABI
(ctypes), against p2o_apply_F on the same plan and inputs: two calls in a
row, the second with fewer right-hand sides and other ragged lengths, each
bitwise equal to the existing entry point's result (same kernels, same
arithmetic) and within the FP64 oracle's tolerance; and the size check."""
import ctypes
from ctypes import c_void_p

import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2OOperator  # noqa: E402
from paper_2501_14911_amd._lib import lib  # noqa: E402

DEV = "cuda"


def _run(fn, op, m, nrhs, nt):
    d = torch.full((nrhs, op.Nt, op.Nd), float("nan"), dtype=op.dtype, device=DEV)
    op._stream()
    st = fn(op._plan, c_void_p(m.data_ptr()), c_void_p(d.data_ptr()), nrhs,
            c_void_p(nt.data_ptr()) if nt is not None else None)
    assert st == 0, lib.p2o_last_error().decode()
    torch.cuda.synchronize()
    return d


@pytest.mark.parametrize("precision", ["bf16", "fp64"])
def test_noalloc_matches_apply_F(precision):
    w = synth.Workload("noalloc", Nd=37, Nm=9000, Nt=21, tau=6.0)
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=8, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    for nrhs, nt in ((8, np.array([21, 5, 0, 21, 13, 1, 20, 21], dtype=np.int32)), (3, None)):
        m_h = synth.param_series(w, nrhs, seed_offset=3 + nrhs)
        m = torch.from_numpy(m_h).to(DEV, op.dtype)
        nt_d = torch.from_numpy(nt).to(DEV) if nt is not None else None
        ref = _run(lib.p2o_apply_F, op, m, nrhs, nt_d)
        got = _run(lib.p2o_apply_F_noalloc, op, m, nrhs, nt_d)
        assert torch.equal(got, ref), (precision, nrhs)
        tol = 1e-12 if precision == "fp64" else 2e-3
        want = oracle.apply_F(F, m_h, nt)
        assert oracle.rel_l2(got.double().cpu().numpy(), want) <= tol


def test_noalloc_rejects_oversized_calls():
    w = synth.CONFIGS["medium"]
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp64", max_rhs=64, device=DEV)
    F = torch.from_numpy(synth.operator_blocks(w)).to(DEV)
    op.load(lambda c0, n: F[:, :, c0:c0 + n])
    m = torch.zeros((64, w.Nt, w.Nm), dtype=torch.float64, device=DEV)
    d = torch.zeros((64, w.Nt, w.Nd), dtype=torch.float64, device=DEV)
    st = lib.p2o_apply_F_noalloc(op._plan, c_void_p(m.data_ptr()), c_void_p(d.data_ptr()), 64, None)
    assert st == -1 and "scratch" in lib.p2o_last_error().decode()
    # a call that fits still works on the same plan afterwards
    st = lib.p2o_apply_F_noalloc(op._plan, c_void_p(m.data_ptr()), c_void_p(d.data_ptr()), 1, None)
    assert st == 0, lib.p2o_last_error().decode()
    torch.cuda.synchronize()
