"""GPU parity of the goal-oriented (QoI) phases through the C ABI against the
FP64 oracle (oracle/posterior.py): the multi-rate p2q map F_q (QoIs every
r-th parameter step) and its adjoint, the cross products F F_q^* and
F_q F^*, the data-to-QoI map Q and the online prediction Q d, and the QoI
posterior covariance, with the stand-in prior gamma I.  Tolerances: 1e-12 /
2e-3 (FP64 / FP16 spectra) for the maps; 1e-10 for the FP64 pipelines that
go through K's factor."""
import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
from oracle import posterior as OP  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2OOperator, cholesky, d2q_apply  # noqa: E402

DEV = "cuda"
WF = synth.Workload("qoi_data", Nd=6, Nm=300, Nt=60, tau=10.0)
WQ = synth.Workload("qoi_map", Nd=3, Nm=300, Nt=60, tau=10.0, seed=synth.SEED + 50)
STRIDE = 5                                   # 12 QoI steps of the 60 parameter steps
TOL = {"fp64": 1e-12, "fp16": 2e-3}


def note(msg):
    print(msg, flush=True)


def build(w, precision, max_rhs=16, stride=1):
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=max_rhs, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    if stride > 1:
        op.set_output_stride(stride)
    return op, F


def dev(x, op):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, op.dtype)


def host(x):
    torch.cuda.synchronize()
    return x.double().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp16"])
def test_multirate_p2q_and_cross_products(precision):
    op, F = build(WF, precision)
    oq, Fq = build(WQ, precision, stride=STRIDE)
    nrhs, Ntq = 5, WQ.Nt // STRIDE
    rng = np.random.default_rng(1)
    m = synth.param_series(WF, nrhs)
    q = rng.standard_normal((nrhs, Ntq, WQ.Nd))
    z = synth.data_series(WF, nrhs)
    got = {"Fq m": host(oq.apply_F(dev(m, oq))), "Fq* q": host(oq.apply_Ft(dev(q, oq))),
           "Fq Fq* q": host(oq.apply_FFt(dev(q, oq))), "F Fq* q": host(op.apply_FGt(oq, dev(q, oq))),
           "Fq F* z": host(oq.apply_FGt(op, dev(z, op)))}
    want = {"Fq m": OP.apply_Fq(Fq, m, STRIDE), "Fq* q": OP.apply_Fqt(Fq, q, STRIDE),
            "Fq Fq* q": OP.apply_Fq(Fq, OP.apply_Fqt(Fq, q, STRIDE), STRIDE),
            "F Fq* q": oracle.apply_F(F, OP.apply_Fqt(Fq, q, STRIDE)),
            "Fq F* z": OP.apply_Fq(Fq, oracle.apply_Ft(F, z), STRIDE)}
    for k in want:
        assert got[k].shape == want[k].shape, (k, got[k].shape, want[k].shape)
        errs = [oracle.rel_l2(got[k][b], want[k][b]) for b in range(nrhs)]
        note(f"[qoi] {precision} {k}: worst rel-L2 {max(errs):.2e}")
        assert max(errs) <= TOL[precision], (k, errs)


def test_d2q_map_prediction_and_qoi_covariance():
    rng = np.random.default_rng(2)
    var, gam = rng.uniform(0.5, 2.0, WF.Nd) * 0.05, 0.8
    op, F = build(WF, "fp64", max_rhs=16)
    oq, Fq = build(WQ, "fp64", max_rhs=16, stride=STRIDE)
    L = cholesky(op.assemble_K(torch.from_numpy(var).to(DEV), prior_var=gam))
    Lo = OP.cholesky_lower(OP.data_space_matrix(F, var, gam))
    Q = op.d2q_map(oq, L, torch.from_numpy(var).to(DEV), gam, batch=7)       # ragged last batch
    Qo = OP.d2q_matrix(Fq, F, var, gam, STRIDE, Lo)
    eq = np.linalg.norm(Q.cpu().numpy() - Qo) / np.linalg.norm(Qo)
    note(f"[qoi] d2q map Q {Qo.shape}: rel {eq:.2e}")
    assert eq <= 1e-10
    d = synth.data_series(WF, 3)
    qp = d2q_apply(Q, torch.from_numpy(d.reshape(3, -1)).to(DEV)).cpu().numpy()
    for b in range(3):
        want = OP.apply_Fq(Fq, OP.map_point(F, d[b], var, gam, Lo), STRIDE).reshape(-1)
        assert oracle.rel_l2(qp[b], want) <= 1e-10
    C = op.qoi_posterior_cov(oq, L, gam, batch=9)
    Co = OP.qoi_posterior_cov(Fq, F, var, gam, STRIDE, Lo)
    ec = np.linalg.norm(C.cpu().numpy().T - Co) / np.linalg.norm(Co)
    note(f"[qoi] Gamma_post(q) {Co.shape}: rel {ec:.2e}")
    assert ec <= 1e-10


def test_multirate_option_checks():
    oq, _ = build(WQ, "fp64", stride=1)
    from paper_2501_14911_amd import P2OError
    with pytest.raises(P2OError):
        oq.set_output_stride(7)                        # does not divide Nt = 60
    oq.set_output_stride(STRIDE)
    m = torch.zeros((1, WQ.Nt, WQ.Nm), dtype=torch.float64, device=DEV)
    from paper_2501_14911_amd._lib import lib
    from ctypes import c_void_p
    dq = torch.zeros((1, WQ.Nt, WQ.Nd), dtype=torch.float64, device=DEV)
    var = torch.ones(1, dtype=torch.float64, device=DEV)
    g = torch.zeros_like(m)
    phi = torch.zeros(1, dtype=torch.float64, device=DEV)
    st = lib.p2o_misfit_grad(oq._plan, c_void_p(m.data_ptr()), c_void_p(dq.data_ptr()), c_void_p(var.data_ptr()), 1,
                             c_void_p(g.data_ptr()), c_void_p(phi.data_ptr()), 1, None)
    assert st == -2                                    # P2O_ERR_STATE: the misfit needs every step
    with pytest.raises(P2OError):
        oq.apply_F(m, nt_active=[30])                  # ragged lengths need stride 1
