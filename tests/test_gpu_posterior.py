"""GPU parity of the offline and online phases (data-space matrix K, its
Cholesky factor and solves, MAP point, posterior-covariance actions) through
the C ABI against the FP64 oracle (oracle/posterior.py), with the stand-in
prior Gamma_prior = gamma I.

Tolerances: K's columns carry the operator's own error (1e-12 FP64, 1e-5
FP32, 2e-3 FP16 per column).  The factorisation and the solves are FP64 on
both sides and are checked on the oracle's own K: backward error
||L L^T - K|| / ||K|| <= 1e-14 (blocked Cholesky is backward stable), and the
factor and solutions against numpy's within 1e-11 at the condition numbers
used (K = Gamma_noise + gamma F F^T with the noise chosen to keep cond(K)
below 1e3).  The MAP point and the posterior actions on an FP64 plan follow
from these: 1e-10."""
import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
from oracle import posterior as OP  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2OOperator, cholesky, cholesky_solve  # noqa: E402

DEV = "cuda"
SMALL = synth.Workload("post_small", Nd=8, Nm=512, Nt=63, tau=8.0)       # N = 504: ragged last 64-block


def note(msg):
    print(msg, flush=True)


def build(w, precision, max_rhs):
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=max_rhs, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    return op, F


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp16", 2e-3)])
def test_assemble_K(precision, tol):
    w = SMALL
    rng = np.random.default_rng(1)
    var = rng.uniform(0.5, 2.0, w.Nd) * 0.05
    op, F = build(w, precision, max_rhs=40)               # 504 columns in batches of 40 (ragged last)
    K = op.assemble_K(torch.from_numpy(var).to(DEV), prior_var=0.7)
    Ko = OP.data_space_matrix(F, var, prior_var=0.7)
    Kg = K.cpu().numpy().T                                # tensor row j = column j of K
    errs = np.linalg.norm(Kg - Ko, axis=0) / np.linalg.norm(Ko, axis=0)
    note(f"[posterior] K {precision}: worst column rel-L2 {errs.max():.3e}")
    assert errs.max() <= tol


@pytest.mark.parametrize("chunk", [512, 100])
def test_assemble_K_from_blocks(chunk):
    """K from the blocks' Gram matrix (FP64 matrix cores, block-diagonal
    prefix sums) against the oracle's K: FP64 rounding only; exactly
    symmetric; and against the column-by-column assembly on an FP64
    spectrum.  chunk 100: six column chunks of the blocks, the last ragged."""
    from paper_2501_14911_amd import assemble_K_from_blocks
    w = SMALL
    rng = np.random.default_rng(4)
    var = rng.uniform(0.5, 2.0, w.Nd) * 0.05
    gam = 0.8
    F = synth.operator_blocks(w)
    Ft = torch.from_numpy(F).to(DEV)
    K = assemble_K_from_blocks(lambda c0, n: Ft[:, :, c0:c0 + n], w.Nd, w.Nm, w.Nt, torch.from_numpy(var).to(DEV),
                               prior_var=gam, chunk_cols=chunk, device=DEV)
    Kg = K.cpu().numpy()
    Ko = OP.data_space_matrix(F, var, gam)
    err = np.linalg.norm(Kg.T - Ko) / np.linalg.norm(Ko)
    note(f"[posterior] K from blocks (chunk {chunk}): rel err {err:.2e}")
    assert err <= 1e-13
    assert np.array_equal(Kg, Kg.T)
    op, _ = build(w, "fp64", max_rhs=64)
    Kc = op.assemble_K(torch.from_numpy(var).to(DEV), prior_var=gam).cpu().numpy()
    assert np.linalg.norm(Kc - Kg) / np.linalg.norm(Kg) <= 1e-12


def test_cholesky_and_solve_on_oracle_K():
    w = SMALL
    F = synth.operator_blocks(w)
    Ko = OP.data_space_matrix(F, 0.05, prior_var=1.0)
    N = Ko.shape[0]
    note(f"[posterior] cond(K) {np.linalg.cond(Ko):.2e}")
    K = torch.from_numpy(Ko.T.copy()).to(DEV)
    L = cholesky(K)
    Lg = np.tril(L.cpu().numpy().T)                       # lower triangle of the column-major factor
    Lo = OP.cholesky_lower(Ko)
    back = np.linalg.norm(Lg @ Lg.T - Ko) / np.linalg.norm(Ko)
    fwd = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    note(f"[posterior] Cholesky: backward error {back:.2e}, factor vs numpy {fwd:.2e}")
    assert back <= 1e-14 and fwd <= 1e-11
    # the strict upper triangle of the column-major matrix holds L^T, bit for bit
    upper = np.triu(np.ones((N, N), dtype=bool), 1)
    assert np.array_equal(L.cpu().numpy().T[upper], Lg.T[upper])
    rng = np.random.default_rng(2)
    for nrhs in (1, 3):
        B = rng.standard_normal((nrhs, N))
        X = cholesky_solve(L, torch.from_numpy(B).to(DEV)).cpu().numpy()
        Xo = OP.solve_with_factor(Lo, B.T).T
        err = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
        note(f"[posterior] solve vs oracle ({nrhs} right-hand sides) {err:.2e}")
        assert err <= 1e-11


def test_cholesky_panels_on_random_spd():
    """Five 256-column panels (the last of 76 columns, its last 64-block of
    12), 128-row update tiles with a ragged last row: factor against numpy's,
    backward error, L^T in the upper triangle, solves against numpy's."""
    n = 1100
    rng = np.random.default_rng(5)
    R = rng.standard_normal((n, n))
    Ko = R @ R.T / n + np.eye(n)
    L = cholesky(torch.from_numpy(Ko.T.copy()).to(DEV)).cpu().numpy().T
    Lg = np.tril(L)
    Ln = np.linalg.cholesky(Ko)
    back = np.linalg.norm(Lg @ Lg.T - Ko) / np.linalg.norm(Ko)
    fwd = np.linalg.norm(Lg - Ln) / np.linalg.norm(Ln)
    note(f"[posterior] Cholesky n={n}: backward error {back:.2e}, factor vs numpy {fwd:.2e}")
    assert back <= 1e-14 and fwd <= 1e-12
    upper = np.triu(np.ones((n, n), dtype=bool), 1)
    assert np.array_equal(L[upper], Lg.T[upper])
    # 1 right-hand side (one launch per block), 5 (one row per lane updates), 40 and 70 (matrix-core
    # updates, ragged right-hand-side tiles)
    for nrhs in (1, 5, 40, 70):
        B = rng.standard_normal((nrhs, n))
        X = cholesky_solve(torch.from_numpy(L.T.copy()).to(DEV), torch.from_numpy(B).to(DEV)).cpu().numpy()
        Xn = np.linalg.solve(Ko, B.T).T
        err = np.linalg.norm(X - Xn) / np.linalg.norm(Xn)
        note(f"[posterior] solve n={n} nrhs={nrhs}: {err:.2e}")
        assert err <= 1e-12


def test_cholesky_reports_non_positive_pivot():
    A = -torch.eye(70, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError, match="pivot 0"):
        cholesky(A)
    B = torch.eye(130, dtype=torch.float64, device=DEV)
    B[100, 100] = -1.0                                   # in the second diagonal block
    with pytest.raises(ValueError, match="pivot 100"):
        cholesky(B)
    C = torch.eye(600, dtype=torch.float64, device=DEV)
    C[300, 300] = -1.0                                   # second panel; the first failure is reported
    C[500, 500] = -2.0
    with pytest.raises(ValueError, match="pivot 300"):
        cholesky(C)
    # a later call on a good matrix resets the report
    cholesky(torch.eye(600, dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_map_point_and_posterior_actions(precision, tol):
    w = SMALL
    rng = np.random.default_rng(3)
    var = rng.uniform(0.5, 2.0, w.Nd * w.Nt) * 0.05
    gam = 0.6
    op, F = build(w, precision, max_rhs=64)
    L = cholesky(op.assemble_K(torch.from_numpy(var).to(DEV), prior_var=gam))
    Lo = OP.cholesky_lower(OP.data_space_matrix(F, var, gam))
    d = synth.data_series(w, 2)
    m = op.map_point(torch.from_numpy(d).to(DEV, op.dtype), L, torch.from_numpy(var).to(DEV), gam)
    m = m.double().cpu().numpy()
    for b in range(2):
        mo = OP.map_point(F, d[b], var, gam, Lo)
        e = oracle.rel_l2(m[b], mo)
        note(f"[posterior] MAP {precision} rhs {b}: {e:.2e}")
        assert e <= tol
    # a single data vector takes the one-launch-per-block solves
    m1 = op.map_point(torch.from_numpy(d[1]).to(DEV, op.dtype), L, torch.from_numpy(var).to(DEV), gam)
    e1 = oracle.rel_l2(m1.double().cpu().numpy(), OP.map_point(F, d[1], var, gam, Lo))
    note(f"[posterior] MAP {precision} single data vector: {e1:.2e}")
    assert e1 <= tol
    v = synth.param_series(w, 2)
    g = op.posterior_cov_apply(torch.from_numpy(v).to(DEV, op.dtype), L, gam).double().cpu().numpy()
    for b in range(2):
        go = OP.posterior_cov_apply(F, v[b], var, gam, Lo)
        e = oracle.rel_l2(g[b], go)
        note(f"[posterior] Gamma_post v {precision} rhs {b}: {e:.2e}")
        assert e <= tol
