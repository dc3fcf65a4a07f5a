"""Full-size GPU parity in the launch configurations the benchmark times.

The 600 x 16384 x 420 workload (BF16 and FP16 spectra, 16.5 GB each; FP32,
33 GB; FP64, 66 GB) and the 600 x 65536 x 420 one-GPU share (BF16, 66 GB).  Blocks are drawn on the GPU
with the counter-based generator; the FP64 oracle regenerates on the CPU
only the sensor rows (for F m and F F* e) or parameter columns (for F* d) it
checks, and computes those outputs exactly.  Where the oracle would need
the whole operator (the misfit value), properties that hold at any size are
checked instead: central differences of the quadratic misfit, the adjoint
identity, and the gradient's agreement with the autograd path.
"""
import sys

import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2O, P2OOperator, misfit  # noqa: E402

TOL = 2e-3
DEV = "cuda"


def note(msg):
    print(msg, flush=True)


def gpu_blocks(w, c0, n, lag_batch=35):
    out = torch.empty((w.Nt, w.Nd, n), dtype=torch.float64, device=DEV)
    cols = torch.arange(c0, c0 + n, device=DEV)
    for k0 in range(0, w.Nt, lag_batch):
        ks = list(range(k0, min(w.Nt, k0 + lag_batch)))
        out[k0:k0 + len(ks)] = synth.operator_rows_cols(w, ks, cols=cols, backend="torch", device=DEV)
    return out


def rows_of_blocks(w, rows):
    return synth.operator_rows_cols(w, range(w.Nt), rows=np.asarray(rows), backend="torch").numpy()


def cols_of_blocks(w, cols):
    return synth.operator_rows_cols(w, range(w.Nt), cols=np.asarray(cols), backend="torch").numpy()


def load_op(w, precision, max_rhs):
    note(f"[fullsize] loading {w.name} {precision}")
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=max_rhs, device=DEV)
    op.load(lambda c0, n: gpu_blocks(w, c0, n))
    return op


def close_op(op):
    op.close()
    del op
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def paper_time():
    w = synth.CONFIGS["paper_time"]
    op = load_op(w, "bf16", 64)
    yield w, op
    close_op(op)


def single_rhs_errors(w, op, nrows=6, ncols=48, seed=11):
    """F m on random sensor rows and F* d on random parameter columns of the
    outputs, against the oracle on those rows / columns of every block.  The
    inputs are N(0, 1) series with no structure, so the sampled error is an
    unbiased estimate of the whole output's."""
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(w.Nd, nrows, replace=False))
    cols = np.sort(rng.choice(w.Nm, ncols, replace=False))
    m = synth.param_series(w, 1)[0]
    d = synth.data_series(w, 1)[0]
    y = op.apply_F(torch.from_numpy(m).to(DEV, op.dtype)).double().cpu().numpy()
    s = op.apply_Ft(torch.from_numpy(d).to(DEV, op.dtype)).double().cpu().numpy()
    ey = oracle.rel_l2(y[:, rows], oracle.apply_F(rows_of_blocks(w, rows), m))
    es = oracle.rel_l2(s[:, cols], oracle.apply_Ft(cols_of_blocks(w, cols), d))
    return ey, es


def test_paper_time_single_rhs(paper_time):
    w, op = paper_time
    ey, es = single_rhs_errors(w, op)
    note(f"  bf16 single: F rows {ey:.3e}, F* columns {es:.3e}")
    assert ey <= TOL and es <= TOL


def test_paper_time_ragged(paper_time):
    w, op = paper_time
    rows = np.sort(np.random.default_rng(12).choice(w.Nd, 4, replace=False))
    n = synth.ragged_lengths(w, 32)
    m = synth.param_series(w, 32, seed_offset=21)
    y = op.apply_F(torch.from_numpy(m).to(DEV, torch.float32), nt_active=n).double().cpu().numpy()
    Fr = rows_of_blocks(w, rows)
    for b in range(0, 32, 7):
        assert np.all(y[b, n[b]:] == 0.0)
        yo = oracle.apply_F(Fr, m[b:b + 1], n[b:b + 1])[0]
        assert oracle.rel_l2(y[b][:, rows], yo) <= TOL


def column_error_estimate(w, h_col, j, k_other, rng):
    """Relative L2 error of one data-space column h = F F* e_j over all Nd x Nt
    outputs, estimated without the whole operator: the spike's own sensor row
    s exactly, plus (Nd - 1) / k times the squared error and squared norm of
    k other sensor rows drawn at random.  F* e_j needs row s of the blocks
    only, so each sampled row r of h costs rows r and s of every block."""
    t0, sidx = divmod(int(j), w.Nd)
    others = np.sort(rng.choice(np.setdiff1d(np.arange(w.Nd), [sidx]), k_other, replace=False))
    rs = np.concatenate([[sidx], others])
    Frs = rows_of_blocks(w, rs)
    e = np.zeros((w.Nt, len(rs)))
    e[t0, 0] = 1.0
    href = oracle.apply_F(Frs, oracle.apply_Ft(Frs, e))          # [Nt, 1 + k]
    err2 = ((h_col[:, rs] - href) ** 2).sum(axis=0)
    ref2 = (href ** 2).sum(axis=0)
    scale = (w.Nd - 1) / k_other
    est = np.sqrt((err2[0] + scale * err2[1:].sum()) / (ref2[0] + scale * ref2[1:].sum()))
    spike_only = np.sqrt(err2[0] / ref2[0])
    return float(est), float(spike_only)


@pytest.fixture(scope="module")
def paper_time_fp16():
    w = synth.CONFIGS["paper_time"]
    op = load_op(w, "fp16", 64)
    yield w, op
    close_op(op)


def test_paper_time_fp16_single_rhs(paper_time_fp16):
    w, op = paper_time_fp16
    ey, es = single_rhs_errors(w, op)
    note(f"  fp16 single: F rows {ey:.3e}, F* columns {es:.3e}")
    assert ey <= TOL and es <= TOL


def test_paper_time_hessian_columns(paper_time_fp16):
    """64 data-space columns in one call (FP16 spectrum, matrix cores); the
    columns with spikes at t = 0 and t = Nt - 1 and two others, each by the
    whole-output estimate of column_error_estimate."""
    w, op = paper_time_fp16
    idx = synth.hessian_column_indices(w, 64)
    E = torch.from_numpy(synth.unit_data_vectors(w, idx)).to(DEV, torch.float32)
    h = op.apply_FFt(E).double().cpu().numpy()
    rng = np.random.default_rng(12)
    for c in (0, 1, 17, 63):
        est, spike = column_error_estimate(w, h[c], idx[c], 12, rng)
        note(f"  F F* column {c} (t0 = {int(idx[c]) // w.Nd}): whole-output estimate {est:.3e} "
             f"(spike row alone {spike:.3e})")
        assert est <= TOL


def test_paper_time_fp32():
    """FP32 spectrum (33 GB) at the same shape: F and F* within 1e-5."""
    w = synth.CONFIGS["paper_time"]
    op = load_op(w, "fp32", 1)
    try:
        ey, es = single_rhs_errors(w, op, seed=21)
        note(f"  fp32 single: F rows {ey:.3e}, F* columns {es:.3e}")
        assert ey <= 1e-5 and es <= 1e-5
    finally:
        close_op(op)


def test_paper_time_fp64():
    """FP64 spectrum (66 GB) at the same shape: F and F* within 1e-12."""
    w = synth.CONFIGS["paper_time"]
    op = load_op(w, "fp64", 1)
    try:
        ey, es = single_rhs_errors(w, op, nrows=4, ncols=32, seed=22)
        note(f"  fp64 single: F rows {ey:.3e}, F* columns {es:.3e}")
        assert ey <= 1e-12 and es <= 1e-12
    finally:
        close_op(op)


@pytest.fixture(scope="module")
def largest():
    w = synth.CONFIGS["largest"]
    note(f"[fullsize] loading {w.name} (66 GB BF16 spectrum)")
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "bf16", max_rhs=16, device=DEV)
    op.load(lambda c0, n: gpu_blocks(w, c0, n))
    yield w, op
    op.close()
    del op
    torch.cuda.empty_cache()


def test_largest_single_and_16_rhs(largest):
    w, op = largest
    rng = np.random.default_rng(13)
    rows = np.sort(rng.choice(w.Nd, 4, replace=False))
    cols = np.sort(rng.choice(w.Nm, 32, replace=False))
    m = synth.param_series(w, 16, backend="torch", smooth=True).numpy()
    y = op.apply_F(torch.from_numpy(m).to(DEV, torch.float32)).double().cpu().numpy()      # 16 RHS, matrix cores
    y1 = op.apply_F(torch.from_numpy(m[0]).to(DEV, torch.float32)).double().cpu().numpy()  # single RHS
    Fr = rows_of_blocks(w, rows)
    yo = oracle.apply_F(Fr, m[[0, 9]])
    e16 = max(oracle.rel_l2(y[b][:, rows], yo[i]) for i, b in enumerate((0, 9)))
    e1 = oracle.rel_l2(y1[:, rows], yo[0])
    d = synth.data_series(w, 16)
    s = op.apply_Ft(torch.from_numpy(d).to(DEV, torch.float32)).double().cpu().numpy()
    so = oracle.apply_Ft(cols_of_blocks(w, cols), d[[3, 15]])
    es = max(oracle.rel_l2(s[b][:, cols], so[i]) for i, b in enumerate((3, 15)))
    note(f"  largest: F rows 16-RHS {e16:.3e}, single {e1:.3e}; F* columns {es:.3e}")
    assert e16 <= TOL and e1 <= TOL and es <= TOL


def test_largest_misfit_gradient_autograd(largest):
    """d = F m_true + 0.01 eps; gradient via autograd at m = 0 and m_true:
    central differences of the quadratic misfit, fused kernel == autograd,
    and the adjoint identity."""
    w, op = largest
    m_true = synth.param_series(w, 1, backend="torch", device=DEV, smooth=True)[0].float()
    with torch.no_grad():
        d_obs = op.apply_F(m_true) + torch.from_numpy(synth.noise(w, 1)[0]).to(DEV, torch.float32)
    sig2 = w.sigma ** 2
    for m0 in (torch.zeros_like(m_true), m_true):
        m = m0.clone().requires_grad_(True)
        phi = misfit(m, op, d_obs, sig2)
        phi.backward()
        g = m.grad.double()
        m2 = m0.clone().requires_grad_(True)
        loss = 0.5 * ((P2O.apply(m2, op).double() - d_obs.double()) ** 2).sum() / sig2
        loss.backward()
        assert oracle.rel_l2(g.cpu().numpy(), m2.grad.double().cpu().numpy()) <= 1e-5
        assert abs(float(phi.detach()) - float(loss.detach())) <= 1e-5 * float(loss.detach())
        v = synth.param_series(w, 1, seed_offset=31, backend="torch", device=DEV)[0].float()
        # exact for a quadratic at any step: take a large one so FP32 rounding
        # of the misfit evaluations stays far below the difference
        eps = float(m_true.norm()) / float(v.norm())
        with torch.no_grad():
            fp = float(misfit(m0 + eps * v, op, d_obs, sig2))
            fm = float(misfit(m0 - eps * v, op, d_obs, sig2))
        fd = (fp - fm) / (2 * eps)
        gv = float((g * v.double()).sum())
        note(f"  misfit {float(phi.detach()):.6e}: directional derivative {gv:.6e}, central difference {fd:.6e}")
        assert abs(fd - gv) <= 1e-3 * abs(gv)
    # At m_true the residual F m_true - d_obs is minus the noise, so the
    # gradient is -F* noise / sigma^2: against the oracle on sampled columns.
    cols = np.sort(np.random.default_rng(14).choice(w.Nm, 32, replace=False))
    m = m_true.clone().requires_grad_(True)
    misfit(m, op, d_obs, sig2).backward()
    g_true = m.grad.double().cpu().numpy()
    noise = synth.noise(w, 1)[0]
    g_ref = -oracle.apply_Ft(cols_of_blocks(w, cols), noise) / sig2
    eg = oracle.rel_l2(g_true[:, cols], g_ref)
    note(f"  gradient at m_true vs oracle on 32 columns: {eg:.3e}")
    assert eg <= TOL
    # at m_true the residual is the noise: misfit ~ chi-square / 2 with Nd*Nt dof
    with torch.no_grad():
        phi_true = float(misfit(m_true, op, d_obs, sig2))
    dof = w.Nd * w.Nt
    assert abs(phi_true - 0.5 * dof) <= 5 * np.sqrt(0.5 * dof)
    # adjoint identity <F m, d> = <m, F* d> up to the BF16 spectrum rounding
    with torch.no_grad():
        lhs = float((op.apply_F(m_true).double() * d_obs.double()).sum())
        rhs = float((m_true.double() * op.apply_Ft(d_obs).double()).sum())
    assert abs(lhs - rhs) <= 2e-3 * abs(lhs)


def test_data_space_matrix_at_paper_grid():
    """Columns of K = sigma^2 I + F F^* at section 5's dimensions (49 sensors,
    513^2 parameters, 500 steps, FP16 spectrum): the batched F F^* call with
    64 right-hand sides over 263,169 parameter series (the compiled L = 1000
    transforms with 16-series tiles, lane offsets above 2^31 bytes), checked
    against the oracle on sampled entries: blocks (i, j) with time indices
    below 40 and three sensors, each entry the exact lag sum of sensor rows of
    the blocks.  An entry's error is measured against sqrt(K_pp K_qq), the
    bound of |K_pq| for a symmetric positive definite K (entries far below it,
    such as K between sensors one step apart, carry the spectrum's absolute
    rounding error of the whole column)."""
    w = synth.CONFIGS["paper_grid"]
    sigma = 1e-2
    op = load_op(w, "fp16", 64)
    try:
        N = op.data_dim()
        K = torch.zeros((N, N), dtype=torch.float64, device=DEV)
        var = torch.tensor([sigma ** 2], dtype=torch.float64, device=DEV)
        op.assemble_K(var, 1.0, K=K, columns=(0, 40 * w.Nd))
        torch.cuda.synchronize()
        rng = np.random.default_rng(8)
        sens = np.sort(rng.choice(w.Nd, 3, replace=False))
        Fr = synth.operator_rows_cols(w, range(40), rows=sens, backend="torch").numpy()      # [40, 3, Nm]
        Kh = K[:40 * w.Nd].cpu().numpy()
        def kref(i, j, a, c):
            v = sum(Fr[i - k, a] @ Fr[j - k, c] for k in range(min(i, j) + 1))
            return v + (sigma ** 2 if i == j and a == c else 0.0)

        errs, rel = [], []
        for i, j in ((0, 0), (1, 0), (5, 3), (17, 17), (39, 20), (25, 38), (39, 39)):
            for a in range(3):
                for c in range(3):
                    ref = kref(i, j, a, c)
                    got = Kh[j * w.Nd + sens[c], i * w.Nd + sens[a]]        # tensor row = column of K
                    errs.append(abs(got - ref) / np.sqrt(kref(i, i, a, a) * kref(j, j, c, c)))
                    rel.append(abs(got - ref) / abs(ref))
        note(f"[fullsize] paper grid K entries: max error vs sqrt(K_pp K_qq) {max(errs):.3e} "
             f"(entrywise relative: median {np.median(rel):.1e}, max {max(rel):.1e})")
        assert max(errs) <= TOL
        # columns past the assembled range are untouched
        assert not torch.any(K[40 * w.Nd:]).item()
    finally:
        close_op(op)
