"""GPU parity of the batched (many right-hand sides) path on the matrix
cores against the FP64 oracle, and against the per-right-hand-side streaming
path on the same plan.  BF16 spectrum (FP16 where stated); right-hand sides
enter the MFMA as a hi + lo pair, so the batched and streaming results differ
only by that split (relative 2^-16) and by summation order."""
import sys

import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2OOperator  # noqa: E402

DEV = "cuda"
TOL_BF16 = 2e-3        # BF16 or FP16 spectrum, FP32 accumulation


def note(msg):
    print(msg, flush=True)


def build(w, max_rhs, precision="bf16"):
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=max_rhs, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    return op, F


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, torch.float32)


def host(x):
    torch.cuda.synchronize()
    return x.double().cpu().numpy()


SHAPES = [
    synth.Workload("odd", Nd=70, Nm=1003, Nt=21, tau=6.0),        # 70 rows, pitch 1008 (partial column tiles)
    synth.Workload("blocks", Nd=37, Nm=9000, Nt=13, tau=5.0),     # three scale blocks / K chunks, ragged last
]
# tile variants also on an operator with two 320-row forward tiles (the last ragged)
TILE_SHAPES = SHAPES + [synth.Workload("tall", Nd=350, Nm=1003, Nt=21, tau=6.0)]


@pytest.mark.parametrize("nrhs", [2, 9, 17, 40, 70])
@pytest.mark.parametrize("w", SHAPES, ids=lambda w: w.name)
def test_batched_forward_adjoint(w, nrhs):
    note(f"[batched] {w.name} nrhs={nrhs}")
    op, F = build(w, nrhs)
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    y = host(op.apply_F(dev(m)))
    s = host(op.apply_Ft(dev(d)))
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    worst = max(max(oracle.rel_l2(y[b], yo[b]), oracle.rel_l2(s[b], so[b])) for b in range(nrhs))
    note(f"  worst rel-L2 vs oracle {worst:.3e}")
    assert worst <= TOL_BF16
    op.set_batched("gemv")
    y2 = host(op.apply_F(dev(m)))
    s2 = host(op.apply_Ft(dev(d)))
    assert oracle.rel_l2(y, y2) <= 5e-5 and oracle.rel_l2(s, s2) <= 5e-5


def test_batched_medium_64_and_ragged():
    w = synth.CONFIGS["medium"]
    note("[batched] medium 64 rhs + ragged")
    op, F = build(w, 64)
    m = synth.param_series(w, 64)
    n = synth.ragged_lengths(w, 64, lo=1)
    y = host(op.apply_F(dev(m), nt_active=n))
    yo = oracle.apply_F(F, m, n)
    for b in range(64):
        assert np.all(y[b, n[b]:] == 0.0)
        assert oracle.rel_l2(y[b], yo[b]) <= TOL_BF16
    d = synth.data_series(w, 64)
    s = host(op.apply_Ft(dev(d), nt_active=n))
    so = oracle.apply_Ft(F, d, n)
    for b in range(64):
        assert np.all(s[b, n[b]:] == 0.0)
        assert oracle.rel_l2(s[b], so[b]) <= TOL_BF16


def test_batched_data_space_columns():
    """64 columns F F* e_j in one call on an FP16 spectrum (the precision that
    meets 2e-3 on every column; a BF16 spectrum does not on early spikes),
    each column against the oracle, plain and with ragged lengths."""
    w = synth.CONFIGS["medium"]
    idx = synth.hessian_column_indices(w, 64)
    e = synth.unit_data_vectors(w, idx)
    op, F = build(w, 64, "fp16")
    n = synth.ragged_lengths(w, 64, lo=1)
    for nt in (None, n):
        h = host(op.apply_FFt(dev(e), nt_active=nt))
        ho = oracle.data_space_hessian(F, e, nt)
        errs = [oracle.rel_l2(h[b], ho[b]) for b in range(64) if np.any(ho[b])]
        note(f"[batched] fp16 F F* columns{' ragged' if nt is not None else ''}: worst rel-L2 {max(errs):.3e} "
             f"(t = 0 column {errs[0]:.3e})")
        assert max(errs) <= TOL_BF16
        if nt is not None:
            for b in range(64):
                assert np.all(h[b, nt[b]:] == 0.0)


def test_batched_misfit_gradient():
    w = synth.CONFIGS["medium"]
    op, F = build(w, 16)
    m = synth.param_series(w, 16)
    d_obs = oracle.apply_F(F, synth.param_series(w, 16, seed_offset=5)) + synth.noise(w, 16)
    phi, g = op.misfit_grad(dev(m), dev(d_obs), torch.tensor([w.sigma ** 2], dtype=torch.float64, device=DEV))
    phi_o, g_o = oracle.misfit_and_grad(F, m, d_obs, w.sigma ** 2)
    phi, g = host(phi), host(g)
    for b in range(16):
        assert abs(phi[b] - phi_o[b]) <= TOL_BF16 * phi_o[b]
        assert oracle.rel_l2(g[b], g_o[b]) <= TOL_BF16


@pytest.mark.parametrize("w", TILE_SHAPES, ids=lambda w: w.name)
def test_every_tile_variant(w):
    """Each matrix-core tile variant the autotuner can pick, forced, against
    the oracle (a full 64-wide group and a ragged one)."""
    from paper_2501_14911_amd import gemm_tiles
    nrhs = 70
    op, F = build(w, nrhs)
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    for t in range(len(gemm_tiles())):
        op.set_gemm_tile(t)
        y = host(op.apply_F(dev(m)))
        s = host(op.apply_Ft(dev(d)))
        worst = max(max(oracle.rel_l2(y[b], yo[b]), oracle.rel_l2(s[b], so[b])) for b in range(nrhs))
        note(f"[batched] {w.name} tile {t}: worst rel-L2 {worst:.3e}")
        assert worst <= TOL_BF16


@pytest.mark.parametrize("w", TILE_SHAPES, ids=lambda w: w.name)
def test_fp16_spectrum_on_matrix_cores(w):
    """FP16-stored spectrum on the matrix cores (FP16 x FP16 products of the
    spectrum and the scaled right-hand sides, LDS-ring tiles): every ring
    variant and the built-in choice against the oracle, at a full and a
    ragged right-hand-side group, within the FP16 bound; and against the same
    plan's streaming FP16 path, which keeps the right-hand sides in FP32: the
    two differ by the right-hand sides' rounding to FP16 (unit roundoff
    2^-11 per entry, about 1.6e-4 on these outputs)."""
    nrhs = 70
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp16", max_rhs=nrhs, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    from paper_2501_14911_amd import gemm_tiles
    rings = [t for t, shape in enumerate(gemm_tiles()) if t >= 7]
    for t in [-1] + rings:
        op.set_gemm_tile(t)
        y = host(op.apply_F(dev(m)))
        s = host(op.apply_Ft(dev(d)))
        worst = max(max(oracle.rel_l2(y[b], yo[b]), oracle.rel_l2(s[b], so[b])) for b in range(nrhs))
        note(f"[batched] fp16 {w.name} tile {t}: worst rel-L2 {worst:.3e}")
        assert worst <= TOL_BF16
    op.set_gemm_tile(-1)
    op.set_batched("gemv")
    y1, s1 = host(op.apply_F(dev(m[:3]))), host(op.apply_Ft(dev(d[:3])))
    op.set_batched("auto")
    y2, s2 = host(op.apply_F(dev(m[:3]))), host(op.apply_Ft(dev(d[:3])))
    for b in range(3):
        assert oracle.rel_l2(y2[b], y1[b]) <= 2.0 ** -11 and oracle.rel_l2(s2[b], s1[b]) <= 2.0 ** -11


def test_fp16_right_hand_side_scales():
    """Right-hand sides of very different magnitudes in one FP16 matrix-core
    call (1e-30 .. 1e30, which FP16 alone cannot hold, and an all-zero one):
    each is scaled on its own, so each meets the bound, the zero one gives
    exact zeros; likewise for data-space columns whose intermediate series
    span that range."""
    w = SHAPES[1]
    nrhs = 9
    op, F = build(w, nrhs, "fp16")
    mags = np.array([1e-30, 1e-10, 1.0, 1e10, 1e30, 3.0e-5, 7.0e4, 0.0, 1.0])
    m = synth.param_series(w, nrhs) * mags[:, None, None]
    d = synth.data_series(w, nrhs) * mags[:, None, None]
    y = host(op.apply_F(dev(m)))
    s = host(op.apply_Ft(dev(d)))
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    for b in range(nrhs):
        if mags[b] == 0.0:
            assert np.all(y[b] == 0.0) and np.all(s[b] == 0.0)
            continue
        ey, es = oracle.rel_l2(y[b], yo[b]), oracle.rel_l2(s[b], so[b])
        note(f"[batched] fp16 scale {mags[b]:.0e}: F {ey:.2e}  F* {es:.2e}")
        assert ey <= TOL_BF16 and es <= TOL_BF16
    idx = synth.hessian_column_indices(w, nrhs)
    e = synth.unit_data_vectors(w, idx) * mags[:, None, None]
    h = host(op.apply_FFt(dev(e)))
    ho = oracle.data_space_hessian(F, e)
    for b in range(nrhs):
        if mags[b] == 0.0:
            assert np.all(h[b] == 0.0)
            continue
        assert oracle.rel_l2(h[b], ho[b]) <= TOL_BF16, (b, mags[b])


def test_autotune_then_apply():
    w = SHAPES[0]
    nrhs = 40
    op, F = build(w, nrhs)
    res = op.autotune(nrhs, reps=2)
    note(f"[batched] autotune {res}")
    from paper_2501_14911_amd import gemm_tiles
    for key in ("fwd", "adj"):
        assert 0 <= res[key][0] < len(gemm_tiles()) and res[key][1] > 0
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    y = host(op.apply_F(dev(m)))
    s = host(op.apply_Ft(dev(d)))
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    assert max(oracle.rel_l2(y[b], yo[b]) for b in range(nrhs)) <= TOL_BF16
    assert max(oracle.rel_l2(s[b], so[b]) for b in range(nrhs)) <= TOL_BF16
    with pytest.raises(Exception):
        op.autotune(nrhs + 1)                    # beyond max_rhs


def test_fp16_autotune_then_apply():
    """The autotuner on an FP16 plan (its operands and right-hand-side scales
    are filled before the timed launches), then calls with the chosen tiles."""
    w = SHAPES[1]
    nrhs = 40
    op, F = build(w, nrhs, "fp16")
    res = op.autotune(nrhs, reps=2)
    note(f"[batched] fp16 autotune {res}")
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    y = host(op.apply_F(dev(m)))
    s = host(op.apply_Ft(dev(d)))
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    assert max(oracle.rel_l2(y[b], yo[b]) for b in range(nrhs)) <= TOL_BF16
    assert max(oracle.rel_l2(s[b], so[b]) for b in range(nrhs)) <= TOL_BF16


def test_mfma_option_needs_a_16_bit_spectrum():
    w = synth.CONFIGS["tiny"]
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp32", max_rhs=2, device=DEV)
    from paper_2501_14911_amd import P2OError
    with pytest.raises(P2OError):
        op.set_batched("mfma")


@pytest.mark.parametrize("w", [synth.Workload("tall16", Nd=330, Nm=1003, Nt=16, tau=4.0),
                               synth.Workload("tall128", Nd=300, Nm=1003, Nt=128, tau=32.0),
                               synth.Workload("few49", Nd=49, Nm=1003, Nt=128, tau=32.0),
                               synth.Workload("few100", Nd=100, Nm=2100, Nt=16, tau=4.0)],
                         ids=lambda w: w.name)
def test_fp16_operand_data_space_columns(w):
    """F F* e_j on an FP16 spectrum with FP16 intermediate operands (forward
    products in the whole-line ring's 320-, 64- and 128-row tiles; compiled
    transform lengths L = 32 and 256; 64 columns, full and ragged): every
    column against the oracle at 2e-3, and against the same
    plan with complex FP32 intermediates, which differ only by the FP16
    rounding of the adjoint products (2^-12 per value) and the scale of the
    right-hand sides' rounding."""
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp16", max_rhs=64, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    e = synth.unit_data_vectors(w, synth.hessian_column_indices(w, 64))
    nt = synth.ragged_lengths(w, 64, lo=w.Nt // 4)
    ref = oracle.data_space_hessian(F, e)
    ref_r = oracle.data_space_hessian(F, e, nt)
    got, got_r = {}, {}
    for on in (True, False):
        op.set_fp16_operands(on)
        got[on] = host(op.apply_FFt(dev(e)))
        got_r[on] = host(op.apply_FFt(dev(e), nt_active=nt))
    for on in (True, False):
        errs = [oracle.rel_l2(got[on][b], ref[b]) for b in range(64)]
        errs_r = [oracle.rel_l2(got_r[on][b], ref_r[b]) for b in range(64) if np.any(ref_r[b])]
        note(f"[batched] {w.name} FFt fp16 operands={on}: worst column {max(errs):.3e}, ragged {max(errs_r):.3e}")
        assert max(errs) <= TOL_BF16 and max(errs_r) <= TOL_BF16
        for b in range(64):
            assert np.all(got_r[on][b, nt[b]:] == 0.0)
    agree = oracle.rel_l2(got[True], got[False])
    note(f"[batched] {w.name} FP16 vs FP32 intermediates: {agree:.3e}")
    assert agree <= 2.0 ** -10

def test_fp16_operand_scales_span_magnitudes():
    """FP16 intermediate operands with right-hand sides from 1e-20 to 1e20 and
    an all-zero one in one call: the a-priori power-of-two scales follow each
    right-hand side, so every column matches the complex FP32 intermediates
    to the FP16 rounding (relative per column), and the zero one stays zero."""
    w = synth.Workload("tall16", Nd=330, Nm=1003, Nt=16, tau=4.0)
    F = synth.operator_blocks(w)
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp16", max_rhs=64, device=DEV)
    Ft = torch.from_numpy(F).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
    d = synth.data_series(w, 41)
    mags = 10.0 ** np.arange(-20, 21)
    x = d * mags[:, None, None]
    x[20] = 0.0
    got = {}
    for on in (True, False):
        op.set_fp16_operands(on)
        got[on] = host(op.apply_FFt(torch.from_numpy(x).to(DEV, torch.float32)))
    assert np.all(got[True][20] == 0.0) and np.all(got[False][20] == 0.0)
    worst = max(oracle.rel_l2(got[True][b], got[False][b]) for b in range(41) if b != 20)
    note(f"[batched] FP16 operands over 1e-20 .. 1e20: worst column vs FP32 intermediates {worst:.3e}")
    assert worst <= 2.0 ** -10
    assert np.all(np.isfinite(got[True]))
