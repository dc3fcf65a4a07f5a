"""GPU parity: the HIP path through the C ABI against the FP64 oracle,
element by element on the same seeded inputs (drawn with numpy on the host,
copied to the device), at sizes that span several tiles and ragged tails.

Tolerances are relative L2 over each whole output, against the oracle run on
the unquantised float64 blocks: 1e-12 (FP64 spectrum and arithmetic),
1e-5 (FP32), 2e-3 (BF16 or FP16 spectrum, FP32 accumulation).
"""
import math
import sys

import numpy as np
import pytest

from conftest import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ensure_built()

import oracle  # noqa: E402
import synth  # noqa: E402
from paper_2501_14911_amd import P2O, P2OT, P2OOperator, misfit  # noqa: E402

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 2e-3, "fp16": 2e-3}
DEV = "cuda"


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def build_op(w, precision, max_rhs=1, F=None, chunk=synth.SCALE_BLOCK):
    F = synth.operator_blocks(w) if F is None else F
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=max_rhs, device=DEV)
    Ft = torch.from_numpy(np.ascontiguousarray(F)).to(DEV)
    op.load(lambda c0, n: Ft[:, :, c0:c0 + n], chunk_cols=chunk)
    return op, F


def to_dev(x, op):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, op.dtype)


def host(x):
    torch.cuda.synchronize()
    return x.double().cpu().numpy()


SMALL = [
    synth.Workload("tiny", Nd=4, Nm=64, Nt=16, tau=4.0),
    synth.Workload("odd", Nd=70, Nm=1003, Nt=21, tau=6.0),          # 70 rows (two row slabs), ragged columns, L=42
    synth.Workload("prime_nt", Nd=3, Nm=9000, Nt=13, tau=5.0),      # three scale blocks, last ragged; L=28
    synth.Workload("one_step", Nd=5, Nm=8, Nt=1, tau=1.0),          # N_t = 1: a plain GEMV
    synth.Workload("one_sensor", Nd=1, Nm=520, Nt=37, tau=9.0),     # L=80
]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp16"])
@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
def test_forward_and_adjoint_small(w, precision):
    """16 right-hand sides, on the batched path (matrix cores for BF16 / FP16)
    and on the streaming one.  Several of these shapes give an output only a
    handful of terms (5 sensors x 8 parameters at N_t = 1), where a single
    output's relative error is not concentrated near its mean; the error is
    therefore taken over all 16 right-hand sides together (hundreds of
    outputs), at the same tolerance as everywhere else."""
    note(f"[parity] {w.name} {precision}")
    nrhs = 16
    op, F = build_op(w, precision, max_rhs=nrhs)
    m = synth.param_series(w, nrhs)
    d = synth.data_series(w, nrhs)
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    for mode in ("auto", "gemv"):
        op.set_batched(mode)
        y = host(op.apply_F(to_dev(m, op)))
        s = host(op.apply_Ft(to_dev(d, op)))
        ey, es = oracle.rel_l2(y, yo), oracle.rel_l2(s, so)
        note(f"  {mode}: rel-L2 F {ey:.3e}  F* {es:.3e}")
        assert ey <= TOL[precision] and es <= TOL[precision], (mode, ey, es)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp16"])
def test_medium_workload(precision):
    w = synth.CONFIGS["medium"]
    note(f"[parity] medium {precision}")
    op, F = build_op(w, precision, max_rhs=3)
    m = synth.param_series(w, 3)
    d = synth.data_series(w, 3)
    y = host(op.apply_F(to_dev(m, op)))
    s = host(op.apply_Ft(to_dev(d, op)))
    yo, so = oracle.apply_F(F, m), oracle.apply_Ft(F, d)
    for b in range(3):
        ey, es = oracle.rel_l2(y[b], yo[b]), oracle.rel_l2(s[b], so[b])
        note(f"  rhs {b}: rel-L2 F {ey:.3e}  F* {es:.3e}")
        assert ey <= TOL[precision] and es <= TOL[precision]


def test_ragged_right_hand_sides():
    w = synth.CONFIGS["medium"]
    note("[parity] ragged medium fp64")
    n = np.array([128, 1, 64, 0, 100, 127], dtype=np.int32)
    op, F = build_op(w, "fp64", max_rhs=len(n))
    m = synth.param_series(w, len(n))
    d = synth.data_series(w, len(n))
    y = host(op.apply_F(to_dev(m, op), nt_active=n))
    s = host(op.apply_Ft(to_dev(d, op), nt_active=n))
    yo, so = oracle.apply_F(F, m, n), oracle.apply_Ft(F, d, n)
    for b, nb in enumerate(n):
        assert np.all(y[b, nb:] == 0.0) and np.all(s[b, nb:] == 0.0)
        if nb:
            assert oracle.rel_l2(y[b], yo[b]) <= 1e-12
            assert oracle.rel_l2(s[b], so[b]) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_data_space_operator_columns(precision):
    """Columns F F* e_j, each checked on its own (the first has its spike at
    t = 0, the second at t = Nt - 1).  A BF16 spectrum does not meet 2e-3 on
    early-spike columns (test_bf16_data_space_columns_at_L840); FP16 does."""
    w = synth.CONFIGS["medium"]
    note(f"[parity] F F* columns medium {precision}")
    idx = synth.hessian_column_indices(w, 4)
    e = synth.unit_data_vectors(w, idx)
    n = np.array([128, 128, 77, 128], dtype=np.int32)
    op, F = build_op(w, precision, max_rhs=4)
    for nt in (None, n):
        h = host(op.apply_FFt(to_dev(e, op), nt_active=nt))
        ho = oracle.data_space_hessian(F, e, nt)
        errs = [oracle.rel_l2(h[b], ho[b]) for b in range(len(idx))]
        note("  per column " + " ".join(f"{x:.2e}" for x in errs))
        assert max(errs) <= TOL[precision], errs
    # one column alone takes the streaming path
    h1 = host(op.apply_FFt(to_dev(e[:1], op)))
    assert oracle.rel_l2(h1[0], oracle.data_space_hessian(F, e[:1])[0]) <= TOL[precision]


# L = 840 (the paper's time shape): the length the library has compiled FFT
# kernels for; 203 columns and 5 sensors leave ragged tiles on both sides.
PAPER_T = synth.Workload("paper_t_small", Nd=5, Nm=203, Nt=420, tau=100.0)
# at least 2048 parameter series: FP32 transforms of L = 840 take 16-series
# tiles on 512-thread workgroups (the last tile ragged)
PAPER_T_WIDE = synth.Workload("paper_t_wide", Nd=3, Nm=2100, Nt=420, tau=100.0)
# section 5's number of time steps: L = 1000
PAPER_T500 = synth.Workload("paper_t500_small", Nd=5, Nm=203, Nt=500, tau=100.0)
# at least 2048 parameter series: FP32 transforms of L = 1000 take 16-series tiles (the last one ragged)
PAPER_T500_WIDE = synth.Workload("paper_t500_wide", Nd=3, Nm=2100, Nt=500, tau=100.0)


def _l840_runs(precision, w=PAPER_T):
    """F, F*, ragged F and F*, F F* (truncate-and-repad) with its spikes at
    t = 0, Nt - 1 and two more, ragged F F* and the misfit epilogue at
    L = 2 Nt (840 by default), on both FFT paths (kernels compiled for that
    length and the runtime-length ones), with the oracle's results."""
    n = np.array([w.Nt, 301, 64, 0], dtype=np.int32)
    nh = np.array([300, w.Nt, 400, 351], dtype=np.int32)
    op, F = build_op(w, precision, max_rhs=4)
    m = synth.param_series(w, 4)
    d = synth.data_series(w, 4)
    e = synth.unit_data_vectors(w, synth.hessian_column_indices(w, 4))
    d_obs = oracle.apply_F(F, synth.param_series(w, 2, seed_offset=11)) + synth.noise(w, 2)
    var = np.array([w.sigma ** 2])
    ref = {"F": oracle.apply_F(F, m), "Ft": oracle.apply_Ft(F, d),
           "F_ragged": oracle.apply_F(F, m, n), "Ft_ragged": oracle.apply_Ft(F, d, n),
           "FFt": oracle.data_space_hessian(F, e), "FFt_ragged": oracle.data_space_hessian(F, e, nh)}
    ref["phi"], ref["grad"] = oracle.misfit_and_grad(F, m[:2], d_obs, var)
    got = {}
    for fixed in (True, False):
        op.set_fixed_fft(fixed)
        r = {"F": host(op.apply_F(to_dev(m, op))), "Ft": host(op.apply_Ft(to_dev(d, op))),
             "F_ragged": host(op.apply_F(to_dev(m, op), nt_active=n)),
             "Ft_ragged": host(op.apply_Ft(to_dev(d, op), nt_active=n)),
             "FFt": host(op.apply_FFt(to_dev(e, op))), "FFt_ragged": host(op.apply_FFt(to_dev(e, op), nt_active=nh))}
        phi, g = op.misfit_grad(to_dev(m[:2], op), to_dev(d_obs, op), torch.from_numpy(var).to(DEV))
        r["phi"], r["grad"] = host(phi), host(g)
        got[fixed] = r
    for fixed, r in got.items():
        for key in ("F", "Ft", "F_ragged", "Ft_ragged", "FFt", "FFt_ragged", "grad"):
            want = ref[key]
            per_rhs = " ".join(f"{oracle.rel_l2(r[key][b], want[b]):.2e}" if np.any(want[b]) else "-"
                               for b in range(len(want)))
            note(f"  fixed={fixed} {key}: per rhs {per_rhs}")
    lens = {"F_ragged": n, "Ft_ragged": n, "FFt_ragged": nh}
    return ref, got, lens


def _per_rhs_errors(r, want):
    return [oracle.rel_l2(r[b], want[b]) for b in range(len(want)) if np.any(want[b])]


def _check_l840(precision, ref, got, lens, keys):
    for fixed, r in got.items():
        for key in keys:
            errs = _per_rhs_errors(r[key], ref[key])
            assert max(errs) <= TOL[precision], (key, fixed, errs)
        for key, nl in lens.items():
            for b, nb in enumerate(nl):
                assert np.all(r[key][b, nb:] == 0.0), (key, fixed, b)
        for b in range(2):
            assert abs(r["phi"][b] - ref["phi"][b]) <= TOL[precision] * ref["phi"][b]
            assert oracle.rel_l2(r["grad"][b], ref["grad"][b]) <= TOL[precision]


@pytest.mark.parametrize("precision,w", [("fp64", PAPER_T), ("fp32", PAPER_T), ("fp16", PAPER_T),
                                         ("fp32", PAPER_T_WIDE), ("fp16", PAPER_T_WIDE)],
                         ids=["fp64", "fp32", "fp16", "fp32-wide", "fp16-wide"])
def test_fixed_and_runtime_length_ffts(precision, w):
    """Both FFT paths against the oracle on every result at L = 840, each
    right-hand side (each F F* column) on its own; with an FP16 spectrum the
    batched calls take the matrix cores, and the two paths must then also
    agree with each other to FP32 rounding.  2100 parameter series take the
    wide tiles on the compiled path (the runtime-length path keeps 8)."""
    note(f"[parity] fixed vs runtime-length FFTs, {w.name} {precision}")
    ref, got, lens = _l840_runs(precision, w)
    _check_l840(precision, ref, got, lens, ("F", "Ft", "F_ragged", "Ft_ragged", "FFt", "FFt_ragged"))
    if precision == "fp16":
        # the two paths' FP32 rounding can move a right-hand side's value
        # across an FP16 rounding boundary (or its scale across a power of
        # two) in the matrix-core operands: agreement to the operand rounding
        for key in got[True]:
            assert oracle.rel_l2(got[True][key], got[False][key]) <= 2.0 ** -11, key


@pytest.mark.parametrize("precision,w", [("fp64", PAPER_T500), ("fp32", PAPER_T500), ("fp16", PAPER_T500),
                                         ("fp32", PAPER_T500_WIDE), ("fp16", PAPER_T500_WIDE)],
                         ids=["fp64", "fp32", "fp16", "fp32-wide", "fp16-wide"])
def test_fixed_and_runtime_length_ffts_at_L1000(precision, w):
    """The same checks at L = 1000 (N_t = 500, the time steps of section 5's
    problem; radices 4, 5, 5, 5), with 4-series tiles and, for 2100
    parameter series, 16-series tiles (compiled kernels only; the
    runtime-length path keeps 4)."""
    note(f"[parity] fixed vs runtime-length FFTs, {w.name} {precision}")
    ref, got, lens = _l840_runs(precision, w)
    _check_l840(precision, ref, got, lens, ("F", "Ft", "F_ragged", "Ft_ragged", "FFt", "FFt_ragged"))
    agree = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 2.0 ** -11}[precision]
    for key in got[True]:
        assert oracle.rel_l2(got[True][key], got[False][key]) <= agree, key


def test_bf16_spectrum_at_L840():
    """BF16 spectrum: F, F* (plain and ragged) and the misfit gradient meet
    2e-3 per right-hand side on both FFT paths, and every result, the F F*
    columns included, agrees between the two paths to FP32 rounding.  Its
    F F* columns' error against the oracle is test_bf16_data_space_columns."""
    note(f"[parity] fixed vs runtime-length FFTs, {PAPER_T.name} bf16")
    ref, got, lens = _l840_runs("bf16")
    _check_l840("bf16", ref, got, lens, ("F", "Ft", "F_ragged", "Ft_ragged"))
    for key in got[True]:
        agree = oracle.rel_l2(got[True][key], got[False][key])
        note(f"  fixed vs runtime-length {key}: {agree:.3e}")
        assert agree <= 1e-5, (key, agree)


@pytest.mark.xfail(strict=True, reason=(
    "A BF16 spectrum's rounding noise is spread evenly over all L lags of the operator, while the column "
    "F F* e_j of a spike at t = 0 is concentrated near lag 0: its relative error grows like the square root "
    "of the decay time (measured 6.3e-3 at tau = 100, L = 840).  Data-space columns meet 2e-3 with an FP16 "
    "spectrum (test_fixed_and_runtime_length_ffts[fp16])."))
def test_bf16_data_space_columns():
    note(f"[parity] F F* columns {PAPER_T.name} bf16 (known to exceed 2e-3)")
    ref, got, lens = _l840_runs("bf16")
    for fixed, r in got.items():
        for key in ("FFt", "FFt_ragged"):
            errs = _per_rhs_errors(r[key], ref[key])
            assert max(errs) <= TOL["bf16"], (key, fixed, errs)


@pytest.mark.parametrize("var_kind", ["scalar", "sensor", "full"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp16"])
def test_misfit_and_gradient(precision, var_kind):
    w = synth.CONFIGS["medium"]
    note(f"[parity] misfit medium {precision} {var_kind}")
    op, F = build_op(w, precision, max_rhs=2)
    m = synth.param_series(w, 2)
    d_obs = oracle.apply_F(F, synth.param_series(w, 2, seed_offset=11)) + synth.noise(w, 2)
    rng = np.random.default_rng(3)
    var = {"scalar": np.array([w.sigma ** 2]),
           "sensor": rng.uniform(0.5, 2.0, w.Nd) * w.sigma ** 2,
           "full": rng.uniform(0.5, 2.0, w.Nd * w.Nt) * w.sigma ** 2}[var_kind]
    phi, g = op.misfit_grad(to_dev(m, op), to_dev(d_obs, op), torch.from_numpy(var).to(DEV))
    phi_o, g_o = oracle.misfit_and_grad(F, m, d_obs, var)
    phi = host(phi)
    g = host(g)
    for b in range(2):
        note(f"  rhs {b}: misfit rel {abs(phi[b] - phi_o[b]) / phi_o[b]:.3e}  grad {oracle.rel_l2(g[b], g_o[b]):.3e}")
        assert abs(phi[b] - phi_o[b]) <= TOL[precision] * phi_o[b]
        assert oracle.rel_l2(g[b], g_o[b]) <= TOL[precision]


def test_spectrum_fp64_matches_dft_definition():
    w = synth.Workload("spec", Nd=6, Nm=300, Nt=21, tau=5.0)
    op, F = build_op(w, "fp64")
    raw = op.spectrum_view().cpu().numpy().view(np.float64).reshape(op.nfreq, w.Nd, op.pitch, 2)
    Fh = raw[..., 0] + 1j * raw[..., 1]
    ref = oracle.spectrum(F, op.L)
    assert np.max(abs(Fh[:, :, w.Nm:])) == 0.0          # zero padding
    err = np.linalg.norm(Fh[:, :, :w.Nm] - ref) / np.linalg.norm(ref)
    assert err <= 1e-14


def _half_codes_to_float(codes, precision):
    if precision == "bf16":
        return (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return codes.view(np.float16).astype(np.float64)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_quantised_spectrum_is_nearest_rounding(precision):
    """Every stored code is the nearest representable value (half an ulp) of
    the exact spectrum times its block's power-of-two scale; blocks use the
    documented exponent rule."""
    w = synth.Workload("spec", Nd=5, Nm=5000, Nt=19, tau=5.0)
    op, F = build_op(w, precision)
    raw = op.spectrum_view().cpu().numpy().view(np.uint16).reshape(op.nfreq, w.Nd, op.pitch, 2)
    sc = op.scales_view().cpu().numpy().astype(np.float64)            # dequantisation multipliers
    ref = oracle.spectrum(F, op.L)
    ulp_bits = 8 if precision == "bf16" else 11
    for part, comp in ((0, ref.real), (1, ref.imag)):
        q = _half_codes_to_float(raw[:, :, : w.Nm, part], precision)
        blk = np.arange(w.Nm) // synth.SCALE_BLOCK
        s = sc[:, blk][:, None, :]                                     # [nfreq, 1, Nm]
        exact = comp / s                                               # the value that was rounded
        mag = np.maximum(abs(exact), 2.0 ** (-14 if precision == "fp16" else -126))
        half_ulp = 2.0 ** (np.floor(np.log2(mag)) - ulp_bits)
        # the oracle's own DFT carries FP64 rounding noise (e.g. ~1e-17 where
        # the Nyquist bin's imaginary part is exactly zero)
        noise = 1e-13 * np.max(abs(ref), axis=(1, 2))[:, None, None] / s
        assert np.all(abs(q - exact) <= half_ulp * (1 + 1e-6) + noise)
    for k in range(op.nfreq):
        for b in range(op.nblk):
            cols = slice(b * synth.SCALE_BLOCK, min((b + 1) * synth.SCALE_BLOCK, w.Nm))
            amax = max(abs(ref[k, :, cols].real).max(), abs(ref[k, :, cols].imag).max())
            e = (15 if precision == "fp16" else 0) - math.ceil(math.log2(amax))
            assert sc[k, b] == 2.0 ** (-e)


def test_nonfinite_blocks_are_rejected():
    w = synth.Workload("nan", Nd=3, Nm=40, Nt=8, tau=3.0)
    F = synth.operator_blocks(w)
    F[5, 1, 7] = np.nan
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "bf16", device=DEV)
    op.load_blocks(torch.from_numpy(F).to(DEV), 0)
    from paper_2501_14911_amd import P2OError
    with pytest.raises(P2OError) as ei:
        op.finalize()
    assert ei.value.status == -5
    with pytest.raises(P2OError):
        op.apply_F(torch.zeros((w.Nt, w.Nm), device=DEV))


def test_bitwise_reproducible():
    w = synth.CONFIGS["medium"]
    op, F = build_op(w, "bf16", max_rhs=2)
    m = to_dev(synth.param_series(w, 2), op)
    d_obs = to_dev(synth.data_series(w, 2), op)
    a = op.apply_F(m).clone()
    b = op.apply_F(m).clone()
    pa, ga = op.misfit_grad(m, d_obs, torch.tensor([1e-4], dtype=torch.float64, device=DEV))
    pa, ga = pa.clone(), ga.clone()
    pb, gb = op.misfit_grad(m, d_obs, torch.tensor([1e-4], dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(pa, pb) and torch.equal(ga, gb)


# ---------------------------------------------------------------- autograd
def test_autograd_gradient_matches_finite_differences_and_transpose():
    w = synth.CONFIGS["medium"]
    note("[autograd] medium fp64")
    op, F = build_op(w, "fp64")
    sigma = w.sigma
    m0 = synth.param_series(w, 1)[0]
    d_obs = oracle.apply_F(F, synth.param_series(w, 1, seed_offset=7)[0]) + synth.noise(w, 1)[0]
    dobs_t = to_dev(d_obs, op)
    m = to_dev(m0, op).requires_grad_(True)
    loss = 0.5 * ((P2O.apply(m, op) - dobs_t) ** 2).sum() / sigma ** 2
    loss.backward()
    g = host(m.grad)
    _, g_o = oracle.misfit_and_grad(F, m0, d_obs, sigma ** 2)
    assert oracle.rel_l2(g, g_o) <= 1e-12
    # central differences are exact for a quadratic up to rounding
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.standard_normal(m0.shape)
        eps = 1e-3 * np.linalg.norm(m0) / np.linalg.norm(v)
        with torch.no_grad():
            fp = float(0.5 * ((P2O.apply(to_dev(m0 + eps * v, op), op) - dobs_t) ** 2).sum() / sigma ** 2)
            fm = float(0.5 * ((P2O.apply(to_dev(m0 - eps * v, op), op) - dobs_t) ** 2).sum() / sigma ** 2)
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - np.sum(g * v)) <= 1e-6 * abs(np.sum(g * v))
    # fused misfit kernel gives the same value and gradient
    m2 = to_dev(m0, op).requires_grad_(True)
    phi = misfit(m2, op, dobs_t, sigma ** 2)
    phi.backward()
    assert abs(float(phi.detach()) - float(loss.detach())) <= 1e-12 * float(loss.detach())
    assert oracle.rel_l2(host(m2.grad), g_o) <= 1e-12


def test_double_backward_gauss_newton_is_symmetric():
    w = synth.CONFIGS["tiny"]
    op, F = build_op(w, "fp64")
    rng = np.random.default_rng(6)
    v = to_dev(rng.standard_normal((w.Nt, w.Nm)), op)
    u = to_dev(rng.standard_normal((w.Nt, w.Nm)), op)

    def gn_direct(x):
        return P2OT.apply(P2O.apply(x, op), op)

    a = float((v * gn_direct(u)).sum())
    b = float((u * gn_direct(v)).sum())
    assert abs(a - b) <= 1e-12 * abs(a)
    fu = oracle.apply_Ft(F, oracle.apply_F(F, host(u)))
    assert oracle.rel_l2(host(gn_direct(u)), fu) <= 1e-12
    # the adjoint's backward is the forward again
    d = to_dev(rng.standard_normal((w.Nt, w.Nd)), op).requires_grad_(True)
    (P2OT.apply(d, op) * u).sum().backward()
    assert oracle.rel_l2(host(d.grad), oracle.apply_F(F, host(u))) <= 1e-12
