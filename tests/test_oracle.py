"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with an
independent route (time-stepping the LTI system, the assembled dense matrix,
numpy.convolve, a GEMV, closed forms, hand-worked fixtures, the convolution
theorem through numpy.fft, exactness of central differences on a quadratic).
A final group plants typical mistakes in copies of the oracle and checks that
some pin catches each one.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import toeplitz as T
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _rand_blocks(rng, Nt, Nd, Nm):
    return rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 3.0)[:, None, None]


def dense_matrix(F):
    """Assemble the (Nd*Nt) x (Nm*Nt) block matrix of equation LTI-matrix
    block by block: block (i, j) = F_{i-j} for i >= j, zero above."""
    Nt, Nd, Nm = F.shape
    Mx = np.zeros((Nd * Nt, Nm * Nt))
    for i in range(Nt):
        for j in range(i + 1):
            Mx[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = F[i - j]
    return Mx


def make_lti(rng, Nw, Nd, Nm):
    A = rng.standard_normal((Nw, Nw))
    A *= 0.9 / max(abs(np.linalg.eigvals(A)))        # stable
    return A, rng.standard_normal((Nd, Nw)), rng.standard_normal((Nw, Nm))


def run_lti(A, B, C, m):
    """Step w_{k+1} = A w_k + C m_k, d_{k+1} = B w_{k+1} from w_0 = 0
    (equation LTI-time-stepping); row k of the result is the paper's d_{k+1}."""
    w = np.zeros(A.shape[0])
    d = np.zeros((len(m), B.shape[0]))
    for k in range(len(m)):
        w = A @ w + C @ m[k]
        d[k] = B @ w
    return d


def lti_blocks(A, B, C, Nt):
    """F_k = B A^k C, k = 0..Nt-1."""
    F = np.zeros((Nt, B.shape[0], C.shape[1]))
    Ak = np.eye(A.shape[0])
    for k in range(Nt):
        F[k] = B @ Ak @ C
        Ak = A @ Ak
    return F


def lti_blocks_and_run(rng, Nw, Nd, Nm, Nt, m):
    A, B, C = make_lti(rng, Nw, Nd, Nm)
    return lti_blocks(A, B, C, Nt), run_lti(A, B, C, m)


# ---------------------------------------------------------------- forward
def test_matches_time_stepping_lti_system():
    rng = np.random.default_rng(1)
    Nt, Nd, Nm, Nw = 23, 3, 5, 17
    m = rng.standard_normal((Nt, Nm))
    F, d_ts = lti_blocks_and_run(rng, Nw, Nd, Nm, Nt, m)
    d = oracle.apply_F(F, m)
    assert oracle.rel_l2(d, d_ts) < 1e-13


def test_matches_dense_block_matrix():
    rng = np.random.default_rng(2)
    Nt, Nd, Nm = 16, 4, 64
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d = oracle.apply_F(F, m)
    d_dense = (dense_matrix(F) @ m.reshape(-1)).reshape(Nt, Nd)
    assert oracle.rel_l2(d, d_dense) < 1e-14


def test_single_step_is_gemv():
    rng = np.random.default_rng(3)
    F = rng.standard_normal((1, 7, 11))
    m = rng.standard_normal((1, 11))
    d = oracle.apply_F(F, m)
    np.testing.assert_allclose(d[0], np.dot(F[0], m[0]), rtol=1e-15, atol=0)
    dd = rng.standard_normal((1, 7))
    np.testing.assert_allclose(oracle.apply_Ft(F, dd)[0], np.dot(F[0].T, dd[0]), rtol=1e-14)


def test_scalar_system_is_numpy_convolution():
    rng = np.random.default_rng(4)
    Nt = 40
    f = rng.standard_normal(Nt)
    m = rng.standard_normal(Nt)
    d = oracle.apply_F(f.reshape(Nt, 1, 1), m.reshape(Nt, 1))[:, 0]
    np.testing.assert_allclose(d, np.convolve(f, m)[:Nt], rtol=1e-12, atol=1e-13)
    # the transpose of a causal convolution is the correlation
    s = oracle.apply_Ft(f.reshape(Nt, 1, 1), m.reshape(Nt, 1))[:, 0]
    corr = np.array([np.dot(f[: Nt - t], m[t:]) for t in range(Nt)])
    np.testing.assert_allclose(s, corr, rtol=1e-12, atol=1e-13)


def test_parameter_impulse_returns_blocks():
    rng = np.random.default_rng(5)
    Nt, Nd, Nm = 12, 3, 6
    F = _rand_blocks(rng, Nt, Nd, Nm)
    t0, j = 4, 2
    m = np.zeros((Nt, Nm))
    m[t0, j] = 1.0
    d = oracle.apply_F(F, m)
    assert np.all(d[:t0] == 0.0)                          # causality
    for t in range(t0, Nt):
        np.testing.assert_array_equal(d[t], F[t - t0][:, j])


def test_data_impulse_returns_sensor_rows():
    # an adjoint solve from one sensor at the last step yields that sensor's
    # row of every block (how Phase 1 builds F from one adjoint solve per sensor)
    rng = np.random.default_rng(6)
    Nt, Nd, Nm = 9, 4, 5
    F = _rand_blocks(rng, Nt, Nd, Nm)
    s_idx = 3
    e = np.zeros((Nt, Nd))
    e[Nt - 1, s_idx] = 1.0
    s = oracle.apply_Ft(F, e)
    for t in range(Nt):
        np.testing.assert_array_equal(s[t], F[Nt - 1 - t][s_idx])


def test_shift_invariance():
    rng = np.random.default_rng(7)
    Nt, Nd, Nm, tau = 20, 3, 4, 5
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    m[Nt - tau:] = 0.0
    m_shift = np.zeros_like(m)
    m_shift[tau:] = m[: Nt - tau]
    d = oracle.apply_F(F, m)
    d_shift = oracle.apply_F(F, m_shift)
    np.testing.assert_allclose(d_shift[tau:], d[: Nt - tau], rtol=1e-13, atol=1e-14)
    assert np.all(d_shift[:tau] == 0.0)


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_dense_transpose():
    rng = np.random.default_rng(8)
    Nt, Nd, Nm = 16, 4, 64
    F = _rand_blocks(rng, Nt, Nd, Nm)
    d = rng.standard_normal((Nt, Nd))
    s = oracle.apply_Ft(F, d)
    s_dense = (dense_matrix(F).T @ d.reshape(-1)).reshape(Nt, Nm)
    assert oracle.rel_l2(s, s_dense) < 1e-14


def test_adjoint_identity():
    rng = np.random.default_rng(9)
    Nt, Nd, Nm = 31, 5, 33
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((3, Nt, Nm))
    d = rng.standard_normal((3, Nt, Nd))
    lhs = np.sum(oracle.apply_F(F, m) * d)
    rhs = np.sum(m * oracle.apply_Ft(F, d))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)


# ---------------------------------------------------------------- ragged
def test_ragged_is_leading_principal_submatrix():
    rng = np.random.default_rng(10)
    Nt, Nd, Nm = 14, 3, 5
    F = _rand_blocks(rng, Nt, Nd, Nm)
    n = np.array([1, 5, 14, 0], dtype=np.int32)
    m = rng.standard_normal((4, Nt, Nm))
    d_in = rng.standard_normal((4, Nt, Nd))
    Mx = dense_matrix(F)
    d = oracle.apply_F(F, m, n)
    s = oracle.apply_Ft(F, d_in, n)
    for b, nb in enumerate(n):
        sub = Mx[: nb * Nd, : nb * Nm]
        np.testing.assert_allclose(d[b, :nb].reshape(-1), sub @ m[b, :nb].reshape(-1),
                                   rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(s[b, :nb].reshape(-1), sub.T @ d_in[b, :nb].reshape(-1),
                                   rtol=1e-13, atol=1e-14)
        assert np.all(d[b, nb:] == 0.0) and np.all(s[b, nb:] == 0.0)


def test_ragged_equals_short_lti_run():
    rng = np.random.default_rng(11)
    Nt, Nd, Nm, Nw, n = 20, 2, 3, 9, 13
    A, B, C = make_lti(rng, Nw, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d = oracle.apply_F(lti_blocks(A, B, C, Nt), m[None], np.array([n]))[0]
    assert oracle.rel_l2(d[:n], run_lti(A, B, C, m[:n])) < 1e-13
    assert np.all(d[n:] == 0.0)


# ---------------------------------------------------------------- spectrum
def test_spectrum_geometric_closed_form():
    rng = np.random.default_rng(12)
    Nt, Nd, Nm, r = 21, 3, 4, 0.83
    A0 = rng.standard_normal((Nd, Nm))
    F = np.stack([r ** k * A0 for k in range(Nt)])
    for L in (2 * Nt, 2 * Nt + 6):
        Fh = oracle.spectrum(F, L)
        w = np.arange(L // 2 + 1)
        z = r * np.exp(-2j * np.pi * w / L)
        closed = (1 - z ** Nt) / (1 - z)
        np.testing.assert_allclose(Fh, closed[:, None, None] * A0[None], rtol=1e-12, atol=1e-12)
    Fh = oracle.spectrum(F, 2 * Nt)
    np.testing.assert_allclose(Fh[0], F.sum(0), rtol=1e-13)
    alt = ((-1.0) ** np.arange(Nt))[:, None, None]
    np.testing.assert_allclose(Fh[Nt], (alt * F).sum(0), rtol=1e-12, atol=1e-13)
    assert np.max(abs(Fh[0].imag)) == 0.0


def test_spectrum_block_diagonalises_the_embedded_circulant():
    # convolution theorem through a library FFT (test reference only)
    rng = np.random.default_rng(13)
    Nt, Nd, Nm = 18, 3, 7
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    for L in (2 * Nt - 1 + 1, 2 * Nt + 4):
        Fh = oracle.spectrum(F, L)
        xh = np.fft.rfft(m, n=L, axis=0)
        yh = np.einsum("wij,wj->wi", Fh, xh)
        y = np.fft.irfft(yh, n=L, axis=0)[:Nt]
        assert oracle.rel_l2(y, oracle.apply_F(F, m)) < 1e-13
        # adjoint: conjugate-transposed blocks
        d = rng.standard_normal((Nt, Nd))
        dh = np.fft.rfft(d[::-1], n=L, axis=0)   # time reversal turns F^T into a causal map
        sh = np.einsum("wij,wi->wj", Fh, dh)
        s = np.fft.irfft(sh, n=L, axis=0)[:Nt][::-1]
        assert oracle.rel_l2(s, oracle.apply_Ft(F, d)) < 1e-13


# ---------------------------------------------------------------- misfit
def test_misfit_gradient_central_difference():
    rng = np.random.default_rng(14)
    Nt, Nd, Nm = 12, 3, 8
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d_obs = rng.standard_normal((Nt, Nd))
    var = rng.uniform(0.5, 2.0, Nd)
    phi, g = oracle.misfit_and_grad(F, m, d_obs, var)
    for trial in range(3):
        v = rng.standard_normal((Nt, Nm))
        eps = 1e-3 * np.linalg.norm(m) / np.linalg.norm(v)
        fp, _ = oracle.misfit_and_grad(F, m + eps * v, d_obs, var)
        fm, _ = oracle.misfit_and_grad(F, m - eps * v, d_obs, var)
        fd = (fp - fm) / (2 * eps)        # exact for a quadratic, up to rounding
        assert abs(fd - np.sum(g * v)) <= 1e-7 * abs(np.sum(g * v)) + 1e-9


def test_misfit_matches_dense_normal_equations():
    rng = np.random.default_rng(15)
    Nt, Nd, Nm = 10, 4, 6
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d_obs = rng.standard_normal((Nt, Nd))
    var = rng.uniform(0.5, 2.0, Nt * Nd)
    Mx = dense_matrix(F)
    r = Mx @ m.reshape(-1) - d_obs.reshape(-1)
    phi_ref = 0.5 * np.sum(r * r / var)
    g_ref = Mx.T @ (r / var)
    phi, g = oracle.misfit_and_grad(F, m, d_obs, var)
    assert abs(phi - phi_ref) <= 1e-13 * phi_ref
    assert oracle.rel_l2(g.reshape(-1), g_ref) < 1e-13


def test_data_space_hessian_is_symmetric_psd():
    rng = np.random.default_rng(16)
    Nt, Nd, Nm = 8, 3, 10
    F = _rand_blocks(rng, Nt, Nd, Nm)
    n = Nt * Nd
    E = np.eye(n).reshape(n, Nt, Nd)
    K = oracle.data_space_hessian(F, E).reshape(n, n).T     # columns F F^T e_j
    Mx = dense_matrix(F)
    np.testing.assert_allclose(K, Mx @ Mx.T, rtol=1e-12, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(0.5 * (K + K.T))) > -1e-10


# ---------------------------------------------------------------- golden
def test_hand_worked_examples():
    g = json.load(open(GOLDEN))
    s = g["scalar_lti"]
    F = np.array(s["F"])
    np.testing.assert_array_equal(oracle.apply_F(F, np.array(s["m"])), np.array(s["d"]))
    np.testing.assert_array_equal(oracle.apply_Ft(F, np.array(s["adj_in"])), np.array(s["adj_out"]))
    Fh = oracle.spectrum(F, s["L"])[:, 0, 0]
    b = s["spectrum_bins"]
    np.testing.assert_allclose(Fh[b].real, s["spectrum_re"], atol=1e-14)
    np.testing.assert_allclose(Fh[b].imag, s["spectrum_im"], atol=1e-14)
    phi, grad = oracle.misfit_and_grad(F, np.array(s["m"]), np.array(s["d_obs"]), s["noise_var"])
    assert phi == s["misfit"]
    np.testing.assert_array_equal(grad, np.array(s["grad"]))
    # the same scalar system, stepped
    A, B, C = s["A"], s["B"], s["C"]
    w, d = 0.0, []
    for mk in np.array(s["m"])[:, 0]:
        w = A * w + C * mk
        d.append(B * w)
    np.testing.assert_array_equal(np.array(d), np.array(s["d"])[:, 0])
    blk = g["block_2x2"]
    F = np.array(blk["F"])
    np.testing.assert_array_equal(oracle.apply_F(F, np.array(blk["m"])), np.array(blk["d"]))
    np.testing.assert_array_equal(oracle.apply_Ft(F, np.array(blk["adj_in"])), np.array(blk["adj_out"]))


def test_rel_l2_hand_worked():
    """The error metric every parity verdict goes through, on hand-computed
    cases whose value differs from its square, the max-norm ratio, the ratio
    over the result's norm and per-right-hand-side maxima or means."""
    g = json.load(open(GOLDEN))
    for key in ("rel_l2", "rel_l2_batched", "rel_l2_zero_reference"):
        c = g[key]
        assert abs(oracle.rel_l2(np.array(c["y"]), np.array(c["y_ref"])) - c["value"]) <= 1e-15, key


def _broken_rel_l2_variants():
    def squared(y, y_ref):
        return float(np.sum((y - y_ref) ** 2) / np.sum(y_ref ** 2))

    def max_norm(y, y_ref):
        return float(np.max(abs(y - y_ref)) / np.max(abs(y_ref)))

    def over_result(y, y_ref):
        return float(np.linalg.norm((y - y_ref).ravel()) / np.linalg.norm(y.ravel()))

    def worst_rhs(y, y_ref):
        return max(float(np.linalg.norm(y[b] - y_ref[b]) / np.linalg.norm(y_ref[b])) for b in range(len(y)))

    return [squared, max_norm, over_result, worst_rhs]


@pytest.mark.parametrize("broken", _broken_rel_l2_variants(), ids=lambda f: f.__name__)
def test_rel_l2_pins_catch_planted_mistakes(broken):
    g = json.load(open(GOLDEN))
    caught = False
    for key in ("rel_l2", "rel_l2_batched"):
        c = g[key]
        y, y_ref = np.array(c["y"]), np.array(c["y_ref"])
        with np.errstate(divide="ignore", invalid="ignore"):
            got = broken(y, y_ref)
        caught |= not abs(got - c["value"]) <= 1e-15
    assert caught


# ---------------------------------------------------------------- planted mistakes
def _broken_forward_variants():
    def dropped_last_lag(F, m, nt_active=None):
        Fz = F.copy()
        Fz[-1] = 0.0
        return T.apply_F(Fz, m, nt_active)

    def off_by_one_lag(F, m, nt_active=None):
        Fs = np.concatenate([F[1:], np.zeros_like(F[:1])])
        return T.apply_F(Fs, m, nt_active)

    def anticausal(F, m, nt_active=None):
        return T.apply_F(F, np.asarray(m)[..., ::-1, :], nt_active)[..., ::-1, :]

    def transposed_blocks(F, m, nt_active=None):
        Ft = np.transpose(F, (0, 2, 1))[:, : F.shape[1], : F.shape[2]]
        return T.apply_F(np.ascontiguousarray(Ft), m, nt_active)

    def sign_flip_odd(F, m, nt_active=None):
        sgn = ((-1.0) ** np.arange(F.shape[0]))[:, None, None]
        return T.apply_F(F * sgn, m, nt_active)

    return [dropped_last_lag, off_by_one_lag, anticausal, transposed_blocks, sign_flip_odd]


@pytest.mark.parametrize("broken", _broken_forward_variants(), ids=lambda f: f.__name__)
def test_pins_catch_planted_forward_mistakes(broken):
    rng = np.random.default_rng(17)
    Nt, Nd, Nm, Nw = 16, 4, 4, 12
    m = rng.standard_normal((Nt, Nm))
    F, d_ts = lti_blocks_and_run(rng, Nw, Nd, Nm, Nt, m)
    caught = oracle.rel_l2(broken(F, m), d_ts) > 1e-8
    caught |= oracle.rel_l2(broken(F, m), (dense_matrix(F) @ m.reshape(-1)).reshape(Nt, Nd)) > 1e-8
    assert caught


def test_pins_catch_planted_adjoint_mistakes():
    rng = np.random.default_rng(18)
    Nt, Nd, Nm = 10, 3, 5
    F = _rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))

    def wrong_direction(F, d):                  # F_k applied forward in time
        S = np.zeros((Nt, Nm))
        for k in range(Nt):
            S[k:] += d[: Nt - k] @ F[k]
        return S

    def dropped_diagonal(F, d):
        Fz = F.copy()
        Fz[0] = 0.0
        return T.apply_Ft(Fz, d)

    for bad in (wrong_direction, dropped_diagonal):
        lhs = np.sum(oracle.apply_F(F, m) * d)
        assert abs(lhs - np.sum(m * bad(F, d))) > 1e-8 * abs(lhs)


def test_generator_is_counter_based_and_reproducible():
    w = synth.CONFIGS["tiny"]
    full = synth.operator_blocks(w)
    rows = synth.operator_blocks(w, rows=[1, 3], cols=[5, 6, 63])
    np.testing.assert_array_equal(rows, full[:, [1, 3]][:, :, [5, 6, 63]])
    z = synth.normal(7, 1, np.arange(200000), 0, 0)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    # Philox4x32-10 known-answer vectors (Salmon et al., SC'11, Random123)
    M = 0xFFFFFFFF
    out = synth.philox4x32_10(np.uint64(0), np.uint64(0), np.uint64(0), np.uint64(0), 0, 0)
    assert [int(x) for x in out] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    out = synth.philox4x32_10(*(np.uint64(M),) * 4, M, M)
    assert [int(x) for x in out] == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    out = synth.philox4x32_10(np.uint64(0x243F6A88), np.uint64(0x85A308D3), np.uint64(0x13198A2E),
                              np.uint64(0x03707344), 0xA4093822, 0x299F31D0)
    assert [int(x) for x in out] == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_generator_torch_matches_numpy():
    torch = pytest.importorskip("torch")
    w = synth.CONFIGS["medium"]
    a = synth.operator_rows_cols(w, [0, 5, 127], rows=[0, 17], cols=np.arange(100))
    b = synth.operator_rows_cols(w, [0, 5, 127], rows=[0, 17], cols=np.arange(100),
                                 backend="torch").numpy()
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-16)
    m1 = synth.param_series(w, 2)
    m2 = synth.param_series(w, 2, backend="torch").numpy()
    np.testing.assert_allclose(m1, m2, rtol=1e-14, atol=1e-15)
