"""Pins for the posterior oracle (oracle/posterior.py) against routes that do
not share its formulas: the dense block matrices of F and F_q, the
parameter-space normal equations of the MAP problem (the Woodbury identity
turned around: K and the data space never appear there), time-stepping an
LTI system for the p2q map, hand-worked factorisations, and planted mistakes
that some pin must catch."""
import json
import os

import numpy as np
import pytest

from oracle import posterior as P
from oracle import toeplitz as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def dense(F):
    """(Nd Nt) x (Nm Nt) block lower-triangular matrix with block (i, j) = F_{i-j}."""
    Nt, Nd, Nm = F.shape
    Mx = np.zeros((Nd * Nt, Nm * Nt))
    for i in range(Nt):
        for j in range(i + 1):
            Mx[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = F[i - j]
    return Mx


def blocks(rng, Nt, Nr, Nm, tau=3.0):
    return rng.standard_normal((Nt, Nr, Nm)) * np.exp(-np.arange(Nt) / tau)[:, None, None] / np.sqrt(Nm)


def normal_equations(F, noise_var, prior_var):
    """H = F_d^T Gamma_noise^{-1} F_d + Gamma_prior^{-1} in parameter space
    (section 2: the Hessian of the MAP objective, equation mmap-problem)."""
    Nt, Nd, _ = F.shape
    Fd = dense(F)
    var = T._noise_var_full(noise_var, Nt, Nd).reshape(-1)
    H = Fd.T @ (Fd / var[:, None]) + np.eye(Fd.shape[1]) / prior_var
    return Fd, var, H


SHAPE = dict(Nt=8, Nd=3, Nm=7)


@pytest.mark.parametrize("var_kind", ["scalar", "sensor", "full"])
def test_data_space_matrix_is_dense_product(var_kind):
    rng = np.random.default_rng(1)
    Nt, Nd, Nm = SHAPE["Nt"], SHAPE["Nd"], SHAPE["Nm"]
    F = blocks(rng, Nt, Nd, Nm)
    var = {"scalar": 0.3, "sensor": rng.uniform(0.1, 1.0, Nd), "full": rng.uniform(0.1, 1.0, Nd * Nt)}[var_kind]
    K = P.data_space_matrix(F, var, prior_var=2.5)
    Fd = dense(F)
    Kref = 2.5 * Fd @ Fd.T + np.diag(T._noise_var_full(var, Nt, Nd).reshape(-1))
    np.testing.assert_allclose(K, Kref, rtol=1e-13, atol=1e-14)
    # a general second factor (F G^T, G not a multiple of F)
    G = blocks(rng, Nt, Nd, Nm)
    np.testing.assert_allclose(P.data_space_matrix(F, var, G=G),
                               Fd @ dense(G).T + np.diag(T._noise_var_full(var, Nt, Nd).reshape(-1)),
                               rtol=1e-13, atol=1e-14)


def test_data_space_matrix_columns_are_operator_columns():
    rng = np.random.default_rng(2)
    F = blocks(rng, 12, 4, 9)
    K = P.data_space_matrix(F, 0.1, prior_var=0.7)
    for j in (0, 3, 17, 47):
        e = np.zeros((12, 4))
        e.reshape(-1)[j] = 1.0
        col = 0.7 * T.data_space_hessian(F, e).reshape(-1)
        col[j] += 0.1
        np.testing.assert_allclose(K[:, j], col, rtol=1e-13, atol=1e-15)
    assert np.allclose(K, K.T, rtol=0, atol=1e-15)
    assert np.min(np.linalg.eigvalsh(K)) > 0.1 - 1e-12          # Gamma_noise + PSD


def test_cholesky_and_solve_hand_worked():
    g = json.load(open(GOLDEN))["cholesky_3x3"]
    K, L, b, x = (np.array(g[k], dtype=float) for k in ("K", "L", "b", "x"))
    np.testing.assert_allclose(P.cholesky_lower(K), L, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P.solve_with_factor(L, b), x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("prior_var", [1.0, 0.3])
def test_map_point_equals_parameter_space_normal_equations(prior_var):
    rng = np.random.default_rng(3)
    Nt, Nd, Nm = SHAPE["Nt"], SHAPE["Nd"], SHAPE["Nm"]
    F = blocks(rng, Nt, Nd, Nm)
    var = rng.uniform(0.05, 0.2, Nd)
    d = rng.standard_normal((Nt, Nd))
    Fd, v, H = normal_equations(F, var, prior_var)
    ref = np.linalg.solve(H, Fd.T @ (d.reshape(-1) / v)).reshape(Nt, Nm)
    np.testing.assert_allclose(P.map_point(F, d, var, prior_var), ref, rtol=1e-11, atol=1e-13)


def test_posterior_cov_apply_is_inverse_hessian():
    rng = np.random.default_rng(4)
    Nt, Nd, Nm = SHAPE["Nt"], SHAPE["Nd"], SHAPE["Nm"]
    F = blocks(rng, Nt, Nd, Nm)
    _, _, H = normal_equations(F, 0.1, 0.5)
    v = rng.standard_normal((Nt, Nm))
    np.testing.assert_allclose(P.posterior_cov_apply(F, v, 0.1, 0.5), np.linalg.solve(H, v.reshape(-1)).reshape(Nt, Nm),
                               rtol=1e-11, atol=1e-13)


def test_qoi_steps_hand_worked():
    assert list(P.qoi_steps(10, 5)) == [4, 9]
    assert list(P.qoi_steps(6, 1)) == [0, 1, 2, 3, 4, 5]
    assert list(P.qoi_steps(500, 10))[:3] == [9, 19, 29] and P.qoi_steps(500, 10)[-1] == 499


def test_p2q_matches_time_stepped_lti_observed_at_qoi_steps():
    """q from stepping w_{k+1} = A w_k + C m_k and observing q_{k+1} = B_q w_{k+1}
    at the QoI steps equals the decimated Toeplitz map of F_q,k = B_q A^k C."""
    rng = np.random.default_rng(5)
    Nw, Nq, Nm, Nt, stride = 10, 3, 4, 12, 3
    A = rng.standard_normal((Nw, Nw))
    A *= 0.9 / max(abs(np.linalg.eigvals(A)))
    Bq, C = rng.standard_normal((Nq, Nw)), rng.standard_normal((Nw, Nm))
    Fq = np.stack([Bq @ np.linalg.matrix_power(A, k) @ C for k in range(Nt)])
    m = rng.standard_normal((Nt, Nm))
    w, q = np.zeros(Nw), []
    for k in range(Nt):
        w = A @ w + C @ m[k]
        q.append(Bq @ w)
    q = np.array(q)[stride - 1::stride]
    np.testing.assert_allclose(P.apply_Fq(Fq, m, stride), q, rtol=1e-12, atol=1e-12)


def test_p2q_adjoint_identity_and_dense_rows():
    rng = np.random.default_rng(6)
    Nt, Nq, Nm, stride = 12, 2, 5, 4
    Fq = blocks(rng, Nt, Nq, Nm)
    m = rng.standard_normal((Nt, Nm))
    q = rng.standard_normal((Nt // stride, Nq))
    lhs = np.sum(P.apply_Fq(Fq, m, stride) * q)
    rhs = np.sum(m * P.apply_Fqt(Fq, q, stride))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    rows = np.concatenate([np.arange(t * Nq, (t + 1) * Nq) for t in P.qoi_steps(Nt, stride)])
    np.testing.assert_allclose(P.apply_Fq(Fq, m, stride).reshape(-1), dense(Fq)[rows] @ m.reshape(-1), rtol=1e-13)


def test_d2q_and_qoi_covariance_match_parameter_space():
    rng = np.random.default_rng(7)
    Nt, Nd, Nq, Nm, stride = 8, 3, 2, 6, 2
    F = blocks(rng, Nt, Nd, Nm)
    Fq = blocks(rng, Nt, Nq, Nm)
    var, gam = rng.uniform(0.05, 0.2, Nd * Nt), 0.8
    Fd, v, H = normal_equations(F, var, gam)
    rows = np.concatenate([np.arange(t * Nq, (t + 1) * Nq) for t in P.qoi_steps(Nt, stride)])
    Fqd = dense(Fq)[rows]
    Hinv = np.linalg.inv(H)
    Q = P.d2q_matrix(Fq, F, var, gam, stride)
    np.testing.assert_allclose(Q, Fqd @ Hinv @ (Fd.T / v[None, :]), rtol=1e-10, atol=1e-12)
    C = P.qoi_posterior_cov(Fq, F, var, gam, stride)
    np.testing.assert_allclose(C, Fqd @ Hinv @ Fqd.T, rtol=1e-10, atol=1e-12)
    assert np.allclose(C, C.T, atol=1e-12) and np.min(np.linalg.eigvalsh(0.5 * (C + C.T))) > 0
    # the online QoI prediction Q d equals F_q applied to the MAP point
    d = rng.standard_normal((Nt, Nd))
    np.testing.assert_allclose(Q @ d.reshape(-1), P.apply_Fq(Fq, P.map_point(F, d, var, gam), stride).reshape(-1),
                               rtol=1e-10, atol=1e-12)


def _broken_map_variants():
    def plus_sign(F, d, var, gam):                  # (I + G* K^-1 F) instead of (I - ...)
        Nt, Nd, _ = F.shape
        L = P.cholesky_lower(P.data_space_matrix(F, var, gam))
        u = gam * T.apply_Ft(F, d / T._noise_var_full(var, Nt, Nd))
        z = P.solve_with_factor(L, T.apply_F(F, u).reshape(-1)).reshape(Nt, Nd)
        return u + gam * T.apply_Ft(F, z)

    def no_noise_weight(F, d, var, gam):            # Gamma_noise^{-1} dropped
        return P.map_point(F, d * T._noise_var_full(var, *F.shape[:2]), var, gam)

    def noise_missing_in_K(F, d, var, gam):         # K = F G* only
        Nt, Nd, _ = F.shape
        K = P.data_space_matrix(F, 1e-12, gam)
        return P.map_point(F, d, var, gam, L=P.cholesky_lower(K))

    def prior_not_scaled(F, d, var, gam):           # G* = F* whatever the prior
        return P.map_point(F, d, var, 1.0)

    return [plus_sign, no_noise_weight, noise_missing_in_K, prior_not_scaled]


@pytest.mark.parametrize("broken", _broken_map_variants(), ids=lambda f: f.__name__)
def test_pins_catch_planted_map_mistakes(broken):
    rng = np.random.default_rng(8)
    Nt, Nd, Nm = SHAPE["Nt"], SHAPE["Nd"], SHAPE["Nm"]
    F = blocks(rng, Nt, Nd, Nm)
    var, gam = rng.uniform(0.05, 0.2, Nd), 0.4
    d = rng.standard_normal((Nt, Nd))
    Fd, v, H = normal_equations(F, var, gam)
    ref = np.linalg.solve(H, Fd.T @ (d.reshape(-1) / v))
    assert np.linalg.norm(broken(F, d, var, gam).reshape(-1) - ref) > 1e-6 * np.linalg.norm(ref)


def test_pins_catch_planted_qoi_step_mistake():
    rng = np.random.default_rng(9)
    Fq = blocks(rng, 12, 2, 3)
    m = rng.standard_normal((12, 3))
    full = T.apply_F(Fq, m)
    # observing at the first step of each QoI interval instead of the last
    assert not np.allclose(P.apply_Fq(Fq, m, 4), full[0::4])
