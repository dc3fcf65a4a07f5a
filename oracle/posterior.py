"""FP64 CPU oracle for the offline and online phases built on the p2o map:
the data-space matrix K and its Cholesky factor, the real-time MAP point,
actions of the posterior covariance, the multi-rate parameter-to-QoI (p2q)
map, the data-to-QoI map and the QoI posterior covariance.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module;
only the test-suite and the benchmark's CPU-baseline leg call it.  It shares
no code with the HIP library.  Each function is the plain definition from
the paper, in float64, with numpy / scipy routines (matrix products, a
Cholesky factorisation, triangular solves) as its steps.

The prior is the stand-in Gamma_prior = gamma I (a scalar variance; the
paper's elliptic prior needs PDE solves and is out of scope), so that
G* := Gamma_prior F* = gamma F* (section 4, Phase 2, the definition of G*
before equation fast-Hessian-matvec) is the same block Toeplitz map as F*
scaled.  The noise covariance Gamma_noise is diagonal (section 4, Phase 2),
given as 1, Nd or Nt*Nd variances as in ``toeplitz.misfit_and_grad``.

Data-space index: j = t * Nd + s (time-major, as the data series
[Nt][Nd]); K is N x N with N = Nt * Nd.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .toeplitz import _noise_var_full, apply_F, apply_Ft


def data_space_matrix(F, noise_var, prior_var=1.0, G=None):
    """K = Gamma_noise + F G^T with G = prior_var * F unless given (section 4,
    Phase 2: K = Gamma_noise + F Gamma_prior F*, equations woodbury and
    fast-Hessian-matvec), as a dense N x N array.

    Block (i, j) of F G^T is sum_k F_{i,k} G_{j,k}^T over the time blocks k
    both block rows reach, k <= min(i, j), with F_{i,k} = F_{i-k}:
        (F G^T)_{ij} = sum_{k=0}^{min(i,j)} F_{i-k} G_{j-k}^T .
    For i = j + d (d >= 0) and b = j - k this is sum_{b=0}^{j} F_{b+d} G_b^T,
    a running sum over j; the blocks above the diagonal are the same with the
    roles of F and G exchanged.
    """
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, _ = F.shape
    G = prior_var * F if G is None else np.asarray(G, dtype=np.float64)
    K = np.zeros((Nt, Nd, Nt, Nd))
    for d in range(Nt):
        # products F_{b+d} G_b^T and F_b G_{b+d}^T for b = 0 .. Nt-1-d
        low = np.cumsum(np.matmul(F[d:], np.transpose(G[:Nt - d], (0, 2, 1))), axis=0)
        up = np.cumsum(np.matmul(F[:Nt - d], np.transpose(G[d:], (0, 2, 1))), axis=0)
        for j in range(Nt - d):
            K[j + d, :, j, :] = low[j]              # block (j + d, j)
            K[j, :, j + d, :] = up[j]               # block (j, j + d)
    K = K.reshape(Nt * Nd, Nt * Nd)
    K[np.diag_indices_from(K)] += _noise_var_full(noise_var, Nt, Nd).reshape(-1)
    return K


def cholesky_lower(K):
    """L with K = L L^T, L lower triangular (section 4, Phase 2: K is
    Cholesky-factorised offline)."""
    return np.linalg.cholesky(np.asarray(K, dtype=np.float64))


def solve_with_factor(L, b):
    """K^{-1} b from the factor L of K = L L^T by the two triangular solves of
    the online phase (section 4, Phase 4): L y = b, then L^T x = y.  ``b`` is
    a vector or an [N, nrhs] array."""
    y = scipy.linalg.solve_triangular(L, b, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


def _flat_data(d, Nt, Nd):
    return np.asarray(d, dtype=np.float64).reshape(Nt * Nd)


def map_point(F, d_obs, noise_var, prior_var=1.0, L=None):
    """MAP point with zero prior mean by equation real-time-parameter
    (section 4, Phase 4):
        m_map = (I - G* K^{-1} F) G* Gamma_noise^{-1} d_obs,  G* = gamma F*,
    in its steps: u = G* Gamma_noise^{-1} d_obs; y = F u; z = K^{-1} y;
    m_map = u - G* z.  ``L`` is K's Cholesky factor (computed here if None).
    d_obs is [Nt, Nd]; returns [Nt, Nm]."""
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, _ = F.shape
    if L is None:
        L = cholesky_lower(data_space_matrix(F, noise_var, prior_var))
    var = _noise_var_full(noise_var, Nt, Nd)
    u = prior_var * apply_Ft(F, np.asarray(d_obs, dtype=np.float64) / var)
    y = apply_F(F, u)
    z = solve_with_factor(L, _flat_data(y, Nt, Nd)).reshape(Nt, Nd)
    return u - prior_var * apply_Ft(F, z)


def posterior_cov_apply(F, v, noise_var, prior_var=1.0, L=None):
    """Gamma_post v by equation fast-Hessian-matvec (section 4, Phase 2):
        Gamma_post = (I - G* K^{-1} F) Gamma_prior,  Gamma_prior = gamma I:
    w = gamma v; y = F w; z = K^{-1} y; Gamma_post v = w - G* z.
    v is [Nt, Nm]; returns [Nt, Nm]."""
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, _ = F.shape
    if L is None:
        L = cholesky_lower(data_space_matrix(F, noise_var, prior_var))
    w = prior_var * np.asarray(v, dtype=np.float64)
    z = solve_with_factor(L, _flat_data(apply_F(F, w), Nt, Nd)).reshape(Nt, Nd)
    return w - prior_var * apply_Ft(F, z)


# ---------------------------------------------------------------- p2q map
def qoi_steps(Nt, stride):
    """Fine time steps at which the QoIs are observed: the QoI grid is
    `stride` times coarser than the parameter grid and its step i ends where
    parameter step stride (i + 1) - 1 ends (0-based; section 5: parameters
    at 10 Hz, QoIs at 1 Hz, N_t = 500, N_t^q = 50)."""
    assert Nt % stride == 0, (Nt, stride)
    return np.arange(stride - 1, Nt, stride)


def apply_Fq(Fq, m, stride=1, nt_active=None):
    """q = F_q m (equation p2q): the block lower-triangular Toeplitz map of
    the QoI blocks Fq [Nt, Nq, Nm] applied on the parameter grid, observed at
    the QoI steps (section 2, remark on distinct temporal discretisations of
    parameters, data and QoIs).  Returns [..., Nt / stride, Nq]."""
    full = apply_F(Fq, m, nt_active)
    return full[..., qoi_steps(np.asarray(Fq).shape[0], stride), :]


def apply_Fqt(Fq, q, stride=1, nt_active=None):
    """F_q^* q, the adjoint of ``apply_Fq``: the QoI series placed at its
    steps on the parameter grid (zeros between), then the adjoint of the
    Toeplitz map.  q is [..., Nt / stride, Nq]."""
    Fq = np.asarray(Fq, dtype=np.float64)
    Nt, Nq, _ = Fq.shape
    q = np.asarray(q, dtype=np.float64)
    full = np.zeros(q.shape[:-2] + (Nt, Nq))
    full[..., qoi_steps(Nt, stride), :] = q
    return apply_Ft(Fq, full, nt_active)


def d2q_matrix(Fq, F, noise_var, prior_var=1.0, stride=1, L=None):
    """Data-to-QoI map Q = F_q (I - G* K^{-1} F) G* Gamma_noise^{-1}
    (section 4, Phase 3, equation d2q-map), as a dense (Nq Ntq) x (Nd Nt)
    array, row by row: row r is Q^T e_r = Gamma_noise^{-1} G (I - F* K^{-1} G)
    F_q^* e_r with G = gamma F (K is symmetric)."""
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, _ = F.shape
    Nq = np.asarray(Fq).shape[1]
    Ntq = Nt // stride
    if L is None:
        L = cholesky_lower(data_space_matrix(F, noise_var, prior_var))
    var = _noise_var_full(noise_var, Nt, Nd)
    Q = np.zeros((Ntq * Nq, Nt * Nd))
    for r in range(Ntq * Nq):
        e = np.zeros(Ntq * Nq)
        e[r] = 1.0
        x = apply_Fqt(Fq, e.reshape(Ntq, Nq), stride)                 # F_q^* e_r
        y = prior_var * apply_F(F, x)                                 # G x
        z = solve_with_factor(L, _flat_data(y, Nt, Nd)).reshape(Nt, Nd)
        w = x - apply_Ft(F, z)                                        # (I - F* K^{-1} G) x
        Q[r] = (prior_var * apply_F(F, w) / var).reshape(-1)          # Gamma_noise^{-1} G w
    return Q


def qoi_posterior_cov(Fq, F, noise_var, prior_var=1.0, stride=1, L=None):
    """Gamma_post(q) = F_q (I - G* K^{-1} F) G_q^* with G_q^* = gamma F_q^*
    (section 4, Phase 3, equation fast-qoi-covariance), dense
    (Nq Ntq) x (Nq Ntq), column by column."""
    F = np.asarray(F, dtype=np.float64)
    Nt = F.shape[0]
    Nq = np.asarray(Fq).shape[1]
    Ntq = Nt // stride
    if L is None:
        L = cholesky_lower(data_space_matrix(F, noise_var, prior_var))
    C = np.zeros((Ntq * Nq, Ntq * Nq))
    for c in range(Ntq * Nq):
        e = np.zeros(Ntq * Nq)
        e[c] = 1.0
        v = apply_Fqt(Fq, e.reshape(Ntq, Nq), stride)                 # F_q^* e_c
        C[:, c] = apply_Fq(Fq, posterior_cov_apply(F, v, noise_var, prior_var, L), stride).reshape(-1)
    return C
