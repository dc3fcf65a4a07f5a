"""FP64 CPU oracle for the parameter-to-observable (p2o) map of a linear
time-invariant system and its adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module;
only the test-suite, the smoke check and the benchmark's CPU-baseline leg
call it.  It shares no code with the HIP library: no FFT, no quantisation,
no kernels.  Every function is the plain definition, in float64, written for
a reader to check against the paper by eye.

Notation (0-based time index).  The discrete system is stepped with a single
step explicit scheme, w_{k+1} = A w_k + C m_k, d_{k+1} = B w_{k+1}, w_0 = 0
(paper section 2, "Discrete LTI system", equations LTI-time-stepping and
LTI-time-discrete).  Unrolled, this is the causal block convolution

    d_t = sum_{k=0}^{t} F_k m_{t-k},    F_k = B A^k C,   t = 0..Nt-1,

i.e. the block lower-triangular Toeplitz matrix of equation ShiftInvariance,
whose first block column is (F_0, F_1, ..., F_{Nt-1}) (the paper's F_{k+1,1};
its d_{t+1} is our d_t).  Operators are given by their time-domain blocks
``F`` with shape [Nt, Nd, Nm]; parameter series m have shape [..., Nt, Nm]
(time-major blocks m_j, section 2 after equation p2o), data series d have
shape [..., Nt, Nd].

The fast method (section 4, "FFT-based GPU-accelerated p2o and p2q
matvecs") reaches these results exactly up to rounding, so the oracle is the
definition itself.
"""
from __future__ import annotations

import numpy as np


def _as_batched(x: np.ndarray, last: int):
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 2:
        return x[None], True
    assert x.ndim == 3 and x.shape[-1] == last, x.shape
    return x, False


def _lengths(nt_active, nrhs: int, Nt: int) -> np.ndarray:
    if nt_active is None:
        return np.full(nrhs, Nt, dtype=np.int64)
    n = np.asarray(nt_active, dtype=np.int64).reshape(-1)
    assert n.shape == (nrhs,) and np.all((n >= 0) & (n <= Nt)), n
    return n


def apply_F(F: np.ndarray, m: np.ndarray, nt_active=None) -> np.ndarray:
    """d = F m: d_t = sum_{k=0}^{t} F_k m_{t-k}  (equations LTI-time-discrete,
    ShiftInvariance, p2o).

    ``nt_active[b]`` = n restricts right-hand side b to the leading n x n
    block principal submatrix: inputs m_t with t >= n count as zero and
    outputs d_t with t >= n are zero.
    """
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, Nm = F.shape
    M, squeeze = _as_batched(m, Nm)
    assert M.shape[1] == Nt
    n = _lengths(nt_active, M.shape[0], Nt)
    D = np.zeros((M.shape[0], Nt, Nd))
    for b in range(M.shape[0]):
        nb = int(n[b])
        mb = M[b, :nb]
        for k in range(nb):
            # every output step t >= k picks up F_k m_{t-k}
            D[b, k:nb] += mb[: nb - k] @ F[k].T
    return D[0] if squeeze else D


def apply_Ft(F: np.ndarray, d: np.ndarray, nt_active=None) -> np.ndarray:
    """m' = F^T d, the adjoint of ``apply_F`` (F is real, so F* = F^T; section 4
    applies the adjoint through the conjugate-transposed Fourier blocks):

        m'_t = sum_{k=0}^{Nt-1-t} F_k^T d_{t+k}.

    ``nt_active`` as in ``apply_F`` (the transpose of the same restriction).
    """
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, Nm = F.shape
    D, squeeze = _as_batched(d, Nd)
    assert D.shape[1] == Nt
    n = _lengths(nt_active, D.shape[0], Nt)
    S = np.zeros((D.shape[0], Nt, Nm))
    for b in range(D.shape[0]):
        nb = int(n[b])
        db = D[b, :nb]
        for k in range(nb):
            # input step t+k >= k reaches parameter step t through F_k^T
            S[b, : nb - k] += db[k:nb] @ F[k]
    return S[0] if squeeze else S


def _noise_var_full(noise_var, Nt: int, Nd: int) -> np.ndarray:
    v = np.asarray(noise_var, dtype=np.float64).reshape(-1)
    if v.size == 1:
        return np.full((Nt, Nd), v[0])
    if v.size == Nd:
        return np.broadcast_to(v[None, :], (Nt, Nd)).copy()
    assert v.size == Nt * Nd, v.size
    return v.reshape(Nt, Nd)


def misfit_and_grad(F, m, d_obs, noise_var, nt_active=None):
    """Data misfit and its gradient with diagonal noise covariance
    Gamma_noise = diag(noise_var) (section 2, MAP objective and normal
    equations mmap-problem; section 4, diagonal Gamma_noise):

        r = F m - d_obs,  Phi = 1/2 r^T Gamma_noise^{-1} r,
        grad Phi = F^T Gamma_noise^{-1} r.

    ``noise_var`` has 1, Nd (per sensor) or Nt*Nd (per step and sensor)
    entries.  Returns (Phi per right-hand side, gradient).
    """
    F = np.asarray(F, dtype=np.float64)
    Nt, Nd, _ = F.shape
    M, squeeze = _as_batched(m, F.shape[2])
    Dobs = np.asarray(d_obs, dtype=np.float64).reshape(M.shape[0], Nt, Nd)
    var = _noise_var_full(noise_var, Nt, Nd)
    n = _lengths(nt_active, M.shape[0], Nt)
    r = apply_F(F, M, n) - Dobs
    for b in range(M.shape[0]):
        r[b, n[b]:] = 0.0            # steps past the active length carry no data
    w = r / var[None]
    phi = 0.5 * np.einsum("btd,btd->b", r, w)
    g = apply_Ft(F, w, n)
    if squeeze:
        return phi[0], g[0]
    return phi, g


def data_space_hessian(F, e, nt_active=None):
    """h = F (F^T e): columns of the data-space operator F Gamma F^* with
    Gamma = I, as used to assemble K = Gamma_noise + F Gamma_prior F^*
    column by column (section 4, Phase 2, equation woodbury)."""
    return apply_F(F, apply_Ft(F, e, nt_active), nt_active)


def spectrum(F: np.ndarray, L: int) -> np.ndarray:
    """Half spectrum of the zero-padded block sequence, by the DFT definition:

        Fhat_w = sum_{k=0}^{Nt-1} F_k exp(-2 pi i w k / L),  w = 0..L/2,

    returned as complex128 [L//2 + 1, Nd, Nm].  Embedding the Toeplitz
    matrix in a block circulant of size L >= 2 Nt - 1 makes the DFT
    block-diagonalise it (section 4, "FFT-based GPU-accelerated p2o and p2q
    matvecs"); this is the block diagonal it produces.
    """
    F = np.asarray(F, dtype=np.float64)
    Nt = F.shape[0]
    w = np.arange(L // 2 + 1)[:, None]
    k = np.arange(Nt)[None, :]
    ph = (w * k) % L                      # exact integer phase index
    W = np.exp(-2j * np.pi * ph / L)      # [nbins, Nt]
    return np.tensordot(W, F, axes=(1, 0))


def rel_l2(y, y_ref) -> float:
    """||y - y_ref||_2 / ||y_ref||_2 in float64 over the whole array (all
    right-hand sides together; pass one right-hand side for a per-RHS error).
    With an all-zero reference it returns the absolute norm ||y||_2."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    den = np.linalg.norm(y_ref.ravel())
    num = np.linalg.norm((y - y_ref).ravel())
    return float(num / den) if den > 0 else float(num)
