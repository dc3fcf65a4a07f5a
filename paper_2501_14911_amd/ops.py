"""Python face of the p2o library: a plan bound to torch-owned device memory,
and autograd functions whose backward passes are the hand-written adjoint.

Every step of a matvec runs in libp2o's HIP kernels; this module only
allocates memory with torch, passes pointers and the current HIP stream,
and checks shapes and dtypes.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int64, c_size_t, c_void_p
from typing import Callable, Optional

import torch

from ._lib import (BATCHED, P2O_FP64, P2O_SRC_F32, P2O_SRC_F64, PRECISIONS, STAGES, check, lib)

SCALE_BLOCK = 4096


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else c_void_p(t.data_ptr())


class P2OOperator:
    """The block lower-triangular Toeplitz map F (Nd sensors, Nm parameters,
    Nt steps) held as its stored spectrum on one GPU.

    ``precision`` is the storage of the spectrum: "fp64", "fp32", "bf16" or
    "fp16" (the last two accumulate in FP32).  Series are float64 for fp64
    plans and float32 otherwise, shaped [nrhs, Nt, Nm] / [nrhs, Nt, Nd]
    (a leading nrhs may be omitted).
    """

    def __init__(self, Nd: int, Nm: int, Nt: int, precision: str = "bf16", max_rhs: int = 1,
                 device="cuda"):
        self.Nd, self.Nm, self.Nt = int(Nd), int(Nm), int(Nt)
        self.precision = precision
        self.max_rhs = int(max_rhs)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the p2o operator lives on a GPU (device 'cuda')")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        plan = c_void_p()
        check(lib.p2o_create(byref(plan), self.Nd, self.Nm, self.Nt, PRECISIONS[precision], self.max_rhs))
        self._plan = plan
        L, nf, pitch, nblk = c_int64(), c_int64(), c_int64(), c_int64()
        check(lib.p2o_get_layout(plan, byref(L), byref(nf), byref(pitch), byref(nblk)))
        self.L, self.nfreq, self.pitch, self.nblk = L.value, nf.value, pitch.value, nblk.value
        fb, wb = c_size_t(), c_size_t()
        check(lib.p2o_required_bytes(plan, byref(fb), byref(wb)))
        self.fhat_bytes, self.ws_bytes = fb.value, wb.value
        self.fhat = torch.empty(self.fhat_bytes, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        check(lib.p2o_bind_storage(plan, _ptr(self.fhat), self.fhat_bytes, _ptr(self.workspace), self.ws_bytes))
        self.ready = False
        self.qstride = 1

    # ------------------------------------------------------------------ plumbing
    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        check(lib.p2o_set_stream(self._plan, c_void_p(s.cuda_stream)))

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib.p2o_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def elem_bytes(self) -> int:
        return {"fp64": 16, "fp32": 8, "bf16": 4, "fp16": 4}[self.precision]

    def spectrum_view(self) -> torch.Tensor:
        """Raw stored spectrum bytes as [nfreq, Nd, pitch * elem_bytes] (read-only use)."""
        n = self.nfreq * self.Nd * self.pitch * self.elem_bytes
        return self.fhat[:n].view(self.nfreq, self.Nd, self.pitch * self.elem_bytes)

    def scales_view(self) -> torch.Tensor:
        """Per-(frequency, 4096-column block) dequantisation multipliers."""
        n = self.nfreq * self.Nd * self.pitch * self.elem_bytes
        off = (n + 255) // 256 * 256
        return self.fhat[off: off + 4 * self.nfreq * self.nblk].view(torch.float32).view(self.nfreq, self.nblk)

    def set_batched(self, mode: str = "auto"):
        """Per-frequency products for several right-hand sides: "auto",
        "gemv" (one streaming pass per right-hand side) or "mfma" (matrix
        cores, BF16 and FP16 spectra only)."""
        check(lib.p2o_set_option(self._plan, 0, BATCHED[mode]))

    def set_gemm_tile(self, tile: int = -1):
        """Force matrix-core tile variant ``tile`` (see ``gemm_tiles()``) for
        both directions, or -1 for the autotuned or built-in choice."""
        check(lib.p2o_set_option(self._plan, 1, int(tile)))

    def set_output_stride(self, r: int = 1):
        """Observe the data series every r-th step (multi-rate output of a p2q
        map): data series then have Nt / r steps, step i being parameter step
        r (i + 1) - 1."""
        check(lib.p2o_set_option(self._plan, 3, int(r)))
        self.qstride = int(r)

    @property
    def Ntd(self) -> int:
        """Steps of this operator's data series (Nt / output stride)."""
        return self.Nt // self.qstride

    def set_fixed_fft(self, on: bool = True):
        """Use the FFT kernels compiled for this plan's transform length when
        the library has them (default), or always the runtime-length ones."""
        check(lib.p2o_set_option(self._plan, 2, 1 if on else 0))

    def set_fp16_operands(self, on: bool = True):
        """Let F F^* calls of an FP16 plan keep their intermediate
        parameter-side spectra as scaled FP16 pairs where possible (default),
        or always as complex FP32."""
        check(lib.p2o_set_option(self._plan, 4, 1 if on else 0))
        self._fp16_operands = bool(on)

    @property
    def fp16_operands(self) -> bool:
        """The setting of set_fp16_operands (True unless switched off); the
        library applies it to FP16 plans whose products run on the matrix
        cores with a compiled transform length."""
        return self.precision == "fp16" and getattr(self, "_fp16_operands", True)

    def autotune(self, nrhs: int, reps: int = 3) -> dict:
        """Time every matrix-core tile variant for calls with ``nrhs``
        right-hand sides and keep the fastest (per direction) for later calls
        with exactly that many.  Overwrites the workspace; synchronises."""
        ft, at = ctypes.c_int32(), ctypes.c_int32()
        fm, am = ctypes.c_double(), ctypes.c_double()
        check(lib.p2o_autotune(self._plan, int(nrhs), int(reps), ctypes.byref(ft), ctypes.byref(at),
                               ctypes.byref(fm), ctypes.byref(am)))
        return {"fwd": (ft.value, fm.value), "adj": (at.value, am.value)}

    # ------------------------------------------------------------------ timing
    def profile(self, enable: bool = True):
        """Start (or stop) per-stage HIP-event timing; resets the totals."""
        check(lib.p2o_profile_enable(self._plan, 1 if enable else 0))

    def stage_times(self, nrhs: Optional[int] = None) -> dict:
        """{stage: (total_ms, launches)} since profiling was enabled, over all
        launches or those of calls with ``nrhs`` right-hand sides (synchronises)."""
        out = {}
        for name, sid in STAGES.items():
            ms, n = ctypes.c_double(), c_int64()
            if nrhs is None:
                check(lib.p2o_profile_read(self._plan, sid, byref(ms), byref(n)))
            else:
                check(lib.p2o_profile_read_nrhs(self._plan, sid, int(nrhs), byref(ms), byref(n)))
            out[name] = (ms.value, n.value)
        return out

    # ------------------------------------------------------------------ loading
    def load_blocks(self, F_chunk: torch.Tensor, col0: int = 0):
        """Transform and store F_k[:, col0:col0+ncols] given as [Nt, Nd, ncols]
        (float64 or float32, on this device)."""
        if F_chunk.device != self.device or F_chunk.dim() != 3:
            raise ValueError("F_chunk must be a [Nt, Nd, ncols] tensor on the operator's device")
        if F_chunk.shape[0] != self.Nt or F_chunk.shape[1] != self.Nd:
            raise ValueError(f"F_chunk shape {tuple(F_chunk.shape)} does not match Nt={self.Nt}, Nd={self.Nd}")
        if F_chunk.dtype not in (torch.float64, torch.float32):
            raise ValueError("F_chunk must be float64 or float32")
        F_chunk = F_chunk.contiguous()
        src = P2O_SRC_F64 if F_chunk.dtype == torch.float64 else P2O_SRC_F32
        self._stream()
        check(lib.p2o_load_blocks(self._plan, _ptr(F_chunk), int(col0), int(F_chunk.shape[2]), src))
        # keep the chunk alive until the stream has consumed it
        torch.cuda.current_stream(self.device).synchronize()

    def finalize(self):
        self._stream()
        check(lib.p2o_load_finalize(self._plan))
        self.ready = True

    def load(self, blocks: Callable[[int, int], torch.Tensor], chunk_cols: int = SCALE_BLOCK):
        """Load every column with ``blocks(col0, ncols) -> [Nt, Nd, ncols]``."""
        for c0 in range(0, self.Nm, chunk_cols):
            n = min(chunk_cols, self.Nm - c0)
            self.load_blocks(blocks(c0, n), c0)
        self.finalize()

    # ------------------------------------------------------------------ applies
    def _series(self, x: torch.Tensor, last: int, name: str, steps: Optional[int] = None):
        steps = self.Nt if steps is None else steps
        if x.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if x.dtype != self.dtype:
            raise ValueError(f"{name} must be {self.dtype} for a {self.precision} operator")
        squeeze = x.dim() == 2
        xb = x.unsqueeze(0) if squeeze else x
        if xb.dim() != 3 or xb.shape[1] != steps or xb.shape[2] != last:
            raise ValueError(f"{name} shape {tuple(x.shape)} must be [nrhs, {steps}, {last}]")
        return xb.contiguous(), squeeze

    def _nt(self, nt_active, nrhs: int):
        if nt_active is None:
            return None
        n = torch.as_tensor(nt_active, dtype=torch.int32, device=self.device).contiguous()
        if n.numel() != nrhs:
            raise ValueError("nt_active needs one length per right-hand side")
        return n

    def apply_F(self, m: torch.Tensor, nt_active=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """d = F m."""
        mb, sq = self._series(m, self.Nm, "m")
        nrhs = mb.shape[0]
        nt = self._nt(nt_active, nrhs)
        d = out if out is not None else torch.empty((nrhs, self.Ntd, self.Nd), dtype=self.dtype, device=self.device)
        self._stream()
        check(lib.p2o_apply_F(self._plan, _ptr(mb), _ptr(d), nrhs, _ptr(nt)))
        return d[0] if sq and out is None else d

    def apply_Ft(self, d: torch.Tensor, nt_active=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """m = F^* d."""
        db, sq = self._series(d, self.Nd, "d", self.Ntd)
        nrhs = db.shape[0]
        nt = self._nt(nt_active, nrhs)
        m = out if out is not None else torch.empty((nrhs, self.Nt, self.Nm), dtype=self.dtype, device=self.device)
        self._stream()
        check(lib.p2o_apply_Ft(self._plan, _ptr(db), _ptr(m), nrhs, _ptr(nt)))
        return m[0] if sq and out is None else m

    def apply_FFt(self, e: torch.Tensor, nt_active=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """h = F F^* e (data-space operator columns)."""
        eb, sq = self._series(e, self.Nd, "e", self.Ntd)
        nrhs = eb.shape[0]
        nt = self._nt(nt_active, nrhs)
        h = out if out is not None else torch.empty((nrhs, self.Ntd, self.Nd), dtype=self.dtype, device=self.device)
        self._stream()
        check(lib.p2o_apply_FFt(self._plan, _ptr(eb), _ptr(h), nrhs, _ptr(nt)))
        return h[0] if sq and out is None else h

    def misfit_grad(self, m: torch.Tensor, d_obs: torch.Tensor, noise_var, nt_active=None):
        """(Phi, grad): Phi = 1/2 (Fm - d_obs)^T Gamma^-1 (Fm - d_obs) per
        right-hand side (float64), grad = F^* Gamma^-1 (Fm - d_obs)."""
        mb, sq = self._series(m, self.Nm, "m")
        db, _ = self._series(d_obs, self.Nd, "d_obs")
        nrhs = mb.shape[0]
        if db.shape[0] != nrhs:
            raise ValueError("m and d_obs need the same number of right-hand sides")
        var = torch.as_tensor(noise_var, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        nt = self._nt(nt_active, nrhs)
        grad = torch.empty_like(mb)
        phi = torch.empty(nrhs, dtype=torch.float64, device=self.device)
        self._stream()
        check(lib.p2o_misfit_grad(self._plan, _ptr(mb), _ptr(db), _ptr(var), var.numel(), _ptr(grad), _ptr(phi),
                                  nrhs, _ptr(nt)))
        if sq:
            return phi[0], grad[0]
        return phi, grad


    # ------------------------------------------------------------------ offline / online phases
    def data_dim(self) -> int:
        """N = Nt * Nd, the data-space dimension."""
        return self.Nt * self.Nd

    def assemble_K(self, noise_var, prior_var: float = 1.0, K: Optional[torch.Tensor] = None,
                   batch: Optional[int] = None, columns: Optional[tuple] = None) -> torch.Tensor:
        """K = Gamma_noise + prior_var F F^* as a dense FP64 [N, N] tensor
        (row j of the tensor is column j of K; K is symmetric), assembled in
        batches of ``batch`` (default max_rhs) columns; ``columns`` = (j0, n)
        assembles only columns j0 .. j0 + n - 1 (the rest of K is left as it
        is)."""
        N = self.data_dim()
        if K is None:
            K = torch.empty((N, N), dtype=torch.float64, device=self.device)
        if K.dtype != torch.float64 or K.device != self.device or K.dim() != 2 or K.shape[1] != N or K.shape[0] != N \
                or K.stride(1) != 1:
            raise ValueError(f"K must be a contiguous float64 [{N}, {N}] tensor on {self.device}")
        var = torch.as_tensor(noise_var, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        b = int(batch or self.max_rhs)
        c0, nc = (0, N) if columns is None else (int(columns[0]), int(columns[1]))
        if c0 < 0 or nc < 0 or c0 + nc > N:
            raise ValueError(f"columns ({c0}, {nc}) outside [0, {N})")
        self._stream()
        for j0 in range(c0, c0 + nc, b):
            check(lib.p2o_assemble_K(self._plan, float(prior_var), _ptr(var), var.numel(), _ptr(K), K.stride(0), j0,
                                     min(b, c0 + nc - j0)))
        return K

    def map_point(self, d_obs: torch.Tensor, L: torch.Tensor, noise_var, prior_var: float = 1.0) -> torch.Tensor:
        """MAP point m_map = (I - G^* K^{-1} F) G^* Gamma_noise^{-1} d_obs,
        G^* = prior_var F^*, from K's Cholesky factor L (``cholesky``)."""
        db, sq = self._series(d_obs, self.Nd, "d_obs")
        nrhs = db.shape[0]
        _check_factor(L, self.data_dim(), self.device)
        var = torch.as_tensor(noise_var, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        m = torch.empty((nrhs, self.Nt, self.Nm), dtype=self.dtype, device=self.device)
        self._stream()
        check(lib.p2o_map_point(self._plan, float(prior_var), _ptr(var), var.numel(), _ptr(L), L.stride(0), _ptr(db),
                                _ptr(m), nrhs))
        return m[0] if sq else m

    def posterior_cov_apply(self, v: torch.Tensor, L: torch.Tensor, prior_var: float = 1.0) -> torch.Tensor:
        """Gamma_post v = (I - G^* K^{-1} F) Gamma_prior v with Gamma_prior =
        prior_var I, from K's Cholesky factor L."""
        vb, sq = self._series(v, self.Nm, "v")
        nrhs = vb.shape[0]
        _check_factor(L, self.data_dim(), self.device)
        out = torch.empty_like(vb)
        self._stream()
        check(lib.p2o_posterior_cov_apply(self._plan, float(prior_var), _ptr(L), L.stride(0), _ptr(vb), _ptr(out), nrhs))
        return out[0] if sq else out


    def apply_FGt(self, G: "P2OOperator", e: torch.Tensor) -> torch.Tensor:
        """h = F G^* e for a second operator G on the same parameter grid
        (e: G's data series, h: this operator's)."""
        eb, sq = G._series(e, G.Nd, "e", G.Ntd)
        nrhs = eb.shape[0]
        h = torch.empty((nrhs, self.Ntd, self.Nd), dtype=self.dtype, device=self.device)
        self._stream()
        G._stream()
        check(lib.p2o_apply_FGt(self._plan, G._plan, _ptr(eb), _ptr(h), nrhs))
        return h[0] if sq else h

    def d2q_map(self, Fq: "P2OOperator", L: torch.Tensor, noise_var, prior_var: float = 1.0,
                batch: Optional[int] = None) -> torch.Tensor:
        """Data-to-QoI map Q = F_q (I - G^* K^{-1} F) G^* Gamma_noise^{-1}
        (G^* = prior_var F^*) as a dense FP64 [Nq Ntq, N] tensor (row r =
        row r of Q), assembled ``batch`` rows per call."""
        N = self.data_dim()
        nq = Fq.Ntd * Fq.Nd
        _check_factor(L, N, self.device)
        var = torch.as_tensor(noise_var, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        Q = torch.empty((nq, N), dtype=torch.float64, device=self.device)
        b = int(batch or min(self.max_rhs, Fq.max_rhs))
        self._stream()
        Fq._stream()
        for r0 in range(0, nq, b):
            check(lib.p2o_d2q_rows(self._plan, Fq._plan, float(prior_var), _ptr(var), var.numel(), _ptr(L), L.stride(0),
                                   r0, min(b, nq - r0), _ptr(Q), Q.stride(0)))
        return Q

    def qoi_posterior_cov(self, Fq: "P2OOperator", L: torch.Tensor, prior_var: float = 1.0,
                          batch: Optional[int] = None) -> torch.Tensor:
        """Gamma_post(q) = F_q (I - G^* K^{-1} F) G_q^* as a dense FP64
        [Nq Ntq, Nq Ntq] tensor (tensor row c = column c; the matrix is
        symmetric)."""
        N = self.data_dim()
        nq = Fq.Ntd * Fq.Nd
        _check_factor(L, N, self.device)
        C = torch.empty((nq, nq), dtype=torch.float64, device=self.device)
        b = int(batch or min(self.max_rhs, Fq.max_rhs))
        self._stream()
        Fq._stream()
        for c0 in range(0, nq, b):
            check(lib.p2o_qoi_posterior_cov(self._plan, Fq._plan, float(prior_var), _ptr(L), L.stride(0), c0,
                                            min(b, nq - c0), _ptr(C), C.stride(0)))
        return C


def d2q_apply(Q: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """q = Q d for data vectors d ([N] or [nrhs, N], float64), the online QoI
    prediction."""
    if Q.dtype != torch.float64 or Q.dim() != 2 or Q.stride(1) != 1:
        raise ValueError("Q must be a float64 [nq, N] tensor with unit column stride")
    nq, N = Q.shape
    db = d.reshape(-1, N).to(torch.float64).contiguous()
    q = torch.empty((db.shape[0], nq), dtype=torch.float64, device=Q.device)
    check(lib.p2o_d2q_apply(_ptr(Q), nq, N, Q.stride(0), _ptr(db), _ptr(q), db.shape[0],
                            c_void_p(torch.cuda.current_stream(Q.device).cuda_stream)))
    return q[0] if d.dim() == 1 else q


def _check_factor(L: torch.Tensor, N: int, device):
    if L.dtype != torch.float64 or L.device != device or L.dim() != 2 or tuple(L.shape) != (N, N) or L.stride(1) != 1:
        raise ValueError(f"L must be a contiguous float64 [{N}, {N}] tensor on {device}")


def assemble_K_from_blocks(blocks: Callable[[int, int], torch.Tensor], Nd: int, Nm: int, Nt: int, noise_var,
                           prior_var: float = 1.0, K: Optional[torch.Tensor] = None, chunk_cols: int = 2048,
                           device="cuda") -> torch.Tensor:
    """K = Gamma_noise + prior_var F F^* (dense FP64 [N, N], N = Nt Nd, row j
    of the tensor = column j of K) from the blocks themselves:
    ``blocks(c0, n)`` returns F_k[:, c0:c0+n] for all k as a [Nt, Nd, n]
    tensor on the device (as for P2OOperator.load).  The Gram matrix of the
    stacked blocks is accumulated chunk by chunk on the FP64 matrix cores and
    turned into K by prefix sums along its block diagonals (no spectrum, no
    FFT: exact up to FP64 rounding)."""
    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    N = Nt * Nd
    if K is None:
        K = torch.empty((N, N), dtype=torch.float64, device=dev)
    if K.dtype != torch.float64 or K.device != dev or K.dim() != 2 or K.shape[0] != N or K.shape[1] != N \
            or K.stride(1) != 1:
        raise ValueError(f"K must be a contiguous float64 [{N}, {N}] tensor on {dev}")
    var = torch.as_tensor(noise_var, dtype=torch.float64, device=dev).reshape(-1).contiguous()
    stream = c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    K.zero_()
    for c0 in range(0, Nm, chunk_cols):
        n = min(chunk_cols, Nm - c0)
        B = blocks(c0, n)
        if tuple(B.shape) != (Nt, Nd, n) or B.device != dev:
            raise ValueError(f"blocks({c0}, {n}) must be a [{Nt}, {Nd}, {n}] tensor on {dev}")
        B = B.to(torch.float64).contiguous()
        check(lib.p2o_gram_accumulate(_ptr(B), Nt, Nd, n, n, _ptr(K), K.stride(0), stream))
        del B
    check(lib.p2o_gram_to_K(_ptr(K), K.stride(0), Nt, Nd, float(prior_var), _ptr(var), var.numel(), stream))
    return K


def cholesky(K: torch.Tensor) -> torch.Tensor:
    """In-place Cholesky factorisation of the symmetric positive definite FP64
    [N, N] tensor K (row j = column j of K): on return its entries (j, i) with
    i >= j, i.e. the lower triangle of the column-major matrix, hold L with
    K = L L^T, and the strict upper triangle holds L^T (read by the backward
    solve).  Raises when a pivot is not positive."""
    if K.dtype != torch.float64 or K.dim() != 2 or K.shape[0] != K.shape[1] or K.stride(1) != 1:
        raise ValueError("K must be a square float64 tensor with unit column stride")
    info = torch.zeros(1, dtype=torch.int32, device=K.device)
    check(lib.p2o_cholesky(_ptr(K), K.shape[0], K.stride(0), _ptr(info),
                           c_void_p(torch.cuda.current_stream(K.device).cuda_stream)))
    bad = int(info.item())
    if bad:
        raise ValueError(f"K is not positive definite (pivot {bad - 1} not positive)")
    return K


def cholesky_solve(L: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """X <- K^{-1} X in place for X of shape [nrhs, N] (each row one
    right-hand side), from the factor as ``cholesky`` leaves it (both
    triangles are read)."""
    N = L.shape[0]
    _check_factor(L, N, L.device)
    if X.dtype != torch.float64 or X.dim() != 2 or X.shape[1] != N or X.stride(1) != 1:
        raise ValueError(f"X must be a float64 [nrhs, {N}] tensor with unit column stride")
    check(lib.p2o_cholesky_solve(_ptr(L), N, L.stride(0), _ptr(X), X.shape[0], X.stride(0),
                                 c_void_p(torch.cuda.current_stream(L.device).cuda_stream)))
    return X


# ---------------------------------------------------------------------- autograd
class P2O(torch.autograd.Function):
    """d = F m with backward m_bar = F^* d_bar (the hand-written adjoint)."""

    @staticmethod
    def forward(ctx, m, op: P2OOperator, nt_active=None):
        ctx.op = op
        ctx.nt_active = nt_active
        return op.apply_F(m, nt_active)

    @staticmethod
    def backward(ctx, g):
        return P2OT.apply(g.contiguous(), ctx.op, ctx.nt_active), None, None


class P2OT(torch.autograd.Function):
    """m = F^* d with backward d_bar = F m_bar."""

    @staticmethod
    def forward(ctx, d, op: P2OOperator, nt_active=None):
        ctx.op = op
        ctx.nt_active = nt_active
        return op.apply_Ft(d, nt_active)

    @staticmethod
    def backward(ctx, g):
        return P2O.apply(g.contiguous(), ctx.op, ctx.nt_active), None, None


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, op: P2OOperator, d_obs, noise_var, nt_active):
        phi, grad = op.misfit_grad(m, d_obs, noise_var, nt_active)
        ctx.save_for_backward(grad)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        (grad,) = ctx.saved_tensors
        if grad.dim() == 2:
            return (gphi.to(grad.dtype) * grad), None, None, None, None
        return gphi.to(grad.dtype)[:, None, None] * grad, None, None, None, None


def misfit(m: torch.Tensor, op: P2OOperator, d_obs: torch.Tensor, noise_var, nt_active=None) -> torch.Tensor:
    """Phi(m) = 1/2 ||F m - d_obs||^2_{Gamma_noise^-1} (float64, per right-hand
    side) with the fused gradient kernel as its backward."""
    return _Misfit.apply(m, op, d_obs, noise_var, nt_active)


def gemm_tiles() -> list:
    """Matrix-core tile variants: [(row_groups, substeps, blocks, rhs_per_group), ...]
    (32 * row_groups * blocks output rows per workgroup)."""
    out = []
    while True:
        rg, ku, mb, nr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        if lib.p2o_gemm_tile_info(len(out), ctypes.byref(rg), ctypes.byref(ku), ctypes.byref(mb),
                                  ctypes.byref(nr)) != 0:
            return out
        out.append((rg.value, ku.value, mb.value, nr.value))


def bandwidth_probe(nbytes: int = 8 << 30, reps: int = 10, device="cuda", blocks: int = 8192) -> dict:
    """Measured streaming read and copy bandwidth (GB/s) of the device, with
    the library's probe kernels, for roofline context."""
    dev = torch.device(device)
    nbytes = nbytes // 2048 * 2048                 # the read probe moves whole 2 KB chunks
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    sink = torch.empty(blocks, dtype=torch.int32, device=dev)
    half = nbytes // 2 // 32 * 32
    dst = torch.empty(half, dtype=torch.uint8, device=dev)
    s = c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    out = {}
    for mode, name, nb, moved in ((0, "read", nbytes, nbytes), (1, "copy", half, 2 * half)):
        d = sink if mode == 0 else dst
        src_p = src if mode == 0 else src[:half]
        check(lib.p2o_bandwidth_probe(mode, _ptr(src_p), _ptr(d), nb, blocks, s))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            check(lib.p2o_bandwidth_probe(mode, _ptr(src_p), _ptr(d), nb, blocks, s))
        b.record()
        torch.cuda.synchronize(dev)
        ms = a.elapsed_time(b) / reps
        out[name + "_GBs"] = moved / (ms * 1e-3) / 1e9
        out[name + "_bytes"] = moved
    del src, dst, sink
    torch.cuda.empty_cache()
    return out
