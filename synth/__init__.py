"""Seeded synthetic inputs for the block lower-triangular Toeplitz p2o operator.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It holds none of the method's arithmetic: it only draws numbers.

Every random value is a pure function of (seed, stream tag, index triple), so
any sub-block of an operand (a few rows of every F_k, one column chunk, one
right-hand side) can be regenerated on its own, on the CPU with numpy or on a
GPU with torch, without materialising the rest.

Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed, counter
(a >> 1, b, c, tag).  Two 53-bit uniforms from the four output words feed a
Box-Muller transform; index ``a`` picks the cosine (even) or sine (odd)
branch, so neighbouring ``a`` share one Philox call.

The integer stream is bit-identical on every backend.  The Box-Muller step
uses the backend's log/sqrt/cos/sin, so values drawn with torch on a GPU may
differ from numpy's in the last bit or two; tests that need bit-identical
inputs on both sides draw them with numpy and copy them to the device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK32 = 0xFFFFFFFF

# stream tags (fourth counter word)
TAG_F = 1        # operator blocks F_k
TAG_M = 2        # parameter series m
TAG_D = 3        # data series d / d_obs
TAG_NOISE = 4    # observation noise

SEED = 14911     # base seed; F uses SEED, m SEED+1, d/noise SEED+2, ...

SCALE_BLOCK = 4096   # column-block width of the generator (and the loader)


# ---------------------------------------------------------------------------
# Philox4x32-10, written once for numpy (uint64 lanes) and torch (int64 lanes)
# ---------------------------------------------------------------------------
def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds on arrays of 32-bit words held in 64-bit lanes.

    Works on numpy uint64 arrays or torch int64 tensors (products of two
    32-bit words wrap modulo 2**64 in torch's signed lanes; only their low
    64 bits are used, then masked).  Returns four word arrays.
    """
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK32
            k1 = (k1 + _W1) & _MASK32
        p0 = c0 * _M0
        p1 = c2 * _M1
        hi0 = (p0 >> 32) & _MASK32
        lo0 = p0 & _MASK32
        hi1 = (p1 >> 32) & _MASK32
        lo1 = p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _as_words(v, like):
    """Broadcastable 64-bit-lane array of a (non-negative) index."""
    if _is_torch(like):
        import torch
        return torch.as_tensor(v, dtype=torch.int64, device=like.device)
    return np.asarray(v, dtype=np.uint64)


def normal(seed: int, tag: int, a, b, c, backend: str = "numpy", device=None):
    """Standard normals z(seed, tag, a, b, c), broadcast over index arrays.

    ``a`` < 2**33, ``b``, ``c`` < 2**32.  ``backend`` is ``"numpy"`` (float64
    ndarray) or ``"torch"`` (float64 tensor on ``device``).
    """
    k0 = seed & _MASK32
    k1 = (seed >> 32) & _MASK32
    if backend == "torch":
        import torch
        dev = torch.device(device) if device is not None else torch.device("cpu")
        a = torch.as_tensor(a, dtype=torch.int64, device=dev)
        b = torch.as_tensor(b, dtype=torch.int64, device=dev)
        c = torch.as_tensor(c, dtype=torch.int64, device=dev)
        a, b, c = torch.broadcast_tensors(a, b, c)
        x0, x1, x2, x3 = philox4x32_10(a >> 1, b.clone(), c.clone(),
                                       torch.full_like(a, tag), k0, k1)
        u1 = 1.0 - ((x0 >> 5).double() * 67108864.0 + (x1 >> 6).double()) * 2.0 ** -53
        u2 = ((x2 >> 5).double() * 67108864.0 + (x3 >> 6).double()) * 2.0 ** -53
        r = torch.sqrt(-2.0 * torch.log(u1))
        th = (2.0 * math.pi) * u2
        return torch.where((a & 1) == 0, r * torch.cos(th), r * torch.sin(th))
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    c = np.asarray(c, dtype=np.uint64)
    a, b, c = np.broadcast_arrays(a, b, c)
    x0, x1, x2, x3 = philox4x32_10(a >> np.uint64(1), b.copy(), c.copy(),
                                   np.full(a.shape, tag, dtype=np.uint64), k0, k1)
    u1 = 1.0 - ((x0 >> np.uint64(5)).astype(np.float64) * 67108864.0
                + (x1 >> np.uint64(6)).astype(np.float64)) * 2.0 ** -53
    u2 = ((x2 >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (x3 >> np.uint64(6)).astype(np.float64)) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    th = (2.0 * math.pi) * u2
    return np.where((a & np.uint64(1)) == 0, r * np.cos(th), r * np.sin(th))


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    """Shape and input recipe of one synthetic problem.

    F_k[i, j] = exp(-k / tau) * z_F(j, i, k) / sqrt(Nm) * mod(i, j), with
    mod = 1 + cos(2*pi*(j/Nm + i/Nd)) / 2 when ``cosine_mod`` else 1.
    """
    name: str
    Nd: int
    Nm: int
    Nt: int
    tau: float
    cosine_mod: bool = False
    sigma: float = 1e-2
    grid: Optional[int] = None          # Nm = grid**2 when set (spatial smoothing)
    seed: int = SEED

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


CONFIGS = {
    # 4 sensors x 64 parameters x 16 steps, FP64
    "tiny": Workload("tiny", Nd=4, Nm=64, Nt=16, tau=4.0),
    # 64 x 4096 (64^2) x 128 steps, cosine spatial modulation, sigma = 1e-2
    "medium": Workload("medium", Nd=64, Nm=4096, Nt=128, tau=32.0, cosine_mod=True, grid=64),
    # 600 x 16384 (128^2) x 420 steps (FFT length 840)
    "paper_time": Workload("paper_time", Nd=600, Nm=16384, Nt=420, tau=100.0, grid=128),
    # 600 x 65536 (256^2) x 420 steps: one GPU's column share
    "largest": Workload("largest", Nd=600, Nm=65536, Nt=420, tau=100.0, grid=256),
    # the paper's numerical example's dimensions (section 5): 49 sensors, a 513^2 parameter grid,
    # 500 steps, and its p2q map with 16 QoIs (observed every 10th step: 50 QoI steps)
    "paper_grid": Workload("paper_grid", Nd=49, Nm=513 * 513, Nt=500, tau=100.0, grid=513),
    "paper_grid_qoi": Workload("paper_grid_qoi", Nd=16, Nm=513 * 513, Nt=500, tau=100.0, grid=513, seed=SEED + 50),
}


def _mod_factor(w: Workload, rows, cols, xp):
    if not w.cosine_mod:
        return 1.0
    ang = 2.0 * math.pi * (cols[None, :] / w.Nm + rows[:, None] / w.Nd)
    return 1.0 + 0.5 * xp.cos(ang)


def operator_rows_cols(w: Workload, ks: Sequence[int], rows=None, cols=None,
                       backend: str = "numpy", device=None):
    """F_k[rows][:, cols] for each k in ``ks`` as a float64 array [len(ks), R, C]."""
    if backend == "torch":
        import torch
        dev = torch.device(device) if device is not None else torch.device("cpu")
        rows_t = torch.arange(w.Nd, device=dev) if rows is None else torch.as_tensor(rows, device=dev)
        cols_t = torch.arange(w.Nm, device=dev) if cols is None else torch.as_tensor(cols, device=dev)
        ks_t = torch.as_tensor(list(ks), dtype=torch.int64, device=dev)
        z = normal(w.seed, TAG_F, cols_t[None, None, :], rows_t[None, :, None],
                   ks_t[:, None, None], backend="torch", device=dev)
        decay = torch.exp(-ks_t.double() / w.tau)[:, None, None]
        out = z * decay / math.sqrt(w.Nm)
        if w.cosine_mod:
            out = out * _mod_factor(w, rows_t.double(), cols_t.double(), torch)[None]
        return out
    rows_a = np.arange(w.Nd) if rows is None else np.asarray(rows)
    cols_a = np.arange(w.Nm) if cols is None else np.asarray(cols)
    ks_a = np.asarray(list(ks), dtype=np.int64)
    z = normal(w.seed, TAG_F, cols_a[None, None, :], rows_a[None, :, None], ks_a[:, None, None])
    decay = np.exp(-ks_a.astype(np.float64) / w.tau)[:, None, None]
    out = z * decay / math.sqrt(w.Nm)
    if w.cosine_mod:
        out = out * _mod_factor(w, rows_a.astype(np.float64), cols_a.astype(np.float64), np)[None]
    return out


def operator_blocks(w: Workload, rows=None, cols=None, backend="numpy", device=None):
    """All time-domain blocks F_k, k = 0..Nt-1, as [Nt, Nd', Nm'] float64."""
    return operator_rows_cols(w, range(w.Nt), rows, cols, backend, device)


def param_series(w: Workload, nrhs: int = 1, seed_offset: int = 1, backend="numpy", device=None,
                 smooth: bool = False):
    """m[b][t][j] ~ N(0, 1), [nrhs, Nt, Nm] float64; optional 3x3 spatial box mean."""
    if backend == "torch":
        import torch
        dev = torch.device(device) if device is not None else torch.device("cpu")
        j = torch.arange(w.Nm, device=dev)[None, None, :]
        t = torch.arange(w.Nt, device=dev)[None, :, None]
        b = torch.arange(nrhs, device=dev)[:, None, None]
        m = normal(w.seed + seed_offset, TAG_M, j, t, b, backend="torch", device=dev)
    else:
        m = normal(w.seed + seed_offset, TAG_M, np.arange(w.Nm)[None, None, :],
                   np.arange(w.Nt)[None, :, None], np.arange(nrhs)[:, None, None])
    if smooth:
        m = box_smooth(w, m)
    return m


def box_smooth(w: Workload, m):
    """3x3 mean over in-grid neighbours of each point on the grid x grid
    parameter mesh (row-major index j = grid*y + x), per time step."""
    g = w.grid
    assert g is not None and g * g == w.Nm
    if _is_torch(m):
        import torch
        x = m.reshape(*m.shape[:-1], g, g)
        s = torch.zeros_like(x)
        n = torch.zeros((g, g), dtype=x.dtype, device=x.device)
        one = torch.ones((g, g), dtype=x.dtype, device=x.device)
    else:
        x = m.reshape(*m.shape[:-1], g, g)
        s = np.zeros_like(x)
        n = np.zeros((g, g))
        one = np.ones((g, g))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ys = slice(max(dy, 0), g + min(dy, 0))
            yd = slice(max(-dy, 0), g + min(-dy, 0))
            xs = slice(max(dx, 0), g + min(dx, 0))
            xd = slice(max(-dx, 0), g + min(-dx, 0))
            s[..., yd, xd] += x[..., ys, xs]
            n[yd, xd] += one[ys, xs]
    return (s / n).reshape(m.shape)


def data_series(w: Workload, nrhs: int = 1, tag: int = TAG_D, backend="numpy", device=None):
    """d[b][t][i] ~ N(0, 1), [nrhs, Nt, Nd] float64."""
    if backend == "torch":
        import torch
        dev = torch.device(device) if device is not None else torch.device("cpu")
        return normal(w.seed + 2, tag, torch.arange(w.Nd, device=dev)[None, None, :],
                      torch.arange(w.Nt, device=dev)[None, :, None],
                      torch.arange(nrhs, device=dev)[:, None, None], backend="torch", device=dev)
    return normal(w.seed + 2, tag, np.arange(w.Nd)[None, None, :],
                  np.arange(w.Nt)[None, :, None], np.arange(nrhs)[:, None, None])


def noise(w: Workload, nrhs: int = 1, backend="numpy", device=None):
    """sigma * eps, eps ~ N(0, 1), [nrhs, Nt, Nd] float64."""
    return w.sigma * data_series(w, nrhs, tag=TAG_NOISE, backend=backend, device=device)


def hessian_column_indices(w: Workload, count: int = 64):
    """``count`` distinct data-space indices j = t*Nd + s, drawn with seed+3;
    the first is at t = 0 and the second at t = Nt-1."""
    rng = np.random.default_rng(w.seed + 3)
    n = w.Nd * w.Nt
    count = min(count, n)
    first = int(rng.integers(0, w.Nd))
    last = (w.Nt - 1) * w.Nd + int(rng.integers(0, w.Nd))
    picked = [first] if first == last else [first, last]
    rest = rng.permutation(n)
    for j in rest:
        if len(picked) >= count:
            break
        if int(j) not in picked:
            picked.append(int(j))
    return np.asarray(picked[:count], dtype=np.int64)


def unit_data_vectors(w: Workload, idx) -> np.ndarray:
    """e_j for each j in ``idx`` as [len(idx), Nt, Nd] float64."""
    e = np.zeros((len(idx), w.Nt * w.Nd))
    e[np.arange(len(idx)), np.asarray(idx)] = 1.0
    return e.reshape(len(idx), w.Nt, w.Nd)


def ragged_lengths(w: Workload, count: int = 32, lo: int = 64):
    """Active lengths N_t^(b) ~ U{lo..Nt}, drawn with seed+4, as int32."""
    rng = np.random.default_rng(w.seed + 4)
    lo = min(lo, w.Nt)
    return rng.integers(lo, w.Nt + 1, size=count).astype(np.int32)
