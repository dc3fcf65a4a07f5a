"""Benchmark of the FFT-based block-Toeplitz p2o path on one MI355X.

Workload: Nd = 600 sensors, Nm = 16384 parameters per step, Nt = 420 steps
(circulant length 840), BF16 spectrum with FP32 accumulation, synthetic
blocks F_k = exp(-k/100) N(0,1)/sqrt(Nm).

One step is one pass over every use of the hot path:
  1. a data-misfit gradient on one right-hand side (r2c FFT of m, streaming
     forward products, inverse FFT fused with the residual and the FP64
     misfit reduction, r2c, streaming adjoint products, inverse FFT):
     one F and one F^* matvec;
  2. 64 data-space operator columns h_j = F F^* e_j in one call (batched
     adjoint and forward products on the matrix cores, truncate-and-repad
     between them): 128 matvecs;
  3. F and F^* on 32 right-hand sides whose active lengths are drawn from
     U{64..420} (batched, ragged): 64 matvecs.
``value`` = matvecs per second over the step (194 per step).  The plain FP64
single-right-hand-side path on an FP64 spectrum of the same operator is timed
beside it for the batched-mixed-precision speedup.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build targets one
GPU (the operator's column share on that GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0
N_HESS = 64
N_RAGGED = 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper_time")
    ap.add_argument("--cpu-sample-cols", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-call-stats", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_blocks(w, c0, n, dev, torch, synth, lag_batch=35):
    """F_k[:, c0:c0+n] for all k as float64 [Nt, Nd, n], drawn on the GPU."""
    out = torch.empty((w.Nt, w.Nd, n), dtype=torch.float64, device=dev)
    cols = torch.arange(c0, c0 + n, device=dev)
    for k0 in range(0, w.Nt, lag_batch):
        ks = list(range(k0, min(w.Nt, k0 + lag_batch)))
        out[k0:k0 + len(ks)] = synth.operator_rows_cols(w, ks, cols=cols, backend="torch", device=dev)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU column sharding "
              "is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2501_14911_amd import P2OOperator

    w = synth.CONFIGS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] workload {w.name}: Nd={w.Nd} Nm={w.Nm} Nt={w.Nt}")

    op = P2OOperator(w.Nd, w.Nm, w.Nt, "bf16", max_rhs=N_HESS, device=dev)
    t0 = time.perf_counter()
    op.profile(True)
    op.load(lambda c0, n: gpu_blocks(w, c0, n, dev, torch, synth))
    load_ms = op.stage_times()["load"][0]
    op.profile(False)
    log(f"[bench] BF16 spectrum loaded ({op.fhat_bytes / 1e9:.2f} GB) in {time.perf_counter() - t0:.1f} s "
        f"(load kernels {load_ms:.1f} ms)")

    # matrix-core tile variants for the two batched widths (autotuner, before timing)
    from paper_2501_14911_amd import gemm_tiles
    tiles = gemm_tiles()
    tuned = {}
    for nr in (N_HESS, N_RAGGED):
        r = op.autotune(nr, reps=2)
        tuned[nr] = {d: {"tile": r[d][0], "shape": tiles[r[d][0]], "ms": r[d][1]} for d in ("fwd", "adj")}
        log(f"[bench] autotune nrhs={nr}: fwd tile {r['fwd'][0]} {tiles[r['fwd'][0]]} {r['fwd'][1]:.3f} ms, "
            f"adj tile {r['adj'][0]} {tiles[r['adj'][0]]} {r['adj'][1]:.3f} ms")

    # inputs
    m = synth.param_series(w, 1, backend="torch", device=dev, smooth=(w.name == "largest"))[0].float()
    d_obs = synth.data_series(w, 1, backend="torch", device=dev)[0].float()
    var = torch.tensor([w.sigma ** 2], dtype=torch.float64, device=dev)
    hidx = synth.hessian_column_indices(w, N_HESS)
    E = torch.from_numpy(synth.unit_data_vectors(w, hidx)).to(dev, torch.float32)
    nt_r = synth.ragged_lengths(w, N_RAGGED)
    nt_r_dev = torch.from_numpy(nt_r).to(dev)
    m_r = synth.param_series(w, N_RAGGED, seed_offset=21, backend="torch", device=dev).float()
    d_r = synth.data_series(w, N_RAGGED, tag=synth.TAG_D + 16, backend="torch", device=dev).float()
    H = torch.empty((N_HESS, w.Nt, w.Nd), dtype=torch.float32, device=dev)
    Y_r = torch.empty((N_RAGGED, w.Nt, w.Nd), dtype=torch.float32, device=dev)
    S_r = torch.empty((N_RAGGED, w.Nt, w.Nm), dtype=torch.float32, device=dev)

    def step(evs=None):
        if evs:
            evs[0].record()
        op.misfit_grad(m, d_obs, var)
        if evs:
            evs[1].record()
        op.apply_FFt(E, out=H)
        if evs:
            evs[2].record()
        op.apply_F(m_r, nt_active=nt_r_dev, out=Y_r)
        op.apply_Ft(d_r, nt_active=nt_r_dev, out=S_r)
        if evs:
            evs[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    op.profile(True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        step(evs[k])
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    part_ms = [sum(e[i].elapsed_time(e[i + 1]) for e in evs) / args.steps for i in range(3)]
    stages = op.stage_times()
    st1, st64, st32 = op.stage_times(1), op.stage_times(N_HESS), op.stage_times(N_RAGGED)
    op.profile(False)
    matvecs = 2 + 2 * N_HESS + 2 * N_RAGGED
    log(f"[bench] {ms_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}): single-RHS gradient "
        f"{part_ms[0]:.3f} ms, 64 F F* columns {part_ms[1]:.3f} ms, 32 ragged F + F* {part_ms[2]:.3f} ms")
    for nr, st in ((1, st1), (N_HESS, st64), (N_RAGGED, st32)):
        for k, (tot, n) in st.items():
            if n:
                log(f"[bench]   nrhs={nr:2d} {k:9s} {tot / n * 1e3:9.1f} us x {n / args.steps:.0f}/step")

    # roofline bookkeeping (algorithmic bytes: spectrum once + series spectra in/out)
    spec_bytes = op.nfreq * w.Nd * w.Nm * op.elem_bytes

    def avg_us(k, st=stages):
        tot, n = st[k]
        return tot / n * 1e3 if n else 0.0

    def vec_bytes(nrhs):
        return op.nfreq * nrhs * (w.Nm + w.Nd) * 8

    def gemm_flop(nrhs):        # real-equivalent flops of one BF16 pass (x2 issued for the hi+lo split)
        return 2.0 * op.nfreq * w.Nd * (2 * w.Nm) * (2 * nrhs)

    kern = {
        "gemv_fwd": {"us": avg_us("gemv_fwd", st1), "bytes": spec_bytes + vec_bytes(1), "nrhs": 1},
        "gemv_adj": {"us": avg_us("gemv_adj", st1), "bytes": spec_bytes + vec_bytes(1), "nrhs": 1},
        "gemm_fwd_64": {"us": avg_us("gemm_fwd", st64), "bytes": spec_bytes + vec_bytes(N_HESS),
                        "flop": gemm_flop(N_HESS), "nrhs": N_HESS},
        "gemm_adj_64": {"us": avg_us("gemm_adj", st64), "bytes": spec_bytes + vec_bytes(N_HESS),
                        "flop": gemm_flop(N_HESS), "nrhs": N_HESS},
        "gemm_fwd_32": {"us": avg_us("gemm_fwd", st32), "bytes": spec_bytes + vec_bytes(N_RAGGED),
                        "flop": gemm_flop(N_RAGGED), "nrhs": N_RAGGED},
        "gemm_adj_32": {"us": avg_us("gemm_adj", st32), "bytes": spec_bytes + vec_bytes(N_RAGGED),
                        "flop": gemm_flop(N_RAGGED), "nrhs": N_RAGGED},
    }
    for k, v in kern.items():
        v["GBs"] = v["bytes"] / (v["us"] * 1e-6) / 1e9 if v["us"] else 0.0
        if "flop" in v and v["us"]:
            v["TFLOPs_issued"] = 2 * v["flop"] / (v["us"] * 1e-6) / 1e12
    # dominant kernel: largest share of the step
    share = {"gemv_fwd": st1["gemv_fwd"][0], "gemv_adj": st1["gemv_adj"][0],
             "gemm_fwd_64": st64["gemm_fwd"][0], "gemm_adj_64": st64["gemm_adj"][0],
             "gemm_fwd_32": st32["gemm_fwd"][0], "gemm_adj_32": st32["gemm_adj"][0]}
    dom = max(share, key=share.get)
    dk = kern[dom]
    dom_tile = None
    if dom.startswith("gemm_"):
        dom_tile = tuned[int(dom.rsplit("_", 1)[1])][dom.split("_")[1]]["tile"]
    traffic = measured_traffic(dom, dom_tile, w)
    roof = {"bound": "hbm", "achieved": dk["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["GBs"] / HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None, "traffic_unit": "bytes/launch",
            "traffic_detail": traffic, "kernel": dom, "tile": dom_tile,
            "algorithmic_bytes_per_launch": dk["bytes"], "avg_launch_us": dk["us"]}

    result = {
        "metric": "F/F* matvecs/s + HBM GB/s vs peak",
        "value": matvecs / (ms_step * 1e-3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: Nd={w.Nd} Nm={w.Nm} Nt={w.Nt} L={op.L}, BF16 spectrum + FP32 "
                               f"accumulation; step = misfit gradient on 1 RHS + 64 F F* columns + F and F* "
                               f"on 32 ragged RHS ({matvecs} matvecs)",
                   "Nd": w.Nd, "Nm": w.Nm, "Nt": w.Nt, "spectrum": "bf16", "matvecs_per_step": matvecs},
        "roofline": roof,
        "parts_ms": {"single_rhs_gradient": part_ms[0], "hessian_64_columns": part_ms[1],
                     "ragged_32_F_and_Ft": part_ms[2]},
        "single_rhs_matvecs_per_s": 2.0 / (part_ms[0] * 1e-3),
        "batched_matvecs_per_s": 2.0 * N_HESS / (part_ms[1] * 1e-3),
        "kernels": kern,
        "kernels_us_by_nrhs": {str(n): {k: avg_us(k, st) for k in st if st[k][1]}
                               for n, st in ((1, st1), (N_HESS, st64), (N_RAGGED, st32))},
        "load_ms": load_ms,
        "autotune": {str(k): v for k, v in tuned.items()},
    }

    from paper_2501_14911_amd import bandwidth_probe
    probe = bandwidth_probe(device=dev)
    result["measured_stream"] = probe
    roof["frac_of_measured_read"] = dk["GBs"] / probe["read_GBs"]
    log(f"[bench] streaming probe: read {probe['read_GBs']:.0f} GB/s, copy {probe['copy_GBs']:.0f} GB/s; "
        f"{dom} at {dk['GBs']:.0f} GB/s = {roof['frac']:.1%} of 8 TB/s, {roof['frac_of_measured_read']:.1%} of read probe")

    if not args.no_call_stats:
        result["calls"] = call_stats(op, w, m, d_obs, E, spec_bytes, vec_bytes, probe["read_GBs"], dev, torch, np,
                                     synth)
    for k, v in result.get("calls", {}).items():
        log(f"[bench] {k:5s} median {v['median_ms']:.3f} ms (p10 {v['p10_ms']:.3f}, p90 {v['p90_ms']:.3f}; "
            f"{v['calls']} calls): {v['matvecs_per_s']:.0f} matvecs/s, spectrum {v['spectrum_GBs']:.0f} GB/s "
            f"= {v['spectrum_frac_of_peak']:.1%} of 8 TB/s")

    if not args.no_accuracy:
        result["accuracy"] = accuracy_sample(op, w, m, E, H, hidx, m_r, Y_r, nt_r, dev, torch, np)
    if not args.no_fp16:
        result["fp16"] = fp16_leg(w, dev, torch, np, synth, P2OOperator, m, d_obs, E, args.no_accuracy)
    if not args.no_fp64:
        result["fp64_plain"] = fp64_plain(w, dev, torch, np, synth, P2OOperator, m, d_obs, var,
                                          args.no_accuracy, result)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_cols, np)
    print(json.dumps(result), flush=True)


# HBM traffic per launch of the timed kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of this benchmark (copy-kernel calibration: fetched KiB x 2,
# written KiB x 1; see profiles/), on the paper_time workload.  The matrix-core
# rows come from the autotuner's launches, which run every tile variant on the
# benchmark's shapes.  Valid only for the kernel source it was measured on:
# keyed by the SHA-1 of that file.
_GEMM = ("paper_2501_14911_amd/csrc/gemm_mfma.hip", "7199a5286c99f5aefcbeb78c705c380f0ce2cc96")
_GEMV = ("paper_2501_14911_amd/csrc/gemv.hip", "c9f87c34e4ec54f35d4392f5aa3152c315a2e18b")
# (kernel, tile): (fetch bytes, write bytes); GEMM rows from the autotuner's launches of every tile
_MEASURED = {
    ('gemm_adj_32', 0): (16768916678, 1765821595),
    ('gemm_adj_32', 1): (16800078712, 1765811099),
    ('gemm_adj_32', 2): (16747575447, 1766837819),
    ('gemm_adj_32', 3): (16721608483, 1765895067),
    ('gemm_adj_32', 4): (16763789192, 1782897371),
    ('gemm_adj_32', 5): (16814063237, 1810694459),
    ('gemm_adj_32', 6): (16761001579, 1811694779),
    ('gemm_adj_32', 9): (16737854099, 1765801979),
    ('gemm_adj_32', 10): (16684835769, 1765801979),
    ('gemm_adj_64', 0): (16952011041, 3537111734),
    ('gemm_adj_64', 1): (17071207469, 3535810102),
    ('gemm_adj_64', 2): (32457111877, 3534912246),
    ('gemm_adj_64', 3): (16982867927, 3533839190),
    ('gemm_adj_64', 4): (33574256827, 3566616630),
    ('gemm_adj_64', 5): (17050211450, 3577760502),
    ('gemm_adj_64', 6): (16932340573, 3670009462),
    ('gemm_adj_64', 9): (16919524673, 3531603958),
    ('gemm_adj_64', 10): (33353343939, 3531603958),
    ('gemm_fwd_32', 0): (18397930027, 261020991),
    ('gemm_fwd_32', 1): (18449910610, 261535935),
    ('gemm_fwd_32', 2): (18759615643, 260724127),
    ('gemm_fwd_32', 3): (20813418312, 260850847),
    ('gemm_fwd_32', 4): (19964104051, 262083615),
    ('gemm_fwd_32', 5): (19929158834, 260336255),
    ('gemm_fwd_32', 6): (18581436609, 260754367),
    ('gemm_fwd_32', 7): (18728610983, 260552511),
    ('gemm_fwd_32', 8): (19034864092, 260919615),
    ('gemm_fwd_64', 0): (20272753353, 522875903),
    ('gemm_fwd_64', 1): (20711815515, 522553439),
    ('gemm_fwd_64', 2): (20641582685, 524484831),
    ('gemm_fwd_64', 3): (25466162858, 519329535),
    ('gemm_fwd_64', 4): (24029962852, 522096895),
    ('gemm_fwd_64', 5): (22905637899, 519834719),
    ('gemm_fwd_64', 6): (20512511248, 534636383),
    ('gemm_fwd_64', 7): (20722395220, 531308415),
    ('gemm_fwd_64', 8): (20646713884, 524907615),
    ('gemv_adj', None): (16586663286, 55188267),
    ('gemv_fwd', None): (17107136589, 16166400),
}
TRAFFIC = {k: ((_GEMV if k[0].startswith("gemv") else _GEMM) + v + ("paper_time",)) for k, v in _MEASURED.items()}


def measured_traffic(kernel, tile, w):
    import hashlib
    ent = TRAFFIC.get((kernel, tile))
    if not ent:
        return None
    src, sha, fetch, write, workload = ent
    if workload != w.name:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), src)
    try:
        cur = hashlib.sha1(open(path, "rb").read()).hexdigest()
    except OSError:
        return None
    if cur != sha:
        return None
    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write, "source": src, "sha1": sha}


def call_stats(op, w, m, d_obs, E, spec_bytes, vec_bytes, read_GBs, dev, torch, np, synth, calls=20, warm=3):
    """Whole calls of F and F* (FFTs and products), separately, at one and at
    64 right-hand sides: 3 warm-ups, then the median and 10th / 90th
    percentiles of `calls` calls, each bracketed by HIP events on the plan's
    stream.  Spectrum GB/s counts the spectrum bytes once per call."""
    m64 = synth.param_series(w, N_HESS, seed_offset=41, backend="torch", device=dev).float()
    d1 = d_obs.unsqueeze(0)
    out = {"F_1": (lambda o: op.apply_F(m.unsqueeze(0), out=o), (1, w.Nt, w.Nd), 1),
           "Ft_1": (lambda o: op.apply_Ft(d1, out=o), (1, w.Nt, w.Nm), 1),
           "F_64": (lambda o: op.apply_F(m64, out=o), (N_HESS, w.Nt, w.Nd), N_HESS),
           "Ft_64": (lambda o: op.apply_Ft(E, out=o), (N_HESS, w.Nt, w.Nm), N_HESS)}
    res = {}
    for name, (fn, shape, nrhs) in out.items():
        o = torch.empty(shape, dtype=torch.float32, device=dev)
        for _ in range(warm):
            fn(o)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        for a, b in evs:
            a.record()
            fn(o)
            b.record()
        torch.cuda.synchronize()
        ts = np.array([a.elapsed_time(b) for a, b in evs])
        med = float(np.median(ts))
        res[name] = {"nrhs": nrhs, "calls": calls, "median_ms": med, "p10_ms": float(np.percentile(ts, 10)),
                     "p90_ms": float(np.percentile(ts, 90)), "matvecs_per_s": nrhs / (med * 1e-3),
                     "spectrum_GBs": spec_bytes / (med * 1e-3) / 1e9,
                     "spectrum_frac_of_peak": spec_bytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "spectrum_frac_of_measured_read": spec_bytes / (med * 1e-3) / 1e9 / read_GBs,
                     "algorithmic_GBs": (spec_bytes + vec_bytes(nrhs)) / (med * 1e-3) / 1e9}
        del o
    del m64
    return res


def accuracy_sample(op, w, m, E, H, hidx, m_r, Y_r, nt_r, dev, torch, np):
    """rel-L2 against the FP64 oracle on sampled sensor rows / parameter
    columns of the same outputs (the oracle regenerates those rows or
    columns of every block)."""
    import oracle
    import synth
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(w.Nd, 8, replace=False))
    cols = np.sort(rng.choice(w.Nm, 64, replace=False))
    out = {}
    d = op.apply_F(m).double().cpu().numpy()
    Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
    out["single_F_8rows"] = oracle.rel_l2(d[:, rows], oracle.apply_F(Fr, m.double().cpu().numpy()))
    din = synth.data_series(w, 1)[0]
    s = op.apply_Ft(torch.from_numpy(din).to(dev, torch.float32)).double().cpu().numpy()
    Fc = synth.operator_rows_cols(w, range(w.Nt), cols=cols, backend="torch").numpy()
    out["single_Ft_64cols"] = oracle.rel_l2(s[:, cols], oracle.apply_Ft(Fc, din))
    # data-space columns: F^T e_(t0, s) needs sensor row s of the blocks only
    h = H.double().cpu().numpy()
    errs = []
    for c in range(4):
        j = int(hidx[c])
        t0, sidx = divmod(j, w.Nd)
        rs = np.unique(np.concatenate([rows, [sidx]]))
        Frs = synth.operator_rows_cols(w, range(w.Nt), rows=rs, backend="torch").numpy()
        e = np.zeros((w.Nt, len(rs)))
        e[t0, np.searchsorted(rs, sidx)] = 1.0
        mt = oracle.apply_Ft(Frs, e)
        href = oracle.apply_F(Frs, mt)
        errs.append(oracle.rel_l2(h[c][:, rs], href))
    out["hessian_columns_4x_rows"] = max(errs)
    y = Y_r.double().cpu().numpy()
    mr = m_r.double().cpu().numpy()
    errs = []
    for b in range(4):
        yo = oracle.apply_F(Fr, mr[b:b + 1], nt_r[b:b + 1])[0]
        errs.append(oracle.rel_l2(y[b][:, rows], yo))
    out["ragged_F_4x_8rows"] = max(errs)
    log("[bench] sampled rel-L2 vs FP64 oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()))
    out["tolerance"] = 2e-3
    return out


def fp16_leg(w, dev, torch, np, synth, P2OOperator, m, d_obs, E, no_acc, calls=10):
    """The same operator with an FP16 spectrum: F and F* at one right-hand
    side (streaming path) and at 64 (matrix cores, FP16 entries split into
    BF16 hi + lo), medians of `calls` whole calls, and rel-L2 against the FP64
    oracle on sampled rows / columns."""
    import oracle
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp16", max_rhs=N_HESS, device=dev)
    op.load(lambda c0, n: gpu_blocks(w, c0, n, dev, torch, synth))
    tuned = op.autotune(N_HESS, reps=2)
    m64 = synth.param_series(w, N_HESS, seed_offset=41, backend="torch", device=dev).float()
    runs = {"F_1": lambda: op.apply_F(m.unsqueeze(0)), "Ft_1": lambda: op.apply_Ft(d_obs.unsqueeze(0)),
            "F_64": lambda: op.apply_F(m64), "Ft_64": lambda: op.apply_Ft(E)}
    out = {"autotune_64": {"fwd_tile": tuned["fwd"][0], "adj_tile": tuned["adj"][0]}}
    for name, fn in runs.items():
        for _ in range(2):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        med = float(np.median([a.elapsed_time(b) for a, b in evs]))
        nr = N_HESS if name.endswith("64") else 1
        out[name] = {"median_ms": med, "matvecs_per_s": nr / (med * 1e-3), "calls": calls}
    if not no_acc:
        rng = np.random.default_rng(1)
        rows = np.sort(rng.choice(w.Nd, 8, replace=False))
        cols = np.sort(rng.choice(w.Nm, 64, replace=False))
        Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
        Fc = synth.operator_rows_cols(w, range(w.Nt), cols=cols, backend="torch").numpy()
        d1 = op.apply_F(m.unsqueeze(0))[0].double().cpu().numpy()
        out["rel_l2_single_F_8rows"] = oracle.rel_l2(d1[:, rows], oracle.apply_F(Fr, m.double().cpu().numpy()))
        s1 = op.apply_Ft(d_obs.unsqueeze(0))[0].double().cpu().numpy()
        out["rel_l2_single_Ft_64cols"] = oracle.rel_l2(s1[:, cols], oracle.apply_Ft(Fc, d_obs.double().cpu().numpy()))
        y = op.apply_F(m64).double().cpu().numpy()
        mh = m64[:4].double().cpu().numpy()
        out["rel_l2_batched_F_4x_8rows"] = max(oracle.rel_l2(y[b][:, rows], oracle.apply_F(Fr, mh[b]))
                                               for b in range(4))
        out["tolerance"] = 2e-3
    log("[bench] FP16 spectrum: " + ", ".join(f"{k} {v['median_ms']:.3f} ms" for k, v in out.items()
                                              if isinstance(v, dict) and "median_ms" in v)
        + ("" if no_acc else ", rel-L2 " + ", ".join(f"{k[7:]} {v:.2e}" for k, v in out.items()
                                                      if k.startswith("rel_l2"))))
    op.close()
    del op, m64
    torch.cuda.empty_cache()
    return out


def fp64_plain(w, dev, torch, np, synth, P2OOperator, m, d_obs, var, no_acc, result, steps=5):
    """The plain path: FP64 spectrum, one right-hand side, F then F^*."""
    import oracle
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "fp64", max_rhs=1, device=dev)
    op.load(lambda c0, n: gpu_blocks(w, c0, n, dev, torch, synth))
    m64, d64 = m.double(), d_obs.double()
    op.misfit_grad(m64, d64, var)
    torch.cuda.synchronize()
    op.profile(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        op.misfit_grad(m64, d64, var)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    st = op.stage_times()
    out = {"ms_per_F_plus_Ft": ms, "matvecs_per_s": 2.0 / (ms * 1e-3),
           "gemv_fwd_us": st["gemv_fwd"][0] / max(1, st["gemv_fwd"][1]) * 1e3,
           "gemv_adj_us": st["gemv_adj"][0] / max(1, st["gemv_adj"][1]) * 1e3}
    out["batched_bf16_speedup_per_matvec"] = result["batched_matvecs_per_s"] / out["matvecs_per_s"]
    out["single_bf16_speedup"] = result["single_rhs_matvecs_per_s"] / out["matvecs_per_s"]
    if not no_acc:
        rows = np.sort(np.random.default_rng(1).choice(w.Nd, 8, replace=False))
        d = op.apply_F(m64).cpu().numpy()
        Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
        out["rel_l2_F_8rows"] = oracle.rel_l2(d[:, rows], oracle.apply_F(Fr, m64.cpu().numpy()))
    log(f"[bench] FP64 plain: {ms:.3f} ms per F + F* ({out['matvecs_per_s']:.1f} matvecs/s); batched BF16 "
        f"speedup per matvec {out['batched_bf16_speedup_per_matvec']:.1f}x")
    op.close()
    del op
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, cols, np):
    """The FP64 oracle (direct block-Toeplitz sums with BLAS) on the host
    cores, on the first ``cols`` parameter columns of the same workload; its
    time is scaled by Nm / cols to a full-size matvec rate."""
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = os.cpu_count()
    cols = min(cols, w.Nm)
    F = synth.operator_rows_cols(w, range(w.Nt), cols=np.arange(cols), backend="torch").numpy()
    m = synth.param_series(w.with_(Nm=cols, grid=None), 1)[0]
    din = synth.data_series(w, 1)[0]
    reps, t_f, t_t = 0, 0.0, 0.0
    while reps < 1 or (t_f + t_t < 10.0 and reps < 50):
        t0 = time.perf_counter()
        oracle.apply_F(F, m)
        t1 = time.perf_counter()
        oracle.apply_Ft(F, din)
        t2 = time.perf_counter()
        t_f, t_t, reps = t_f + (t1 - t0), t_t + (t2 - t1), reps + 1
    full = (t_f + t_t) / reps * (w.Nm / cols)
    log(f"[bench] oracle on {cols} columns x {reps}: F {t_f / reps:.2f} s, F* {t_t / reps:.2f} s "
        f"({cores} BLAS threads)")
    return {"value": 2.0 / full, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "sample": f"F and F* on parameter columns 0..{cols - 1} of {w.Nm} (all {w.Nd} sensors, "
                      f"{w.Nt} steps), FP64 numpy block-Toeplitz sums, repeated {reps} times; time per "
                      f"matvec scaled by {w.Nm}/{cols}",
            "seconds_measured": t_f + t_t}


if __name__ == "__main__":
    main()
