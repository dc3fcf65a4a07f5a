"""Benchmark of the FFT-based block-Toeplitz p2o path on one MI355X.

Workload: Nd = 600 sensors, Nm = 16384 parameters per step, Nt = 420 steps
(circulant length 840), synthetic blocks F_k = exp(-k/100) N(0,1)/sqrt(Nm),
half spectrum stored in FP16 (per-block power-of-two scales) with FP32
accumulation: the 16-bit storage whose every result, the data-space columns
included, meets 2e-3 (with BF16 the columns of early spikes do not).

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
beside it for the batched-mixed-precision speedup, and so are a BF16 spectrum
(whole calls), the FP32 spectrum, the 600 x 65536 x 420 one-GPU share (BF16,
66 GB) and the offline / online phases at the paper's dimensions.

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
FP64_MFMA_PEAK_TFLOPS = 78.6
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
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-largest", action="store_true")
    ap.add_argument("--no-posterior", action="store_true")
    ap.add_argument("--no-small", action="store_true")
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

    def loaded(precision, max_rhs, wl=w):
        o = P2OOperator(wl.Nd, wl.Nm, wl.Nt, precision, max_rhs=max_rhs, device=dev)
        t0 = time.perf_counter()
        o.profile(True)
        o.load(lambda c0, n: gpu_blocks(wl, c0, n, dev, torch, synth))
        ms = o.stage_times()["load"][0]
        o.profile(False)
        log(f"[bench] {precision.upper()} spectrum of {wl.name} loaded ({o.fhat_bytes / 1e9:.2f} GB) in "
            f"{time.perf_counter() - t0:.1f} s (load kernels {ms:.1f} ms)")
        return o, ms

    op16, load16_ms = loaded("fp16", N_HESS)    # the step
    op, load_ms = loaded("bf16", N_HESS)        # BF16 comparison: whole calls and accuracy

    # matrix-core tile variants for the batched widths (autotuner, before timing)
    from paper_2501_14911_amd import gemm_tiles
    tiles = gemm_tiles()
    tuned = {}
    for name, o, nr in (("fp16", op16, N_RAGGED), ("fp16", op16, N_HESS), ("bf16", op, N_HESS)):
        r = o.autotune(nr, reps=2)
        tuned[f"{name}_{nr}"] = {d: {"tile": r[d][0], "shape": tiles[r[d][0]], "ms": r[d][1]} for d in ("fwd", "adj")}
        log(f"[bench] autotune {name} nrhs={nr}: fwd tile {r['fwd'][0]} {tiles[r['fwd'][0]]} {r['fwd'][1]:.3f} ms, "
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
        op16.misfit_grad(m, d_obs, var)
        if evs:
            evs[1].record()
        op16.apply_FFt(E, out=H)
        if evs:
            evs[2].record()
        op16.apply_F(m_r, nt_active=nt_r_dev, out=Y_r)
        op16.apply_Ft(d_r, nt_active=nt_r_dev, out=S_r)
        if evs:
            evs[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    op16.profile(True)
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
    st1, st32, st64 = op16.stage_times(1), op16.stage_times(N_RAGGED), op16.stage_times(N_HESS)
    op16.profile(False)
    matvecs = 2 + 2 * N_HESS + 2 * N_RAGGED
    log(f"[bench] {ms_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}): single-RHS gradient "
        f"{part_ms[0]:.3f} ms, 64 F F* columns {part_ms[1]:.3f} ms, 32 ragged F + F* {part_ms[2]:.3f} ms")
    for label, st in (("nrhs= 1", st1), ("nrhs=64", st64), ("nrhs=32", st32)):
        for k, (tot, n) in st.items():
            if n:
                log(f"[bench]   {label} {k:9s} {tot / n * 1e3:9.1f} us x {n / args.steps:.0f}/step")

    # Roofline bookkeeping.  The per-unit figure is the stored spectrum: one
    # pass over it, (Nt+1) Nd Nm complex values of 4 bytes (BF16 or FP16),
    # is what a launch of the products must read whatever its right-hand-side
    # count; the right-hand-side and result spectra (8 bytes per bin and
    # series value) are reported beside it, not in it.
    spec_bytes = op16.nfreq * w.Nd * w.Nm * op16.elem_bytes

    def avg_us(st, k):
        tot, n = st[k]
        return tot / n * 1e3 if n else 0.0

    def vec_bytes(nrhs, param_bytes=8):     # parameter-side values as complex FP32 (8 B) or FP16 pairs (4 B)
        return op.nfreq * nrhs * (w.Nm * param_bytes + w.Nd * 8)

    def gemm_flop(nrhs):        # real-equivalent flops of one pass
        return 2.0 * op.nfreq * w.Nd * (2 * w.Nm) * (2 * nrhs)

    # kernel: (stage times, stage, spectrum precision, right-hand sides, products issued per real-equivalent
    # flop: one FP16 product per form)
    kdefs = {
        "gemv_fwd": (st1, "gemv_fwd", "fp16", 1, None), "gemv_adj": (st1, "gemv_adj", "fp16", 1, None),
        "gemm_fwd_64": (st64, "gemm_fwd", "fp16", N_HESS, 1), "gemm_adj_64": (st64, "gemm_adj", "fp16", N_HESS, 1),
        "project_64": (st64, "project", "fp16", N_HESS, None),
        "gemm_fwd_32": (st32, "gemm_fwd", "fp16", N_RAGGED, 1), "gemm_adj_32": (st32, "gemm_adj", "fp16", N_RAGGED, 1),
    }
    # The 64 data-space columns run with FP16 intermediate operands (the
    # library's default for an FP16 plan with matrix-core products and a
    # compiled transform length): the adjoint writes FP16 pairs, the re-pad
    # reads and writes them, and the forward products take FP16 right-hand
    # sides in the whole-line ring (tile 13 above 128 sensors, 17 / 18 below;
    # not autotuned).
    f16_ops = op16.fp16_operands
    variant = {"gemm_fwd_64": "fp16_rhs", "gemm_adj_64": "fp16_out"} if f16_ops else {}
    kern = {}
    for k, (st, stage, prec, nr, issue) in kdefs.items():
        us = avg_us(st, stage)
        v = {"us": us, "spectrum": prec, "nrhs": nr, "launches_per_step": st[stage][1] / args.steps}
        if k in variant:
            v["operands"] = variant[k]
        if k.startswith("project"):
            # truncate-and-repad: reads the adjoint products and writes the
            # forward operand, each a complex value per bin and series (8 B
            # as complex FP32, 4 B as FP16 pairs)
            v["operand_bytes"] = 4 if f16_ops else 8
            v["bytes"] = 2 * op.nfreq * nr * w.Nm * v["operand_bytes"]
            v["GBs"] = v["bytes"] / (us * 1e-6) / 1e9 if us else 0.0
        else:
            v["spectrum_bytes"] = spec_bytes
            v["rhs_bytes"] = vec_bytes(nr, 4 if k in variant else 8)
            v["GBs"] = spec_bytes / (us * 1e-6) / 1e9 if us else 0.0
            v["GBs_incl_rhs"] = (spec_bytes + v["rhs_bytes"]) / (us * 1e-6) / 1e9 if us else 0.0
        if issue and us:
            v["TFLOPs_real_equiv"] = gemm_flop(nr) / (us * 1e-6) / 1e12
            v["TFLOPs_issued"] = issue * gemm_flop(nr) / (us * 1e-6) / 1e12
        kern[k] = v
    share = {k: kdefs[k][0][kdefs[k][1]][0] for k in kdefs}
    dom = max((k for k in share if not k.startswith("project")), key=share.get)
    dk = kern[dom]
    dom_tile = None
    if dom.startswith("gemm_"):
        nr = int(dom.rsplit("_", 1)[1])
        if variant.get(dom) == "fp16_rhs":       # the library's whole-line tile for the sensor count
            dom_tile = 17 if w.Nd <= 64 else 18 if w.Nd <= 128 else 13
        else:
            dom_tile = tuned[f"{dk['spectrum']}_{nr}"][dom.split("_")[1]]["tile"]
    traffic = measured_traffic(dom, dom_tile, dk["spectrum"], w, variant.get(dom, ""))
    roof = {"bound": "hbm", "achieved": dk["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["GBs"] / HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None, "traffic_unit": "bytes/launch",
            "traffic_detail": traffic, "kernel": dom, "tile": dom_tile, "spectrum": dk["spectrum"],
            "operands": variant.get(dom, "complex_fp32"),
            "algorithmic_bytes_per_launch": spec_bytes, "avg_launch_us": dk["us"],
            "achieved_incl_rhs": dk.get("GBs_incl_rhs"), "frac_incl_rhs": (dk.get("GBs_incl_rhs") or 0) / HBM_PEAK_GBS,
            "rhs_bytes_per_launch": dk.get("rhs_bytes")}
    if "TFLOPs_issued" in dk:
        roof["mfma_TFLOPs_issued"] = dk["TFLOPs_issued"]
        roof["mfma_frac_issued"] = dk["TFLOPs_issued"] / BF16_MFMA_PEAK_TFLOPS

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
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: Nd={w.Nd} Nm={w.Nm} Nt={w.Nt} L={op16.L}, FP16 spectrum, FP32 "
                               f"accumulation; step = misfit gradient on 1 RHS + 64 F F* columns + F and F* on 32 "
                               f"ragged RHS ({matvecs} matvecs)",
                   "Nd": w.Nd, "Nm": w.Nm, "Nt": w.Nt, "spectrum": "fp16", "matvecs_per_step": matvecs},
        "roofline": roof,
        "parts_ms": {"single_rhs_gradient": part_ms[0], "hessian_64_columns": part_ms[1],
                     "ragged_32_F_and_Ft": part_ms[2]},
        "single_rhs_matvecs_per_s": 2.0 / (part_ms[0] * 1e-3),
        "batched_matvecs_per_s": 2.0 * N_HESS / (part_ms[1] * 1e-3),
        "kernels": kern,
        "kernels_us": {lbl: {k: avg_us(st, k) for k in st if st[k][1]}
                       for lbl, st in (("nrhs_1", st1), ("nrhs_64", st64), ("nrhs_32", st32))},
        "load_ms": {"bf16": load_ms, "fp16": load16_ms},
        "autotune": tuned,
    }

    from paper_2501_14911_amd import bandwidth_probe
    probe = bandwidth_probe(device=dev)
    result["measured_stream"] = probe
    roof["frac_of_measured_read"] = dk["GBs"] / probe["read_GBs"]
    log(f"[bench] streaming probe: read {probe['read_GBs']:.0f} GB/s, copy {probe['copy_GBs']:.0f} GB/s; "
        f"{dom} ({dk['spectrum']}) at {dk['GBs']:.0f} GB/s of spectrum = {roof['frac']:.1%} of 8 TB/s, "
        f"{roof['frac_of_measured_read']:.1%} of read probe")

    if not args.no_call_stats:
        result["calls"] = {}
        for name, o in (("bf16", op), ("fp16", op16)):
            cs = call_stats(o, w, m, d_obs, E, spec_bytes, probe["read_GBs"], dev, torch, np, synth)
            result["calls"].update({f"{name}_{k}": v for k, v in cs.items()})
    for k, v in result.get("calls", {}).items():
        log(f"[bench] {k:10s} median {v['median_ms']:.3f} ms (p10 {v['p10_ms']:.3f}, p90 {v['p90_ms']:.3f}; "
            f"{v['calls']} calls): {v['matvecs_per_s']:.0f} matvecs/s, spectrum {v['spectrum_GBs']:.0f} GB/s "
            f"= {v['spectrum_frac_of_peak']:.1%} of 8 TB/s")

    if not args.no_accuracy:
        result["accuracy"] = accuracy_sample(op, op16, w, m, H, hidx, m_r, Y_r, nt_r, dev, torch, np)
    op.close()
    op16.close()
    del op, op16, H, Y_r, S_r, E
    torch.cuda.empty_cache()
    if not args.no_fp32:
        result["fp32"] = single_rhs_leg(w, "fp32", dev, torch, np, synth, P2OOperator, args.no_accuracy)
    if not args.no_fp64:
        result["fp64_plain"] = fp64_plain(w, dev, torch, np, synth, P2OOperator, m, d_obs, var,
                                          args.no_accuracy, result)
    if not args.no_small:
        result["small_configs"] = small_configs_leg(dev, torch, np, synth, P2OOperator, args.no_accuracy)
    if not args.no_largest:
        result["largest"] = largest_leg(dev, torch, np, synth, P2OOperator, args.no_accuracy)
    if not args.no_posterior:
        result["posterior_paper_grid"] = posterior_leg(dev, torch, np, synth, P2OOperator, args.no_accuracy)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_cols, np)
    print(json.dumps(result), flush=True)


# HBM traffic per launch of the timed kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of this benchmark (copy-kernel calibration: fetched KiB x 2,
# written KiB x 1; see profiles/), on the paper_time workload.  The matrix-core
# rows with an empty operand variant come from the autotuner's launches, which
# run every tile variant on the benchmark's shapes (complex FP32 operands); the
# fp16_out / fp16_rhs rows from the step's own 64-column F F* launches (FP16
# intermediate operands).  Valid only for the kernel source it was measured
# on: keyed by the SHA-1 of that file.
_GEMM = ("paper_2501_14911_amd/csrc/gemm_mfma.hip", "500f3eee6e4788c3c66404861889c195fa1fa646")
_GEMV = ("paper_2501_14911_amd/csrc/gemv.hip", "c9f87c34e4ec54f35d4392f5aa3152c315a2e18b")
# (kernel, tile, spectrum precision, operand variant): (fetch bytes, write bytes)
_MEASURED = {
    ('gemm_adj_64', 0, 'bf16', ''): (16942853753, 3537489346),
    ('gemm_adj_64', 1, 'bf16', ''): (17104500028, 3534946371),
    ('gemm_adj_64', 2, 'bf16', ''): (31768355830, 3534329218),
    ('gemm_adj_64', 3, 'bf16', ''): (16983260948, 3533991704),
    ('gemm_adj_64', 4, 'bf16', ''): (33554990155, 3566467287),
    ('gemm_adj_64', 5, 'bf16', ''): (17063562877, 3577773911),
    ('gemm_adj_64', 6, 'bf16', ''): (16942112813, 3669423276),
    ('gemm_adj_64', 9, 'bf16', ''): (16938900097, 3531606765),
    ('gemm_adj_64', 10, 'bf16', ''): (33539370174, 3544518295),
    ('gemm_adj_64', 15, 'bf16', ''): (16901021082, 3534618477),
    ('gemm_adj_64', 16, 'bf16', ''): (33664828213, 3531677762),
    ('gemm_fwd_64', 0, 'bf16', ''): (20323290132, 523066045),
    ('gemm_fwd_64', 1, 'bf16', ''): (20719164951, 522427112),
    ('gemm_fwd_64', 2, 'bf16', ''): (20641849215, 524829544),
    ('gemm_fwd_64', 3, 'bf16', ''): (25562691581, 519522387),
    ('gemm_fwd_64', 4, 'bf16', ''): (24013753316, 522089533),
    ('gemm_fwd_64', 5, 'bf16', ''): (22932785187, 519748648),
    ('gemm_fwd_64', 6, 'bf16', ''): (20514379486, 534824466),
    ('gemm_fwd_64', 7, 'bf16', ''): (20777059613, 531616786),
    ('gemm_fwd_64', 8, 'bf16', ''): (20645856334, 525254589),
    ('gemm_fwd_64', 11, 'bf16', ''): (29230050768, 533705213),
    ('gemm_fwd_64', 12, 'bf16', ''): (24999208790, 555568296),
    ('gemm_fwd_64', 13, 'bf16', ''): (20388694676, 528415954),
    ('gemm_fwd_64', 14, 'bf16', ''): (29962048433, 529273704),
    ('gemm_adj_32', 9, 'fp16', ''): (16922849448, 1765827702),
    ('gemm_adj_32', 10, 'fp16', ''): (16851931162, 1775968801),
    ('gemm_adj_32', 15, 'fp16', ''): (16839668069, 1765926476),
    ('gemm_adj_32', 16, 'fp16', ''): (16917589911, 1765803084),
    ('gemm_adj_64', 9, 'fp16', ''): (16996708068, 3531649432),
    ('gemm_adj_64', 10, 'fp16', ''): (33744490742, 3554068077),
    ('gemm_adj_64', 15, 'fp16', ''): (16887236772, 3534404077),
    ('gemm_adj_64', 16, 'fp16', ''): (33796669647, 3531618242),
    ('gemm_fwd_32', 7, 'fp16', ''): (19039659940, 260075263),
    ('gemm_fwd_32', 8, 'fp16', ''): (19138077045, 260911529),
    ('gemm_fwd_32', 11, 'fp16', ''): (21691994840, 262634537),
    ('gemm_fwd_32', 12, 'fp16', ''): (20537077202, 266294591),
    ('gemm_fwd_32', 13, 'fp16', ''): (18543777981, 262786303),
    ('gemm_fwd_32', 14, 'fp16', ''): (18541415644, 263958569),
    ('gemm_fwd_64', 7, 'fp16', ''): (21117670687, 526445053),
    ('gemm_fwd_64', 8, 'fp16', ''): (20645911622, 525184957),
    ('gemm_fwd_64', 11, 'fp16', ''): (27885444225, 531038546),
    ('gemm_fwd_64', 12, 'fp16', ''): (23608629043, 535116136),
    ('gemm_fwd_64', 13, 'fp16', ''): (20385855376, 527147069),
    ('gemm_fwd_64', 14, 'fp16', ''): (32336739755, 527812818),
    ('gemv_adj', None, 'fp16', ''): (16586661619, 55188224),
    ('gemv_fwd', None, 'fp16', ''): (17107815270, 16166400),
    ('gemm_adj_64', 15, 'fp16', 'fp16_out'): (16892934072, 1767214934),
    ('gemm_fwd_64', 13, 'fp16', 'fp16_rhs'): (18530538730, 529057821),
}
TRAFFIC = {k: ((_GEMV if k[0].startswith("gemv") else _GEMM) + v + ("paper_time",)) for k, v in _MEASURED.items()}


def measured_traffic(kernel, tile, precision, w, variant=""):
    import hashlib
    ent = TRAFFIC.get((kernel, tile, precision, variant))
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


def call_stats(op, w, m, d_obs, E, spec_bytes, read_GBs, dev, torch, np, synth, calls=20, warm=3):
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
                     "spectrum_frac_of_measured_read": spec_bytes / (med * 1e-3) / 1e9 / read_GBs}
        del o
    del m64
    return res


def column_error_estimate(w, h_col, j, k_other, rng, np):
    """Relative L2 error of one data-space column h = F F* e_j over all
    Nd x Nt outputs against the FP64 oracle, estimated without the whole
    operator: the spike's own sensor row s exactly, plus (Nd - 1) / k times
    the squared error and squared norm of k other sensor rows drawn at random
    (F* e_j needs row s of the blocks only, so a sampled output row r costs
    rows r and s of every block).  Returns (estimate, spike row alone)."""
    import oracle
    import synth
    t0, sidx = divmod(int(j), w.Nd)
    others = np.sort(rng.choice(np.setdiff1d(np.arange(w.Nd), [sidx]), k_other, replace=False))
    rs = np.concatenate([[sidx], others])
    Frs = synth.operator_rows_cols(w, range(w.Nt), rows=rs, backend="torch").numpy()
    e = np.zeros((w.Nt, len(rs)))
    e[t0, 0] = 1.0
    href = oracle.apply_F(Frs, oracle.apply_Ft(Frs, e))
    err2 = ((h_col[:, rs] - href) ** 2).sum(axis=0)
    ref2 = (href ** 2).sum(axis=0)
    scale = (w.Nd - 1) / k_other
    est = np.sqrt((err2[0] + scale * err2[1:].sum()) / (ref2[0] + scale * ref2[1:].sum()))
    return float(est), float(np.sqrt(err2[0] / ref2[0]))


def accuracy_sample(op, op16, w, m, H, hidx, m_r, Y_r, nt_r, dev, torch, np):
    """rel-L2 against the FP64 oracle.  F m and F* d on N(0, 1) inputs: on
    random sensor rows / parameter columns of the outputs (an unbiased sample:
    the inputs have no structure).  Data-space columns: the whole-output
    estimate of column_error_estimate for the columns whose spikes sit at
    t = 0 (the hardest case: output concentrated near lag 0) and t = Nt - 1."""
    import oracle
    import synth
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(w.Nd, 8, replace=False))
    cols = np.sort(rng.choice(w.Nm, 64, replace=False))
    Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
    Fc = synth.operator_rows_cols(w, range(w.Nt), cols=cols, backend="torch").numpy()
    mh = m.double().cpu().numpy()
    din = synth.data_series(w, 1)[0]
    out = {}
    for name, o in (("bf16", op), ("fp16", op16)):
        d = o.apply_F(m).double().cpu().numpy()
        out[f"{name}_single_F_8rows"] = oracle.rel_l2(d[:, rows], oracle.apply_F(Fr, mh))
        s = o.apply_Ft(torch.from_numpy(din).to(dev, torch.float32)).double().cpu().numpy()
        out[f"{name}_single_Ft_64cols"] = oracle.rel_l2(s[:, cols], oracle.apply_Ft(Fc, din))
    h = H.double().cpu().numpy()
    crng = np.random.default_rng(2)
    for c in (0, 1):
        est, spike = column_error_estimate(w, h[c], hidx[c], 8, crng, np)
        t0 = int(hidx[c]) // w.Nd
        out[f"fp16_hessian_column_t{t0}_whole_output_estimate"] = est
        out[f"fp16_hessian_column_t{t0}_spike_row"] = spike
    y = Y_r.double().cpu().numpy()
    mr = m_r.double().cpu().numpy()
    out["fp16_ragged_F_4x_8rows"] = max(oracle.rel_l2(y[b][:, rows], oracle.apply_F(Fr, mr[b:b + 1], nt_r[b:b + 1])[0])
                                        for b in range(4))
    log("[bench] rel-L2 vs FP64 oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()))
    out["tolerance"] = 2e-3
    return out


def single_rhs_leg(w, precision, dev, torch, np, synth, P2OOperator, no_acc, calls=10):
    """F and F* on one right-hand side (streaming products) with a spectrum
    in `precision`: medians of `calls` whole calls, spectrum GB/s, and
    rel-L2 against the FP64 oracle on random rows / columns."""
    import oracle
    op = P2OOperator(w.Nd, w.Nm, w.Nt, precision, max_rhs=1, device=dev)
    op.load(lambda c0, n: gpu_blocks(w, c0, n, dev, torch, synth))
    dt = op.dtype
    m = synth.param_series(w, 1, backend="torch", device=dev)[0].to(dt)
    d = synth.data_series(w, 1, backend="torch", device=dev)[0].to(dt)
    spec = op.nfreq * w.Nd * w.Nm * op.elem_bytes
    out = {"spectrum_bytes": spec}
    for name, fn in (("F_1", lambda: op.apply_F(m)), ("Ft_1", lambda: op.apply_Ft(d))):
        for _ in range(2):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        med = float(np.median([a.elapsed_time(b) for a, b in evs]))
        out[name] = {"median_ms": med, "matvecs_per_s": 1e3 / med, "spectrum_GBs": spec / (med * 1e-3) / 1e9,
                     "spectrum_frac_of_peak": spec / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, "calls": calls}
    if not no_acc:
        rng = np.random.default_rng(3)
        rows = np.sort(rng.choice(w.Nd, 6, replace=False))
        cols = np.sort(rng.choice(w.Nm, 48, replace=False))
        Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
        Fc = synth.operator_rows_cols(w, range(w.Nt), cols=cols, backend="torch").numpy()
        y = op.apply_F(m).double().cpu().numpy()
        s = op.apply_Ft(d).double().cpu().numpy()
        out["rel_l2_F_6rows"] = oracle.rel_l2(y[:, rows], oracle.apply_F(Fr, m.double().cpu().numpy()))
        out["rel_l2_Ft_48cols"] = oracle.rel_l2(s[:, cols], oracle.apply_Ft(Fc, d.double().cpu().numpy()))
        out["tolerance"] = {"fp64": 1e-12, "fp32": 1e-5}.get(precision, 2e-3)
    log(f"[bench] {precision.upper()} spectrum: " + ", ".join(
        f"{k} {v['median_ms']:.3f} ms ({v['spectrum_frac_of_peak']:.1%} of 8 TB/s)" for k, v in out.items()
        if isinstance(v, dict)) + ("" if no_acc else f", rel-L2 F {out['rel_l2_F_6rows']:.2e}, "
                                                      f"F* {out['rel_l2_Ft_48cols']:.2e}"))
    op.close()
    del op
    torch.cuda.empty_cache()
    return out


def largest_leg(dev, torch, np, synth, P2OOperator, no_acc, calls=10, nrhs=16):
    """The 600 x 65536 x 420 one-GPU share, BF16 spectrum (66 GB): F and F*
    at one and at 16 right-hand sides (medians of `calls` whole calls) and
    the misfit gradient at m_true (d = F m_true + 0.01 eps), with the
    gradient against the FP64 oracle on random parameter columns there (the
    residual is minus the noise, so the oracle needs those columns only)."""
    import oracle
    w = synth.CONFIGS["largest"]
    op = P2OOperator(w.Nd, w.Nm, w.Nt, "bf16", max_rhs=nrhs, device=dev)
    t0 = time.perf_counter()
    op.load(lambda c0, n: gpu_blocks(w, c0, n, dev, torch, synth))
    log(f"[bench] largest: BF16 spectrum ({op.fhat_bytes / 1e9:.1f} GB) loaded in {time.perf_counter() - t0:.1f} s")
    r = op.autotune(nrhs, reps=2)
    spec = op.nfreq * w.Nd * w.Nm * op.elem_bytes
    m_true = synth.param_series(w, 1, backend="torch", device=dev, smooth=True)[0].float()
    noise = torch.from_numpy(synth.noise(w, 1)[0]).to(dev, torch.float32)
    with torch.no_grad():
        d_obs = op.apply_F(m_true) + noise
    var = torch.tensor([w.sigma ** 2], dtype=torch.float64, device=dev)
    m16 = synth.param_series(w, nrhs, backend="torch", device=dev, smooth=True).float()
    d16 = synth.data_series(w, nrhs, backend="torch", device=dev).float()
    out = {"workload": f"{w.name}: Nd={w.Nd} Nm={w.Nm} Nt={w.Nt}, BF16 spectrum", "spectrum_bytes": spec,
           "autotune_16": {"fwd_tile": r["fwd"][0], "adj_tile": r["adj"][0]}}
    runs = {"F_1": (lambda: op.apply_F(m_true), 1), "Ft_1": (lambda: op.apply_Ft(d_obs), 1),
            "F_16": (lambda: op.apply_F(m16), nrhs), "Ft_16": (lambda: op.apply_Ft(d16), nrhs),
            "misfit_grad_1": (lambda: op.misfit_grad(m_true, d_obs, var), 2)}
    for name, (fn, nmv) in runs.items():
        for _ in range(2):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        med = float(np.median([a.elapsed_time(b) for a, b in evs]))
        passes = 2 if name.startswith("misfit") else 1
        out[name] = {"median_ms": med, "matvecs_per_s": nmv / (med * 1e-3),
                     "spectrum_GBs": passes * spec / (med * 1e-3) / 1e9,
                     "spectrum_frac_of_peak": passes * spec / (med * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if not no_acc:
        cols = np.sort(np.random.default_rng(14).choice(w.Nm, 32, replace=False))
        _, g = op.misfit_grad(m_true, d_obs, var)
        g = g.double().cpu().numpy()
        Fc = synth.operator_rows_cols(w, range(w.Nt), cols=cols, backend="torch").numpy()
        g_ref = -oracle.apply_Ft(Fc, synth.noise(w, 1)[0]) / w.sigma ** 2
        out["rel_l2_gradient_at_m_true_32cols"] = oracle.rel_l2(g[:, cols], g_ref)
        out["tolerance"] = 2e-3
    log("[bench] largest: " + ", ".join(f"{k} {v['median_ms']:.3f} ms ({v['spectrum_frac_of_peak']:.1%})"
                                        for k, v in out.items() if isinstance(v, dict) and "median_ms" in v)
        + ("" if no_acc else f", gradient rel-L2 {out['rel_l2_gradient_at_m_true_32cols']:.2e}"))
    op.close()
    del op, m16, d16
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
    out["batched_fp16_speedup_per_matvec"] = result["batched_matvecs_per_s"] / out["matvecs_per_s"]
    out["single_fp16_speedup"] = result["single_rhs_matvecs_per_s"] / out["matvecs_per_s"]
    if not no_acc:
        rows = np.sort(np.random.default_rng(1).choice(w.Nd, 8, replace=False))
        d = op.apply_F(m64).cpu().numpy()
        Fr = synth.operator_rows_cols(w, range(w.Nt), rows=rows, backend="torch").numpy()
        out["rel_l2_F_8rows"] = oracle.rel_l2(d[:, rows], oracle.apply_F(Fr, m64.cpu().numpy()))
    log(f"[bench] FP64 plain: {ms:.3f} ms per F + F* ({out['matvecs_per_s']:.1f} matvecs/s); batched FP16 "
        f"speedup per matvec {out['batched_fp16_speedup_per_matvec']:.1f}x")
    op.close()
    del op
    torch.cuda.empty_cache()
    return out


def small_configs_leg(dev, torch, np, synth, P2OOperator, no_acc, calls=200, timed=50):
    """The two small configurations: 4 x 64 x 16 in FP64 and 64 x 4096 x 128
    (L = 256) in FP64 and FP32.  Per call of F, F* and the misfit gradient on
    one right-hand side: the median and 10th / 90th percentiles of `timed`
    calls, each bracketed by HIP events, after 10 warm-ups; the mean of
    `calls` back-to-back calls (events around the batch: launch overhead
    included, no per-call event); and the error of F m and F* d against the
    FP64 oracle (the whole output).  The FP32 spectrum of the second
    configuration (270 MB) is about the size of the 256 MB last-level cache,
    so its repeated calls are cache-assisted."""
    import oracle
    out = {}
    for name, prec in (("tiny", "fp64"), ("medium", "fp64"), ("medium", "fp32")):
        w = synth.CONFIGS[name]
        F = synth.operator_blocks(w)
        op = P2OOperator(w.Nd, w.Nm, w.Nt, prec, max_rhs=1, device=dev)
        Ft = torch.from_numpy(F).to(dev)
        op.load(lambda c0, n: Ft[:, :, c0:c0 + n])
        dt = torch.float64 if prec == "fp64" else torch.float32
        m = synth.param_series(w, 1)
        d = synth.data_series(w, 1)
        d_obs = oracle.apply_F(F, synth.param_series(w, 1, seed_offset=11)) + synth.noise(w, 1)
        mt, dtt, dot = (torch.from_numpy(x[0]).to(dev, dt) for x in (m, d, d_obs))
        var = torch.tensor([w.sigma ** 2], dtype=torch.float64, device=dev)
        res = {"shape": f"{w.Nd} x {w.Nm} x {w.Nt}", "L": op.L, "spectrum_bytes": op.fhat_bytes}
        for key, fn in (("F", lambda: op.apply_F(mt)), ("Ft", lambda: op.apply_Ft(dtt)),
                        ("misfit_grad", lambda: op.misfit_grad(mt, dot, var))):
            for _ in range(10):
                fn()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            for _ in range(calls):
                fn()
            b.record()
            torch.cuda.synchronize()
            res[f"{key}_us"] = a.elapsed_time(b) / calls * 1e3
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(timed)]
            for ea, eb in evs:
                ea.record()
                fn()
                eb.record()
            torch.cuda.synchronize()
            per = np.array([ea.elapsed_time(eb) * 1e3 for ea, eb in evs])
            res[f"{key}_us_median"] = float(np.median(per))
            res[f"{key}_us_p10"], res[f"{key}_us_p90"] = (float(x) for x in np.percentile(per, [10, 90]))
        res["F_spectrum_GBs"] = op.fhat_bytes / (res["F_us_median"] * 1e-6) / 1e9
        res["F_spectrum_frac_of_peak"] = res["F_spectrum_GBs"] / HBM_PEAK_GBS
        if op.fhat_bytes < 300e6 and name != "tiny":
            res["note"] = "spectrum about the size of the 256 MB last-level cache: repeated calls are cache-assisted"
        if not no_acc:
            res["rel_l2_F"] = float(oracle.rel_l2(op.apply_F(mt).double().cpu().numpy(), oracle.apply_F(F, m)[0]))
            res["rel_l2_Ft"] = float(oracle.rel_l2(op.apply_Ft(dtt).double().cpu().numpy(), oracle.apply_Ft(F, d)[0]))
        out[f"{name}_{prec}"] = res
        log(f"[bench] {name} {prec} ({res['shape']}): median per call F {res['F_us_median']:.1f} us, "
            f"F* {res['Ft_us_median']:.1f} us, misfit+gradient {res['misfit_grad_us_median']:.1f} us "
            f"(back-to-back {res['F_us']:.1f} / {res['Ft_us']:.1f} / {res['misfit_grad_us']:.1f} us)" +
            (f"; rel-L2 F {res['rel_l2_F']:.1e}, F* {res['rel_l2_Ft']:.1e}" if not no_acc else ""))
        op.close()
        del op, Ft
    torch.cuda.empty_cache()
    return out


def posterior_leg(dev, torch, np, synth, P2OOperator, no_acc, batch=64, qstride=10, sigma=1e-2):
    """The offline and online phases at the dimensions of the paper's
    numerical example (section 5: Nd = 49, Nm = 513^2, Nt = 500; 16 QoIs every
    10th step), FP16 spectra, stand-in prior Gamma_prior = I, Gamma_noise =
    sigma^2 I: assembly of K (24,500 columns, `batch` per call), its Cholesky
    factorisation, the MAP point (two adjoint and one forward application and
    the two triangular solves), the d2q map Q (800 rows), the online
    prediction Q d, and the QoI posterior covariance (800 columns).  Times
    are HIP events on the stream; K is checked against the FP64 oracle on
    sampled entries (blocks with time indices below 40, two sensors)."""
    import oracle
    from paper_2501_14911_amd import cholesky, d2q_apply
    wf, wq = synth.CONFIGS["paper_grid"], synth.CONFIGS["paper_grid_qoi"]
    t0 = time.perf_counter()
    op = P2OOperator(wf.Nd, wf.Nm, wf.Nt, "fp16", max_rhs=batch, device=dev)
    op.load(lambda c0, n: gpu_blocks(wf, c0, n, dev, torch, synth))
    oq = P2OOperator(wq.Nd, wq.Nm, wq.Nt, "fp16", max_rhs=batch, device=dev)
    oq.load(lambda c0, n: gpu_blocks(wq, c0, n, dev, torch, synth))
    oq.set_output_stride(qstride)
    log(f"[bench] posterior: FP16 spectra of F ({op.fhat_bytes / 1e9:.1f} GB) and F_q ({oq.fhat_bytes / 1e9:.1f} GB) "
        f"loaded in {time.perf_counter() - t0:.1f} s")
    var = torch.tensor([sigma ** 2], dtype=torch.float64, device=dev)
    N, nq = op.data_dim(), oq.Ntd * oq.Nd

    def timed(fn, reps=1):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            out = fn()
        b.record()
        torch.cuda.synchronize()
        return out, a.elapsed_time(b) / reps

    out = {"workload": f"paper grid: Nd={wf.Nd} Nm={wf.Nm} Nt={wf.Nt}, Nq={wq.Nd} every {qstride}th step; FP16 spectra, "
                       f"prior I, noise sigma={sigma}", "data_dim": N, "qoi_dim": nq}
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    _, out["assemble_K_ms"] = timed(lambda: op.assemble_K(var, 1.0, K=K))
    out["assemble_K_ms_per_column"] = out["assemble_K_ms"] / N
    if not no_acc:
        # sampled entries of K: block (i, j), sensors (p, q): sum_k F_{i-k}[p] . F_{j-k}[q] + delta sigma^2
        rng = np.random.default_rng(5)
        sens = np.sort(rng.choice(wf.Nd, 2, replace=False))
        Fr = synth.operator_rows_cols(wf, range(40), rows=sens, backend="torch").numpy()     # [40, 2, Nm]
        Kh = K.cpu().numpy()
        def kref(i, j, a, c):
            v = sum(Fr[i - k, a] @ Fr[j - k, c] for k in range(min(i, j) + 1))
            return v + (sigma ** 2 if i == j and a == c else 0.0)

        errs = []
        for i, j in ((0, 0), (1, 0), (5, 3), (17, 17), (39, 20), (25, 38)):
            for a in range(2):
                for c in range(2):
                    got = Kh[j * wf.Nd + sens[c], i * wf.Nd + sens[a]]      # tensor row = column of K
                    # error against sqrt(K_pp K_qq), the bound of |K_pq| for an SPD K
                    errs.append(abs(got - kref(i, j, a, c)) / np.sqrt(kref(i, i, a, a) * kref(j, j, c, c)))
        out["K_sampled_max_err_vs_diag"] = float(max(errs))
    # the same K from the blocks themselves (Gram matrix of the stacked blocks on
    # the FP64 matrix cores, block-diagonal prefix sums; the blocks regenerated
    # on the GPU chunk by chunk, as a loader would supply them): exact up to
    # FP64 rounding, so it also measures the column route's FP16 error
    from paper_2501_14911_amd import assemble_K_from_blocks
    K2 = torch.empty_like(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assemble_K_from_blocks(lambda c0, n: gpu_blocks(wf, c0, n, dev, torch, synth), wf.Nd, wf.Nm, wf.Nt, var, 1.0,
                           K=K2, chunk_cols=4096, device=dev)
    torch.cuda.synchronize()
    out["assemble_K_from_blocks_ms"] = (time.perf_counter() - t1) * 1e3
    dK = (K - K2).abs().max().item()
    out["K_column_route_max_err_vs_blocks"] = dK / K2.abs().max().item()
    del K2
    torch.cuda.empty_cache()
    L, out["cholesky_ms"] = timed(lambda: cholesky(K))
    d_obs = synth.data_series(wf, 1, backend="torch", device=dev)[0].float() * 0.1
    m_map, out["map_point_ms"] = timed(lambda: op.map_point(d_obs, L, var, 1.0), reps=5)
    Q, out["d2q_map_ms"] = timed(lambda: op.d2q_map(oq, L, var, 1.0))
    dvec = d_obs.double().reshape(1, -1)
    q, out["d2q_apply_ms"] = timed(lambda: d2q_apply(Q, dvec), reps=20)
    C, out["qoi_posterior_cov_ms"] = timed(lambda: op.qoi_posterior_cov(oq, L, 1.0))
    if not no_acc:
        # the online prediction Q d agrees with F_q applied to the MAP point (same operators)
        qm = oq.apply_F(m_map.unsqueeze(0))[0].double().reshape(-1)
        out["Qd_vs_Fq_map_rel"] = float((q[0] - qm).norm() / qm.norm())
        Ch = C.cpu().numpy()
        out["qoi_cov_symmetry_rel"] = float(np.linalg.norm(Ch - Ch.T) / np.linalg.norm(Ch))
    # Rooflines.  Each batched call reads the stored spectrum once per product
    # whatever its right-hand-side count (<= batch); a triangular-solve pair
    # reads the factor once (the forward solve its lower triangle, the
    # backward solve its upper one: N^2 FP64 values).  Algorithmic bytes:
    # spectrum passes x spectrum bytes + solves x 8 N^2.  The Cholesky
    # factorisation is N^3 / 3 FP64 flops (N^3 / 6 multiply-adds).
    fb, fqb, lb = float(op.fhat_bytes), float(oq.fhat_bytes), 8.0 * N * N
    nbk, nbq = -(-N // batch), -(-nq // batch)
    phases = {"assemble_K": (nbk * 2 * fb, out["assemble_K_ms"]),
              "map_point": (3 * fb + lb, out["map_point_ms"]),
              "d2q_map": (nbq * (fqb + 3 * fb + lb), out["d2q_map_ms"]),
              "qoi_posterior_cov": (nbq * (4 * fqb + 2 * fb + lb), out["qoi_posterior_cov_ms"])}
    roof = {k: {"bound": "hbm", "algorithmic_bytes": b, "achieved": b / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS} for k, (b, ms) in phases.items()}
    chol_flop = N ** 3 / 3.0
    roof["cholesky"] = {"bound": "mfma", "algorithmic_flops": chol_flop,
                        "achieved": chol_flop / (out["cholesky_ms"] * 1e-3) / 1e12, "peak": FP64_MFMA_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": chol_flop / (out["cholesky_ms"] * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS}
    gram_flop = float(N) * N * wf.Nm                 # lower triangle of A A^T: N (N + 1) / 2 x Nm multiply-adds
    roof["assemble_K_from_blocks"] = {
        "bound": "mfma", "algorithmic_flops": gram_flop, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
        "achieved": gram_flop / (out["assemble_K_from_blocks_ms"] * 1e-3) / 1e12,
        "frac": gram_flop / (out["assemble_K_from_blocks_ms"] * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "note": "time includes generating the blocks on the GPU chunk by chunk"}
    out["roofline"] = roof
    log("[bench] posterior (paper grid): " + ", ".join(f"{k} {v:.3g}" for k, v in out.items()
                                                      if isinstance(v, float)))
    log("[bench] posterior rooflines: " + ", ".join(f"{k} {v['achieved']:.0f} {v['unit']} ({100 * v['frac']:.1f}%)"
                                                  for k, v in roof.items()))
    op.close()
    oq.close()
    del op, oq, K, L, Q, C
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, cols, np):
    """The FP64 oracle (direct block-Toeplitz sums with BLAS) on the host
    cores, on the first ``cols`` parameter columns of the same workload; its
    time is scaled by Nm / cols to a full-size matvec rate."""
    import oracle
    import synth
    # The oracle's BLAS pool uses the threads the job is given (OMP_NUM_THREADS,
    # 16 per GPU on the benchmark boxes); the host's own count is reported beside it.
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = int(os.environ.get("OMP_NUM_THREADS", "1"))
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = None
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
            "host_os_cpu_count": os.cpu_count(), "host_affinity_cpus": affinity,
            "sample": f"F and F* on parameter columns 0..{cols - 1} of {w.Nm} (all {w.Nd} sensors, "
                      f"{w.Nt} steps), FP64 numpy block-Toeplitz sums, repeated {reps} times; time per "
                      f"matvec scaled by {w.Nm}/{cols}",
            "seconds_measured": t_f + t_t}


if __name__ == "__main__":
    main()
