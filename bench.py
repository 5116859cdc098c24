#!/usr/bin/env python3
"""Benchmark of the truncated cosine-series Poisson solution (arXiv 2307.12041, Sec. III-A/III-C).

One step = one full evaluation of the hot path on one batch of blocks: the coefficient
contraction, reduction, spectral scale and energy (pp_energy) followed by the per-block
energy gradient (pp_field).  Work unit: one (block, u, p) triple, n * Mu * Mp "pairs" per step.

Default workload: 2,000,000 standard cells (width U[1,8], height 1) + 500 macros (sides U[50,400]),
centres uniform in a 16384 x 16384 region, truncation Mu x Mp = 2048 x 2048, precision bf16x3.
Inputs are synthetic (seeded, see workloads/), resident in HBM before the timed region.

Printed: one JSON line with the throughput, the roofline of the dominant kernel (its average
launch duration measured live with HIP events on the launching stream), the FP64 plain
throughput on the same workload, accuracy figures, and the FP64 oracle timed on the host on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block·freq² pairs/s for energy+forces, BF16-split vs FP64 plain, at rel err"
PEAK_TFLOPS = {"bf16x3": 2500.0, "bf16": 2500.0, "fp8x3": 5000.0, "fp8": 5000.0, "fp32": 157.3,
               "fp64": 78.6}   # MI355X dense matrix peaks of each operand type
MFMA_MULT = {"bf16x3": 3, "bf16": 1, "fp8x3": 3, "fp8": 1, "fp32": 1, "fp64": 1}   # executed products per algorithmic one
DTYPE = {"bf16x3": "bf16", "bf16": "bf16", "fp8x3": "fp8", "fp8": "fp8", "fp32": "f32", "fp64": "f64"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    nb = float(np.linalg.norm(np.ravel(b)))
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b))) / (nb if nb > 0 else 1.0)


def tile_rel_max(a, b, t=64):
    """Largest relative error over t x t tiles of two coefficient arrays (each tile judged against its own
    norm, so that no tile is hidden by the larger low-frequency coefficients)."""
    worst = 0.0
    for u0 in range(0, b.shape[0], t):
        for p0 in range(0, b.shape[1], t):
            nb = float(np.linalg.norm(b[u0:u0 + t, p0:p0 + t]))
            if nb > 0:
                worst = max(worst, float(np.linalg.norm(a[u0:u0 + t, p0:p0 + t] - b[u0:u0 + t, p0:p0 + t])) / nb)
    return worst


def row_tile_rel_max(g, gr, t=256):
    """Largest relative error over tiles of t consecutive blocks of a per-block output."""
    worst = 0.0
    for i0 in range(0, gr.shape[0], t):
        nb = float(np.linalg.norm(gr[i0:i0 + t]))
        if nb > 0:
            worst = max(worst, float(np.linalg.norm(g[i0:i0 + t] - gr[i0:i0 + t])) / nb)
    return worst


def errors_vs(ref, out):
    """Errors of one run's (E, a, gx, gy) against a reference run on the same workload."""
    E, a, gx, gy = (v.cpu().numpy() for v in out)
    Er, ar, gxr, gyr = (v.cpu().numpy() for v in ref)
    g, gr = np.stack([gx, gy], axis=1), np.stack([gxr, gyr], axis=1)
    return {"E": abs(float(E) - float(Er)) / abs(float(Er)), "a": rel(a, ar), "a_tile64_max": tile_rel_max(a, ar),
            "g": rel(g, gr), "g_tile256_max": row_tile_rel_max(g, gr),
            "g_max_block": float(np.max(np.hypot(gx - gxr, gy - gyr)) / np.max(np.hypot(gxr, gyr)))}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The sources that build each precision's contraction kernels and their launches: a committed counter
# summary (profiles/traffic_*, profiles/mfma_*) is used only while these files are unchanged.
COMMON_SOURCES = ("api.hip", "common.h", "basis_gen.h", "kernels_common.hip")
KERNEL_SOURCES = {"bf16x3": ("kernels_bf16.hip",), "bf16": ("kernels_bf16.hip",), "bf16mix": ("kernels_bf16.hip",),
                  "fp8x3": ("kernels_bf16.hip", "kernels_fp8.hip"), "fp8": ("kernels_bf16.hip", "kernels_fp8.hip"),
                  "fp64": ("kernels_f64.hip",), "fp32": ("kernels_f64.hip",)}


def code_tokens(src):
    """The code of a C++ source without its comments and with whitespace runs collapsed (string and
    character literals kept), so that a change of comments or layout alone keeps the hash below."""
    import re
    pat = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'', re.S)
    code = pat.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ", src)
    return " ".join(code.split())


def kernel_source_hash(precision="bf16x3"):
    """sha256 of the code (comments and layout aside) of one precision's kernel sources; counter
    figures are reported only for the kernels they were taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2307_12041_amd", "csrc")
    hs = hashlib.sha256()
    for f in COMMON_SOURCES + KERNEL_SOURCES[precision]:
        hs.update(code_tokens(open(os.path.join(d, f)).read()).encode())
        hs.update(b"\0")
    return hs.hexdigest()


def measured_traffic(workload, precision, stage):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (profiles/traffic_<precision>_<workload>.json), or None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{precision}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash(precision):
        return None
    st = rec.get("stages", {}).get(stage)
    return None if st is None else st.get("hbm_bytes_per_launch")


def measured_mfma(workload, precision):
    """Counter-measured MFMA utilisation of the contractions from the committed rocprofv3 summary
    (profiles/mfma_<precision>_<workload>.json), or None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"mfma_{precision}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash(precision):
        return None
    return rec.get("kernels")


def library_gemm(torch, dev, wl, stages, args, max_operand_bytes=20 * 2**30):
    """Context for the contraction rate, not part of the path: the vendor bf16 GEMM (torch.mm, which
    calls hipBLASLt, fp32 accumulation) timed with HIP events on torch's stream, one product of
    stored operands of the coefficient contraction's shape (Mu x n times n x Mp, the store-mode
    forward's plain product without its table build) and one square 8192^3 product.  Random normal
    operands; only the time is used.  Beside it, the time per product of this library's own
    contractions in the timed run (the x3 split executes three per launch, generating its operands)."""
    cases = {"contraction_shape": (wl.Mu, wl.n, wl.Mp), "square_8192": (8192, 8192, 8192)}
    rec = {"gemm": "torch.mm bf16 -> hipBLASLt"}
    for name, (m, k, nn) in cases.items():
        if 2 * k * (m + nn) > max_operand_bytes:
            rec[name] = {"shape": [m, k, nn], "skipped": "operands above the size cap"}
            continue
        A = torch.randn(m, k, device=dev, dtype=torch.bfloat16)
        B = torch.randn(k, nn, device=dev, dtype=torch.bfloat16)
        torch.mm(A, B)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.library_steps):
            torch.mm(A, B)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.library_steps
        tf = 2.0 * m * k * nn / (ms * 1e-3) / 1e12
        rec[name] = {"shape": [m, k, nn], "ms": round(ms, 3), "tflops": round(tf, 1),
                     "frac_of_bf16_peak": round(tf / PEAK_TFLOPS["bf16"], 4)}
        del A, B
        torch.cuda.empty_cache()
    mult = MFMA_MULT[args.precision]
    ours = {}
    for st in ("fwd", "bwd"):
        per = stages[st][0] / stages[st][1] / mult
        ours[st] = {"ms_per_product": round(per, 3),
                    "executed_tflops": round(2.0 * wl.pairs / (per * 1e-3) / 1e12, 1)}
    rec["ours_" + args.precision] = ours
    cs = rec["contraction_shape"]
    if "ms" in cs:
        log(f"[bench] library bf16 GEMM {cs['shape']}: {cs['ms']:.2f} ms ({cs['tflops']:.0f} TFLOP/s); square 8192^3: "
            + (f"{rec['square_8192']['tflops']:.0f} TFLOP/s" if "ms" in rec["square_8192"] else "skipped")
            + f"; ours per product: fwd {ours['fwd']['ms_per_product']:.2f} ms ({ours['fwd']['executed_tflops']:.0f}),"
            f" bwd {ours['bwd']['ms_per_product']:.2f} ms ({ours['bwd']['executed_tflops']:.0f})")
    return rec


def mfma_sustained(torch, pp, dev, iters, reps=3):
    """The bf16 matrix rate the chip sustains with every CU loaded: the library's calibration kernel
    (one workgroup of four waves per CU, each wave 16 MFMAs per iteration on normally distributed
    operands, nothing else in its loop), timed with HIP events on torch's stream.  Under such a load
    the power limit sets the clock, so this is the practical ceiling of an MFMA-bound kernel on data
    like the contractions' operands."""
    wg = torch.cuda.get_device_properties(dev).multi_processor_count
    out = torch.empty(wg * 256, dtype=torch.float32, device=dev)
    pp.mfma_calibrate(out, workgroups=wg, iters=iters)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pp.mfma_calibrate(out, workgroups=wg, iters=iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = wg * 4 * 16 * iters * 32768.0 / (ms * 1e-3) / 1e12
    return {"kernel": "k_mfma_calibrate (pp_mfma_calibrate)", "workgroups": wg, "iters": iters, "ms": round(ms, 3),
            "tflops": round(tf, 1), "frac_of_bf16_peak": round(tf / PEAK_TFLOPS["bf16"], 4)}


def timed_steps(pp, torch, t, wl, prec, steps, warmup, ws, positions=None, basis="recompute"):
    """Warm up, then time `steps` evaluations (energy + gradient).  With `positions` (a list of
    (x, y) device tensors) step k evaluates positions[k % len]."""
    kw = dict(W=wl.W, H=wl.H, precision=prec, workspace=ws, basis=basis)

    def args(k):
        if positions is None:
            return t
        x, y = positions[k % len(positions)]
        return [x, y, t[2], t[3]]

    for k in range(warmup):
        E, a = pp.energy(*args(k), Mu=wl.Mu, Mp=wl.Mp, **kw)
        pp.field(*args(k), a, **kw)
    torch.cuda.synchronize()
    pp.timing_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        E, a = pp.energy(*args(k), Mu=wl.Mu, Mp=wl.Mp, **kw)
        gx, gy = pp.field(*args(k), a, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = {}
    for st in ("tables", "seeds", "build", "fwd", "reduce", "energy", "prep", "bwd", "final", "point", "potential"):
        ms, cnt = pp.timing_query(st)
        if cnt:
            stages[st] = (ms, cnt)
    pp.timing_enable(False)
    return (t1 - t0), stages, (E, a, gx, gy)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4, help="workload index in workloads.CONFIGS")
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "bf16", "fp8x3", "fp8", "fp32", "fp64"])
    ap.add_argument("--basis", default="recompute", choices=["recompute", "store"],
                    help="basis tables regenerated on chip, or built in HBM once per step")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--fp32-steps", type=int, default=2, help="steps of the FP32 path on the same workload (0: skip)")
    ap.add_argument("--mix-steps", type=int, default=3,
                    help="steps of the mixed bf16 split (three products on the low-frequency tiles only) on the "
                         "same workload (0: skip)")
    ap.add_argument("--fp8-steps", type=int, default=3, help="steps of the FP8X3 and FP8 paths on the same workload "
                                                             "(0: skip)")
    ap.add_argument("--bins", type=int, default=-1,
                    help="bins per axis of the Sec. III-D bin-scheme comparison leg (-1: the workload's truncation "
                         "when Mu = Mp; 0: skip)")
    ap.add_argument("--eval-precision", default="bf16x3", choices=["bf16x3", "bf16", "fp32", "fp64", "none"],
                    help="time the evaluation calls (point field at the block centres, block potentials)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=12000, help="blocks in the oracle's timed sample")
    ap.add_argument("--jitter", action="store_true",
                    help="each timed step evaluates new positions: the base positions plus N(0,1) jitter, prepared "
                         "on the device before the timed region (the repeated-evaluation workload)")
    ap.add_argument("--library-steps", type=int, default=3,
                    help="timed calls of the vendor bf16 GEMM (torch.mm, hipBLASLt) on stored operands of the "
                         "coefficient contraction's shape and on a square 8192^3 product, for context (0: skip)")
    ap.add_argument("--mfma-calibration-iters", type=int, default=40000,
                    help="iterations of the matrix-core calibration kernel (one workgroup per CU, 16 bf16 MFMAs "
                         "per wave and iteration on normally distributed operands), timed for the sustained bf16 "
                         "matrix rate under load (0: skip)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="run one device copy of this many GiB first (reference kernel for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the multi-GPU sharding (blocks split over GPUs, one all-reduce of the Mu x Mp moments) is a "
              "design, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_12041_amd as pp
    from workloads import make_config

    dev = "cuda:0"
    wl = make_config(args.workload)
    pairs = wl.pairs
    log(f"[bench] workload {wl.name}: n={wl.n} Mu={wl.Mu} Mp={wl.Mp} pairs/step={pairs:.3e}")
    t = [torch.as_tensor(v, device=dev) for v in wl.arrays()]
    need = max([pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=p) for p in ("fp32", "fp64", "fp8x3", "bf16mix")]
               + [pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=args.precision, basis=args.basis)])
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    log(f"[bench] workspace {need / 2**20:.1f} MiB")
    if args.copy_calibration_gib > 0:
        nb = int(args.copy_calibration_gib * 2**30)
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst

    positions = None
    if args.jitter:
        from workloads import jitter
        positions = []
        for k in range(args.steps):
            j = jitter(wl, k)
            positions.append((torch.as_tensor(j.x, device=dev), torch.as_tensor(j.y, device=dev)))
        log(f"[bench] {args.steps} jittered position sets resident on the device")
    dt, stages, (E, a, gx, gy) = timed_steps(pp, torch, t, wl, args.precision, args.steps, args.warmup, ws, positions,
                                             basis=args.basis)
    value = pairs * args.steps / dt
    log(f"[bench] {args.precision}: {dt / args.steps * 1e3:.2f} ms/step, {value:.4e} pairs/s; stages "
        + ", ".join(f"{k}={v[0] / v[1]:.2f}ms x{v[1] // args.steps}" for k, v in stages.items()))

    # Roofline of the dominant kernel: the stage with the largest total time.
    dom = max(("fwd", "bwd"), key=lambda s: stages[s][0])
    avg_ms = stages[dom][0] / stages[dom][1]
    alg_flops = 2.0 * pairs                  # one contraction: 2 flops per (block, u, p)
    achieved = alg_flops / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    X = "x3" if args.precision == "bf16x3" else "plain"
    if args.basis == "recompute":
        kernel_name = {"fwd": f"k_fwd1_bf16<{X}> (coefficient contraction)",
                       "bwd": f"k_bwd1_bf16<{X}> (gradient contraction, gx and gy launches)"}[dom]
    else:
        kernel_name = {"fwd": f"k_fwd_bf16_st<{X}> (coefficient contraction)",
                       "bwd": f"k_bwd_bf16_st<{X}> (gradient contraction, gx and gy launches)"}[dom]
    if args.precision in ("fp64", "fp32"):
        T = "double" if args.precision == "fp64" else "float"
        kernel_name = {"fwd": f"k_fwd_mat<{T}>", "bwd": f"k_bwd_mat<{T}>"}[dom]
    if args.precision in ("fp8x3", "fp8"):
        X = "x3" if args.precision == "fp8x3" else "plain"
        kernel_name = {"fwd": f"k_fwd_fp8<{X}> (coefficient contraction)",
                       "bwd": f"k_bwd_fp8<{X}> (gradient contraction, gx and gy launches)"}[dom]
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(wl.name, args.precision, dom),
                "kernel": kernel_name, "avg_launch_ms": round(avg_ms, 3), "launches_per_step": stages[dom][1] // args.steps,
                "algorithmic_flops_per_launch": alg_flops,
                "executed_mfma_tflops": round(achieved * MFMA_MULT[args.precision], 2),
                "executed_mfma_frac": round(achieved * MFMA_MULT[args.precision] / peak, 4),
                "mfma_counters": measured_mfma(wl.name, args.precision)}

    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision],
           "data": "synthetic",
           "config": {"workload": wl.name + ("_jittered" if args.jitter else ""), "n_blocks": wl.n, "Mu": wl.Mu,
                      "Mp": wl.Mp, "W": wl.W, "H": wl.H, "precision": args.precision, "basis": args.basis,
                      "pairs_per_step": pairs},
           "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
           "roofline": roofline}

    ref = None
    if not args.no_fp64 and args.precision != "fp64":
        dt64, st64, ref = timed_steps(pp, torch, t, wl, "fp64", args.fp64_steps, 1, ws)
        v64 = pairs * args.fp64_steps / dt64
        log(f"[bench] fp64 plain: {dt64 / args.fp64_steps * 1e3:.1f} ms/step, {v64:.4e} pairs/s")
        out["fp64_plain"] = {"value": v64, "unit": "pairs/s", "ms_per_step": dt64 / args.fp64_steps * 1e3,
                             "steps": args.fp64_steps,
                             "stages_ms_per_step": {k: round(v[0] / args.fp64_steps, 3) for k, v in st64.items()},
                             "mfma_counters": measured_mfma(wl.name, "fp64")}
        out["speedup_vs_fp64_plain"] = value / v64

    if args.fp32_steps > 0 and args.precision != "fp32":
        dt32, st32, r32 = timed_steps(pp, torch, t, wl, "fp32", args.fp32_steps, 1, ws)
        v32 = pairs * args.fp32_steps / dt32
        log(f"[bench] fp32: {dt32 / args.fp32_steps * 1e3:.1f} ms/step, {v32:.4e} pairs/s")
        out["fp32_plain"] = {"value": v32, "unit": "pairs/s", "ms_per_step": dt32 / args.fp32_steps * 1e3,
                             "steps": args.fp32_steps,
                             "stages_ms_per_step": {k: round(v[0] / args.fp32_steps, 3) for k, v in st32.items()}}
        if ref is not None:
            out["fp32_plain"]["rel_err_vs_fp64_gpu"] = errors_vs(ref, r32)
        out["speedup_vs_fp32"] = value / v32

    mix_run = None
    if args.mix_steps > 0 and args.precision == "bf16x3" and args.basis == "recompute":
        # The mixed split on the same workload: three products on the low-frequency tiles, one elsewhere.
        dtm, stm, rm = timed_steps(pp, torch, t, wl, "bf16mix", args.mix_steps, 1, ws)
        mix_run = rm
        vm = pairs * args.mix_steps / dtm
        rec = {"value": vm, "unit": "pairs/s", "ms_per_step": dtm / args.mix_steps * 1e3, "steps": args.mix_steps,
               "stages_ms_per_step": {k: round(v[0] / args.mix_steps, 3) for k, v in stm.items()},
               "speedup_vs_bf16x3": vm / value, "mfma_counters": measured_mfma(wl.name, "bf16mix")}
        if ref is not None:
            rec["rel_err_vs_fp64_gpu"] = errors_vs(ref, rm)
        out["bf16mix"] = rec
        log(f"[bench] bf16mix: {dtm / args.mix_steps * 1e3:.1f} ms/step, {vm:.4e} pairs/s; stages "
            + ", ".join(f"{k}={v[0] / v[1]:.2f}ms x{v[1] // args.mix_steps}" for k, v in stm.items())
            + (f"; vs fp64 {rec['rel_err_vs_fp64_gpu']}" if ref is not None else ""))

    fp8_runs = {}
    if args.fp8_steps > 0 and args.precision not in ("fp8x3", "fp8"):
        # The FP8 operand types (e4m3 on the scaled f8f6f4 MFMA) on the same workload: time, stages,
        # the gradient contraction's share of the fp8 matrix peak, and the error against FP64.
        out["fp8"] = {}
        for p8 in ("fp8x3", "fp8"):
            dt8, st8, r8 = timed_steps(pp, torch, t, wl, p8, args.fp8_steps, 1, ws)
            v8 = pairs * args.fp8_steps / dt8
            fp8_runs[p8] = r8
            bwd_ms = st8["bwd"][0] / st8["bwd"][1]
            rec = {"value": v8, "unit": "pairs/s", "ms_per_step": dt8 / args.fp8_steps * 1e3, "steps": args.fp8_steps,
                   "stages_ms_per_step": {k: round(v[0] / args.fp8_steps, 3) for k, v in st8.items()},
                   "bwd_launch_ms": round(bwd_ms, 3),
                   "bwd_frac_of_fp8_peak": round(2.0 * pairs / (bwd_ms * 1e-3) / 1e12 / PEAK_TFLOPS[p8], 4),
                   "speedup_vs_" + args.precision: v8 / value,
                   "mfma_counters": measured_mfma(wl.name, p8), "traffic": {
                       st: measured_traffic(wl.name, p8, st) for st in ("fwd", "bwd")}}
            if ref is not None:
                rec["rel_err_vs_fp64_gpu"] = errors_vs(ref, r8)
            out["fp8"][p8] = rec
            log(f"[bench] {p8}: {dt8 / args.fp8_steps * 1e3:.1f} ms/step, {v8:.4e} pairs/s; stages "
                + ", ".join(f"{k}={v[0] / v[1]:.2f}ms x{v[1] // args.fp8_steps}" for k, v in st8.items())
                + (f"; vs fp64 {rec['rel_err_vs_fp64_gpu']}" if ref is not None else ""))

    if args.library_steps > 0 and args.precision in ("bf16x3", "bf16"):
        out["library_gemm"] = library_gemm(torch, dev, wl, stages, args)
    if args.mfma_calibration_iters > 0 and args.precision in ("bf16x3", "bf16"):
        cal = mfma_sustained(torch, pp, dev, args.mfma_calibration_iters)
        out["mfma_sustained"] = cal
        roofline["executed_frac_of_sustained"] = round(roofline["executed_mfma_tflops"] / cal["tflops"], 4)
        log(f"[bench] sustained bf16 MFMA rate (calibration kernel, every CU loaded): {cal['tflops']:.0f} TFLOP/s "
            f"({cal['frac_of_bf16_peak']:.3f} of the datasheet peak); the dominant kernel executes "
            f"{roofline['executed_frac_of_sustained']:.3f} of it")

    if args.eval_precision != "none":
        # The evaluation rows: psi and xi at every block centre (two contractions: psi and xi_x share
        # one, xi_y is the other) and the block potentials N_i (one contraction), from the
        # coefficients of the timed run; 1/2 sum_i N_i must equal the energy of those coefficients.
        ep = args.eval_precision
        wse = torch.empty(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=ep), dtype=torch.uint8, device=dev)
        pp.point_field(t[0], t[1], a, W=wl.W, H=wl.H, precision=ep, workspace=wse)
        pp.block_potential(*t, a, W=wl.W, H=wl.H, precision=ep, workspace=wse)
        torch.cuda.synchronize()
        pp.timing_enable(True)
        psi, xix, xiy = pp.point_field(t[0], t[1], a, W=wl.W, H=wl.H, precision=ep, workspace=wse)
        N = pp.block_potential(*t, a, W=wl.W, H=wl.H, precision=ep, workspace=wse)
        torch.cuda.synchronize()
        tp, cp = pp.timing_query("point")
        tn, cn = pp.timing_query("potential")
        pp.timing_enable(False)
        Ev = float(E.cpu())
        ident = abs(0.5 * float(N.sum().cpu()) - Ev) / abs(Ev)
        out["evaluation"] = {
            "precision": ep,
            "point_field_ms": tp, "point_field_contractions": cp,
            "point_field_pairs_per_s": pairs / (tp * 1e-3),
            "block_potential_ms": tn,
            "block_potential_pairs_per_s": pairs / (tn * 1e-3),
            "achieved_tflops_per_contraction": round(2.0 * pairs / ((tp + tn) / (cp + cn) * 1e-3) / 1e12, 2),
            "half_sum_N_vs_E": ident}
        log(f"[bench] evaluation ({ep}): point field {tp:.1f} ms ({cp} contractions), block potentials {tn:.1f} ms; "
            f"|1/2 sum N - E| / E = {ident:.2e}")

    m_bins = (wl.Mu if wl.Mu == wl.Mp else 0) if args.bins < 0 else args.bins
    if m_bins > 0:
        # The bin scheme of Sec. III-D at m x m bins and the same truncation M = m: its cost, and how
        # far its coefficients, its bin-centre potential and field and its block gradients (weighted
        # back from the bins) are from the direct sum's.
        Mb = min(m_bins, wl.Mu, wl.Mp)
        wsb = torch.empty(pp.bin_workspace_size(wl.W, wl.H, wl.n, m_bins, Mb, Mb), dtype=torch.uint8, device=dev)
        Pb = pp.bin_density(*t, W=wl.W, H=wl.H, m=m_bins, workspace=wsb)
        ab = pp.bin_coeffs(Pb, W=wl.W, H=wl.H, Mu=Mb, Mp=Mb, workspace=wsb)
        fb = pp.bin_field(ab, W=wl.W, H=wl.H, m=m_bins, workspace=wsb)
        pp.bin_interp(*t, None, fb[1], fb[2], W=wl.W, H=wl.H, workspace=wsb)
        torch.cuda.synchronize()
        pp.timing_enable(True)
        Pb = pp.bin_density(*t, W=wl.W, H=wl.H, m=m_bins, workspace=wsb)
        ab = pp.bin_coeffs(Pb, W=wl.W, H=wl.H, Mu=Mb, Mp=Mb, workspace=wsb)
        fb = pp.bin_field(ab, W=wl.W, H=wl.H, m=m_bins, workspace=wsb)
        _, gxb, gyb = pp.bin_interp(*t, None, fb[1], fb[2], W=wl.W, H=wl.H, workspace=wsb)
        torch.cuda.synchronize()
        td, _ = pp.timing_query("bin_density")
        tcf, _ = pp.timing_query("bin_coeffs")
        tf, _ = pp.timing_query("bin_field")
        ti, _ = pp.timing_query("bin_interp")
        pp.timing_enable(False)
        gemm_flops = 2.0 * m_bins * Mb * m_bins + 2.0 * Mb * Mb * m_bins + 2 * 2.0 * Mb * m_bins * Mb \
            + 3 * 2.0 * m_bins * m_bins * Mb
        if ref is not None:
            a_dir, g_dir, dir_name = ref[1], (ref[2], ref[3]), "fp64 direct sum (GPU)"
        else:
            a_dir, g_dir, dir_name = a, (gx, gy), f"{args.precision} direct sum (GPU)"
        a_dir = a_dir[:Mb, :Mb].contiguous()
        fd = pp.bin_field(a_dir, W=wl.W, H=wl.H, m=m_bins, workspace=wsb)
        abn, adn = ab.cpu().numpy(), a_dir.cpu().numpy()
        lo = min(64, Mb)
        gbin = np.concatenate([gxb.cpu().numpy(), gyb.cpu().numpy()])
        gdir = np.concatenate([g_dir[0].cpu().numpy(), g_dir[1].cpu().numpy()])
        bins = {"m": m_bins, "M": Mb, "density_ms": td, "coeffs_ms": tcf, "field_ms": tf, "interp_ms": ti,
                "total_ms": td + tcf + tf + ti,
                "transforms": "dense FP64 GEMMs against cos/sin tables (O(m^3) per transform), not the FFT of "
                              "Sec. III-D; the cost is that of this comparison path",
                "transform_gemm_tflops_fp64": round(gemm_flops / ((tcf + tf) * 1e-3) / 1e12, 2),
                "compared_with": dir_name,
                "coeffs_rel_diff": rel(abn, adn),
                f"coeffs_rel_diff_u_p_below_{lo}": rel(abn[:lo, :lo], adn[:lo, :lo]),
                "psi_rel_diff_at_bin_centres": rel(fb[0].cpu().numpy(), fd[0].cpu().numpy()),
                "xi_rel_diff_at_bin_centres": rel(np.concatenate([fb[1].cpu().numpy(), fb[2].cpu().numpy()]),
                                                  np.concatenate([fd[1].cpu().numpy(), fd[2].cpu().numpy()])),
                "block_gradient_rel_diff": rel(gbin, gdir)}
        out["bin_scheme"] = bins
        log(f"[bench] bin scheme m={m_bins}: density {td:.2f} ms, coefficients {tcf:.2f} ms, field {tf:.2f} ms, "
            f"interpolation {ti:.2f} ms; vs direct: a {bins['coeffs_rel_diff']:.3e}, "
            f"psi {bins['psi_rel_diff_at_bin_centres']:.3e}, xi {bins['xi_rel_diff_at_bin_centres']:.3e}, "
            f"block gradient {bins['block_gradient_rel_diff']:.3e}")

    # Accuracy against the FP64 path of the GPU (every element; per 64 x 64 coefficient tile and per
    # 256-block gradient tile as well, so that no tile hides behind the large low frequencies).
    if not args.no_accuracy and ref is not None:
        acc = errors_vs(ref, (E, a, gx, gy))
        out["rel_err"] = {"vs_fp64_gpu": acc}
        log(f"[bench] rel err vs fp64 GPU {acc}")

    if not args.no_cpu_baseline:
        # The CPU-baseline leg: the FP64 oracle on the host, timed on a bounded sample of the workload,
        # and (unless --no-accuracy) the oracle's direct sums of sampled coefficients, three in every
        # 256 x 256 tile, against which the GPU's coefficients are stated one by one (each scaled by
        # f_up sum_i |S'_iu T'_ip|, the magnitude that bounds the rounding of its sum).
        import oracle
        if not args.no_accuracy:
            rng = np.random.default_rng(12345)
            us, ps = [], []
            for u0 in range(0, wl.Mu, 256):
                for p0 in range(0, wl.Mp, 256):
                    for _ in range(3):
                        u, p = int(rng.integers(u0, min(u0 + 256, wl.Mu))), int(rng.integers(p0, min(p0 + 256, wl.Mp)))
                        if u or p:
                            us.append(u)
                            ps.append(p)
            us, ps = np.array(us), np.array(ps)
            t0 = time.perf_counter()
            ao, _, Rabs = oracle.coeffs_sampled_full(wl.W, wl.H, *wl.arrays(), us, ps)
            fac = oracle.coef_factors(wl.W, wl.H, wl.Mu, wl.Mp)[us, ps]
            log(f"[bench] oracle coefficient samples in {time.perf_counter() - t0:.1f} s")
            den = np.abs(fac) * Rabs
            runs = {args.precision: (E, a, gx, gy)}
            if ref is not None:
                runs["fp64"] = ref
            runs.update(fp8_runs)
            if mix_run is not None:
                runs["bf16mix"] = mix_run
            vs = {}
            for name, r in runs.items():
                an = r[1].cpu().numpy()[us, ps]
                e = np.abs(an - ao) / np.where(den > 0, den, 1.0)
                vs[name] = {"relative_norm": rel(an, ao), "scaled_max": float(e.max()), "scaled_median": float(np.median(e))}
            out.setdefault("rel_err", {})["sampled_coeffs_vs_oracle"] = {
                "sample": f"{len(us)} coefficients, three in every 256 x 256 tile, each a direct FP64 oracle sum over "
                          f"all {wl.n} blocks; scaled error |a - a*| / (f_up sum_i |S'_iu T'_ip|)", **vs}
            log(f"[bench] sampled coefficients vs oracle {vs}")
        rng = np.random.default_rng(777)
        idx = np.sort(rng.choice(wl.n, args.cpu_sample, replace=False))
        xs, ys, wsz, hs = (v[idx] for v in wl.arrays())
        t0 = time.perf_counter()
        Eo, ao, _ = oracle.energy(wl.W, wl.H, xs, ys, wsz, hs, wl.Mu, wl.Mp)
        oracle.grad(wl.W, wl.H, xs, ys, wsz, hs, ao)
        tc = time.perf_counter() - t0
        cp = args.cpu_sample * wl.Mu * wl.Mp
        out["cpu_baseline"] = {"value": cp / tc, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"energy + gradient of {args.cpu_sample} blocks drawn (seeded) from the "
                                         f"{wl.n}-block workload at the full {wl.Mu}x{wl.Mp} truncation, FP64 "
                                         f"direct summation; {tc:.1f} s",
                               "seconds": tc}
        log(f"[bench] oracle: {tc:.1f} s for {cp:.3e} pairs on {oracle.num_threads()} threads ({cpu_model()})")
        # one core, beside the paper's single-threaded setting: a smaller sample of the same work
        threads = oracle.num_threads()
        k1 = max(1, args.cpu_sample // 30)
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        _, a1, _ = oracle.energy(wl.W, wl.H, xs[:k1], ys[:k1], wsz[:k1], hs[:k1], wl.Mu, wl.Mp)
        oracle.grad(wl.W, wl.H, xs[:k1], ys[:k1], wsz[:k1], hs[:k1], a1)
        t1 = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        out["cpu_baseline"]["single_thread"] = {"value": k1 * wl.Mu * wl.Mp / t1, "unit": "pairs/s", "cores": 1,
                                                "sample": f"the first {k1} blocks of the same sample; {t1:.1f} s"}
        log(f"[bench] oracle on one thread: {t1:.1f} s for {k1 * wl.Mu * wl.Mp:.3e} pairs")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
