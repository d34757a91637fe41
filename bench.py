#!/usr/bin/env python3
"""Throughput of the SSP-RK3 SRMHD step on one MI355X.

Workload: the circularly polarised Alfven wave on the box diagonal,
k = 2 pi (1,1,1), 256^3 cells, rho = p = B0 = eta = 1, gamma 4/3, CFL 0.5,
plain FP64 state (5 conserved + 3 staggered B + Newton guess W), MP5 + HLL +
UCT + SSP-RK3.  A step is one full RK3 step (3 stages) over the whole box;
the metric is cell updates per second (N^3 steps / s).

Prints one JSON line.  Besides the contract keys it carries:
  roofline      -- the dominant kernel (largest share of the step) with its
                   algorithmic bytes and flops per launch over its average
                   duration from HIP events recorded on the library's stream
                   during a second, instrumented run of the same steps;
  cpu_baseline  -- the FP64 CPU oracle timed on this host on a bounded sample
                   (the same wave at 64^3, a few steps, all cores).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector (packed)
STEP_BYTES = 560.0          # algorithmic HBM bytes per cell-step of the state

# Algorithmic HBM bytes and FP64/FP32 arithmetic operations per unit (cell,
# face or edge) of each kernel, for the plain FP64 form and the mixed form.
# Bytes: every array element the kernel must read or write, once.  Flops:
# adds, multiplies, divides and square roots of the formulas (FMA = 2), MP5
# counted on its limiter path (49 per call, 14 calls per face, 12 per edge;
# the UCT kernel computes the three edges of a cell).
KERNEL_UNITS = {
    # class: (bytes fp64, bytes mixed, flops per unit)
    "c2p": (144.0, 112.0, 200.0),
    "flux_x": (168.0, 88.0, 940.0),
    "flux_y": (168.0, 88.0, 940.0),
    "flux_z": (168.0, 88.0, 940.0),
    "uct": (192.0, 120.0, 1920.0),
    "update": (336.0, 276.0, 80.0),
}


def profiled_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3
    summaries (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings),
    or None when the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2401_03008_amd", "csrc", "srmhd_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        txt = open(f).read()
        if f"srmhd_kernels.hip: {sha}" not in txt:
            continue
        for line in txt.splitlines():
            if line.startswith("traffic_bytes_per_launch ") and kernel_name in line:
                return int(line.rsplit(":", 1)[1])
    return None


def run_form(n, precision, steps, warmup, mlp=None):
    """Mcell-updates/s of one form on the diagonal CPA at n^3 (mlp: the
    learned Newton guess), then Newton statistics over 2 more steps."""
    import torch
    from paper_2401_03008_amd import inputs
    from paper_2401_03008_amd.solver import Solver
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    S = Solver(n, precision=precision, collect_stats=False)
    S.init(prim5, bf)
    del prim5, bf
    if mlp is not None:
        S.set_mlp(mlp)
        S.set_guess("mlp")
    S.step(warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(S.stream)
    S.step(steps)
    e1.record(S.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    S.close()
    # Newton statistics of the same form (a separate run with counters on)
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    S2 = Solver(n, precision=precision, collect_stats=True)
    S2.init(prim5, bf)
    del prim5, bf
    if mlp is not None:
        S2.set_mlp(mlp)
        S2.set_guess("mlp")
    S2.step(2)
    d = S2.diagnostics()
    S2.close()
    del S, S2
    torch.cuda.empty_cache()
    v = n ** 3 * steps / (ms / 1e3) / 1e6
    return {"cells": n ** 3, "steps": steps, "ms_per_step": round(ms / steps, 3),
            "Mcell_updates_per_s": round(v, 1),
            "hbm_roofline_frac_step": round(v * 1e6 * STEP_BYTES / (HBM_PEAK_GBS * 1e9), 4),
            "newton_mean_iters": round(d["newton_iters"] / max(d["newton_calls"], 1), 3),
            "mlp_fallback_rate": round(d["mlp_fallbacks"] / max(d["newton_calls"], 1), 5)}


def cpu_baseline(seconds_target=15.0):
    """The oracle (as it stands) on the same wave at 64^3, all host cores."""
    import oracle
    from paper_2401_03008_amd import inputs
    oracle.build(force=False)
    n = 64
    prim5, bf, _ = inputs.cpa(n, diagonal=True)
    g = oracle.Grid(n)
    cons, W = g.init(prim5, bf)
    t0 = time.perf_counter()
    g.step(cons, bf, W, 1)
    one = time.perf_counter() - t0
    nsteps = max(1, min(8, int(seconds_target / max(one, 1e-3))))
    t0 = time.perf_counter()
    g.step(cons, bf, W, nsteps)
    el = time.perf_counter() - t0
    return {"value": n ** 3 * nsteps / el / 1e6, "unit": "Mcell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"diagonal CPA {n}^3, {nsteps} RK3 steps after 1 warm-up step, FP64, "
                      f"OpenMP over z ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--stats", action="store_true", help="collect Newton statistics while timed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the per-form runs (plain FP64 and mixed) at --forms-n")
    ap.add_argument("--forms-n", type=int, default=512)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (a reference "
                         "kernel for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU decomposition is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_03008_amd import inputs
    from paper_2401_03008_amd.solver import Solver

    if args.copy_calibration:
        nb = args.copy_calibration * (1 << 20)
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.copy_calibration} MiB done",
              file=sys.stderr, flush=True)
        del src, dst

    n = args.n
    print(f"[bench] building the {n}^3 diagonal CPA", file=sys.stderr, flush=True)
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    S = Solver(n, precision=args.precision, collect_stats=args.stats)
    S.init(prim5, bf)
    del prim5, bf
    S.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({args.warmup} steps)", file=sys.stderr, flush=True)

    stream = S.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    S.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = n ** 3 * args.steps / (ms / 1e3) / 1e6
    diag = S.diagnostics()
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} Mcell/s",
          file=sys.stderr, flush=True)

    roof = None
    kernels = {}
    if not args.no_kernel_timing:
        S.kernel_timing(True)
        S.step(args.steps)
        kt = S.kernel_times()
        S.kernel_timing(False)
        tot = sum(v[0] for v in kt.values())
        for k, (kms, cnt) in kt.items():
            if cnt:
                kernels[k] = {"avg_ms": kms / cnt, "launches": cnt, "share": kms / tot}
        dom = max((k for k in kernels if k in KERNEL_UNITS), key=lambda k: kt[k][0])
        b64, bmx, fl = KERNEL_UNITS[dom]
        units = n ** 3
        avg_s = kernels[dom]["avg_ms"] / 1e3
        bytes_per = (bmx if args.precision == "mixed" else b64) * units
        flops_per = fl * units
        gbs = bytes_per / avg_s / 1e9
        tfl = flops_per / avg_s / 1e12
        fpeak = FP32_PEAK_TFLOPS if (args.precision == "mixed" and dom.startswith("flux")) else FP64_PEAK_TFLOPS
        # the roof that binds is the one with the larger minimum time
        if bytes_per / (HBM_PEAK_GBS * 1e9) >= flops_per / (fpeak * 1e12):
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
        else:
            roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": fpeak,
                    "unit": "TFLOP/s", "frac": round(tfl / fpeak, 4), "traffic": None}
        if args.precision == "fp64" and n == 256:
            dom_name = {"update": "k_update<2, double>"}.get(dom)
            tr = profiled_traffic(dom_name) if dom_name else None
            roof["traffic"] = tr
        roof.update({"kernel": dom, "avg_ms": round(kernels[dom]["avg_ms"], 4),
                     "alg_bytes_per_launch": bytes_per, "alg_flops_per_launch": flops_per,
                     "alu_tflops": round(tfl, 3), "hbm_gbs": round(gbs, 1)})
        print(f"[bench] kernel timing: {json.dumps(kernels)}", file=sys.stderr, flush=True)
    S.close()

    forms = None
    if not args.no_forms:
        from paper_2401_03008_amd.learned import train_default
        forms = {}
        for prec in ("fp64", "mixed"):
            print(f"[bench] form {prec} at {args.forms_n}^3", file=sys.stderr, flush=True)
            forms[prec] = run_form(args.forms_n, prec, max(5, args.steps // 2), 2)
        print("[bench] training the learned guess", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        mlp, hist, npairs = train_default()
        train_s = time.perf_counter() - t0
        for prec in ("fp64", "mixed"):
            key = f"{prec}+learned"
            print(f"[bench] form {key} at {args.forms_n}^3", file=sys.stderr, flush=True)
            forms[key] = run_form(args.forms_n, prec, max(5, args.steps // 2), 2, mlp=mlp)
        forms["learned_training"] = {"pairs": npairs, "adam_steps": 1500, "batch": 4096,
                                     "final_loss": hist[-1][1], "seconds": round(train_s, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    line = {
        "metric": "Mcell-updates/s per RK step (3D SRMHD) + HBM-roofline fraction, plain vs mixed",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 state + f32 REC/flux",
        "data": "synthetic",
        "config": {"workload": f"CPA Alfven wave on the box diagonal, {n}^3, FP64 state, "
                               f"MP5 + HLL + UCT + SSP-RK3, CFL 0.5",
                   "cells": n ** 3, "precision": args.precision,
                   "newton_stats": bool(args.stats)},
        "hbm_roofline_frac_step": round(value * 1e6 * STEP_BYTES / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "forms": forms,
        "final_step_dt": diag["dt"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
