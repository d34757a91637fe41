#!/usr/bin/env python3
"""Throughput of the SSP-RK3 SRMHD step on one MI355X.

Workload: the circularly polarised Alfven wave on the box diagonal,
k = 2 pi (1,1,1), 512^3 cells (--n), rho = p = B0 = eta = 1, gamma 4/3, CFL 0.5,
plain FP64 state (5 conserved + 3 staggered B + Newton guess W), MP5 + HLL +
UCT + SSP-RK3.  A step is one full RK3 step (3 stages) over the whole box;
the metric is cell updates per second (N^3 steps / s).

Prints one JSON line.  Besides the contract keys it carries:
  roofline      -- the dominant kernel (largest share of the step) with its
                   algorithmic bytes and flops per launch over its average
                   duration from HIP events recorded on the library's stream
                   during a second, instrumented run of the same steps;
  stream_copy_gbs, hbm_roofline_frac_step_vs_copy
                -- the measured bandwidth of a plain 2 GiB device copy, and the
                   step-level HBM fraction (state bytes per cell-step x rate)
                   against it as well as against the 8 TB/s peak;
  copy_floor    -- the bytes every kernel of a step must move, intermediates
                   included (the per-unit figures below times each class's
                   launches), the time a plain copy would take to move them,
                   and that time over the measured step;
  cpu_baseline  -- the FP64 CPU oracle timed on this host on a bounded sample
                   (the same wave at 64^3, a few steps, all cores; then one
                   thread);
  forms         -- the same wave at 512^3 in the FP64 and mixed forms, each
                   also with HO, with MC + SSP-RK2 and with the learned Newton
                   guess (rate, step-level HBM fraction, per-kernel ms), and
                   the learned guess's iteration report on 512^3 turbulence.
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
# Algorithmic HBM bytes per cell-step of the state (FP64): each stage reads
# the state (and U^n after the first stage) and W and writes the state and W:
# SSP-RK3 144 + 208 + 208, SSP-RK2 144 + 208.
STEP_BYTES = 560.0
STEP_BYTES_RK2 = 352.0

# State bytes per cell of each kernel class: the evolved arrays (the 8 state
# arrays and W, FP64 in every form) it must read or write, once, averaged over
# the class's launches in a step -- the per-cell-step traffic of the state,
# 560 B over a step, apportioned to the kernels that touch it.  update: reads
# the stage's input state (64 B) and, in stages 2 and 3, U^n (64 B), writes
# the stage's output (64 B): (128 + 192 + 192)/3.  c2p: reads the state and W,
# writes W.  The flux and UCT passes touch no state array beyond the normal
# face B (their operands are intermediates; flux_xy reads two of them).  The
# roofline's achieved bandwidth and fraction use these bytes.
STATE_BYTES = {"c2p": 80.0, "flux_xy": 16.0, "flux_z": 8.0,
               "uct_x": 16.0, "uct_y": 16.0, "uct_z": 16.0, "update": 512.0 / 3,
               "update_c2p": 176.0}
# With the fused update + inversion (stages 1 and 2: 128 + 16 and 192 + 16 B,
# W included), the plain update runs in stage 3 only.
STATE_BYTES_FUSED_UPDATE = 192.0

# Bytes and FP64/FP32 arithmetic operations per unit (cell, face or edge) of
# each kernel class with its intermediates, for the plain FP64 form and the
# mixed form (FP32 primitives, face arrays and face-B copies), averaged over
# the class's launches in one step (reported beside the state-byte roofline).
# Bytes: every array element the kernel must read or write, once.  flux_xy
# (per cell: its x and its y face): the 8 primitives and the two normal face B
# in, per face 5 fluxes + a+- + 4 face velocities out.  flux_z: 7 primitives
# + normal B in, 11 face arrays out (the pass of stage 1 also reads the x and
# y speeds for the CFL sum: (184 + 152 + 152)/3).  uct_k (one edge
# orientation): the 4 velocities of the P faces, B_P and B_Q, and a+- of the
# P and Q faces in, E_k (FP64) out.  c2p: the state and W in; the primitives,
# W (and, mixed, the FP32 face-B copies) out.  update: stage 1 reads 15
# fluxes, 3 edge fields and U^n and writes the RK register; stages 2 and 3
# also read U^n ((272 + 336 + 336)/3).  Flops: adds, multiplies, divides and
# square roots of the formulas (FMA = 2), MP5 counted on its limiter path (49
# per call, 14 calls per face, 12 per edge).
KERNEL_UNITS = {
    # class: (bytes fp64, bytes mixed, flops per unit)
    "c2p": (144.0, 124.0, 200.0),
    "flux_xy": (256.0, 128.0, 1880.0),
    "flux_z": (488.0 / 3, 244.0 / 3, 940.0),
    "uct_x": (88.0, 48.0, 640.0),
    "uct_y": (88.0, 48.0, 640.0),
    "uct_z": (88.0, 48.0, 640.0),
    "update": (944.0 / 3, 764.0 / 3, 80.0),
    # the update fused with the next stage's inversion (stages 1 and 2): also
    # writes the primitives (FP64, or FP32 in the mixed form, with the FP32
    # face-B copies) and reads and writes W
    "update_c2p": ((272.0 + 336.0) / 2 + 80.0, (212.0 + 276.0) / 2 + 60.0, 280.0),
}
# the plain update in stage 3 only (when stages 1 and 2 run fused)
KERNEL_UNITS_FUSED_UPDATE = (336.0, 276.0, 80.0)
# rocprofv3 kernel names of each class's FP64 launches in one step (name,
# launches per step), for the HBM traffic read from the profiles (the mixed
# form's names have float for double, and the x-y flux kernel's tile is 64x8)
PROFILED_KERNEL = {
    "c2p": [("k_c2p<false, false, false>", 1)],
    "flux_xy": [("k_flux_xy<double, false, 0, 4>", 3)],
    "flux_z": [("k_flux<2, double, true, false, 0, true>", 1),
               ("k_flux<2, double, false, false, 0, true>", 2)],
    "uct_x": [("k_uct<0, double, 0, true>", 3)],
    "uct_y": [("k_uct<1, double, 0, true>", 3)],
    "uct_z": [("k_uct<2, double, 0, true>", 3)],
    "update": [("k_update<3, double>", 1)],
    "update_c2p": [("k_update_c2p<1, double, false>", 1), ("k_update_c2p<2, double, false>", 1)],
}


def profiled_name(name, mixed):
    """The rocprofv3 name of an FP64 kernel's launch in the given form."""
    if not mixed:
        return name
    if name.startswith("k_flux_xy<"):
        return "k_flux_xy<float, false, 0, 8>"
    return name.replace("double", "float")


KERNEL_SOURCES = ("srmhd_kernels.hip", "srmhd_kernels.hpp", "srmhd_phys.hpp")


def kernel_sources_sha():
    """sha256[:16] over the stage kernels' sources, in KERNEL_SOURCES order."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2401_03008_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel_cls, workload):
    """Bytes per launch of class `kernel_cls` leaving the L2 (HBM or the
    memory-side cache), averaged over its launches in one step, from the
    committed rocprofv3 summary of `workload` (e.g. "cpa512 fp64"): FETCH_SIZE
    and WRITE_SIZE scaled by a plain copy's readings, the reads cross-checked
    against the 128/64/32-byte request counts; None when there is no such
    summary or the kernel sources changed since the counters were taken."""
    import glob
    sha = kernel_sources_sha()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        txt = open(f).read()
        if f"kernel sources sha256[:16]: {sha}" not in txt or f"workload: {workload}\n" not in txt:
            continue
        got = {}
        for line in txt.splitlines():
            if line.startswith("traffic_bytes_per_launch "):
                name, val = line[len("traffic_bytes_per_launch "):].rsplit(":", 1)
                got[name.strip()] = int(val)
        parts = [(profiled_name(k, workload.endswith("mixed")), w)
                 for k, w in PROFILED_KERNEL[kernel_cls]]
        if all(k in got for k, _ in parts):
            return int(sum(got[k] * w for k, w in parts) / sum(w for _, w in parts))
    return None


def step_bytes_with_intermediates(kernels, steps, precision):
    """Bytes per cell and step that the timed kernels must move, intermediates
    included: each class's per-unit bytes (KERNEL_UNITS) times its launches
    per step.  `kernels`: {class: {"launches": ...}} over `steps` steps."""
    col = 1 if precision == "mixed" else 0
    fused = "update_c2p" in kernels
    total = 0.0
    for k, v in kernels.items():
        if k in KERNEL_UNITS:
            u = KERNEL_UNITS_FUSED_UPDATE if (fused and k == "update") else KERNEL_UNITS[k]
            total += u[col] * v["launches"] / steps
    return total


def stream_copy_gbs(gib=2, reps=5):
    """Measured HBM bandwidth of a plain device copy of `gib` GiB (read +
    write bytes over the average of `reps` copies, HIP events): the practical
    ceiling the step-level fraction is also quoted against."""
    import torch
    nb = gib * (1 << 30)
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nb / (ms / 1e3) / 1e9


def run_form(n, precision, steps, warmup, mlp=None, guess="mlp", **scheme):
    """Mcell-updates/s of one form on the diagonal CPA at n^3 (mlp: the
    learned Newton guess, in mode `guess`; scheme: recon / time_order /
    high_order), then Newton statistics over 2 more steps."""
    import torch
    from paper_2401_03008_amd import inputs
    from paper_2401_03008_amd.solver import Solver
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    S = Solver(n, precision=precision, collect_stats=False, **scheme)
    S.init(prim5, bf)
    del prim5, bf
    if mlp is not None:
        S.set_mlp(mlp)
        S.set_guess(guess)
    S.step(warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(S.stream)
    S.step(steps)
    e1.record(S.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    S.kernel_timing(True)
    S.step(2)
    kt = S.kernel_times()
    S.close()
    # Newton statistics of the same form (a separate run with counters on)
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    S2 = Solver(n, precision=precision, collect_stats=True, **scheme)
    S2.init(prim5, bf)
    del prim5, bf
    if mlp is not None:
        S2.set_mlp(mlp)
        S2.set_guess(guess)
    S2.step(2)
    d = S2.diagnostics()
    S2.close()
    del S, S2
    torch.cuda.empty_cache()
    v = n ** 3 * steps / (ms / 1e3) / 1e6
    sb = STEP_BYTES_RK2 if scheme.get("time_order", 3) == 2 else STEP_BYTES
    return {"cells": n ** 3, "steps": steps, "ms_per_step": round(ms / steps, 3),
            "Mcell_updates_per_s": round(v, 1),
            "hbm_roofline_frac_step": round(v * 1e6 * sb / (HBM_PEAK_GBS * 1e9), 4),
            "newton_mean_iters": round(d["newton_iters"] / max(d["newton_calls"], 1), 3),
            "mlp_fallback_rate": round(d["mlp_fallbacks"] / max(d["newton_calls"], 1), 5),
            "kernel_ms": {k: round(t / c, 4) for k, (t, c) in kt.items() if c}}


def workload_label(n, precision="fp64", high_order=False, recon="mp5", time_order=3,
                   guess="prev"):
    """config.workload of the timed run: what the timed steps compute."""
    scheme = ("point-value MP5, sixth-order INT/DER (HO)" if high_order else
              ("MP5" if recon == "mp5" else "linear MC"))
    prec = "FP64" if precision == "fp64" else "FP64 state, FP32 REC and face fluxes"
    g = {"prev": "previous-W", "mlp": "learned (where no usable previous W)",
         "mlp_all": "learned (every cell)", "cold": "cold"}[guess]
    return (f"CPA Alfven wave on the box diagonal, {n}^3, {prec}, {scheme} + HLL + UCT + "
            f"SSP-RK{time_order}, CFL 0.5, {g} Newton guess")


def cpu_baseline(seconds_target=15.0):
    """The oracle (as it stands) on the same wave at 64^3, on all host cores,
    then on one thread."""
    import oracle
    from paper_2401_03008_amd import inputs
    oracle.build(force=False)
    n = 64
    prim5, bf, _ = inputs.cpa(n, diagonal=True)
    g = oracle.Grid(n)

    def rate(max_steps):
        cons, W = g.init(prim5, bf)
        t0 = time.perf_counter()
        g.step(cons, bf, W, 1)
        one = time.perf_counter() - t0
        nsteps = max(1, min(max_steps, int(seconds_target / max(one, 1e-3))))
        t0 = time.perf_counter()
        g.step(cons, bf, W, nsteps)
        el = time.perf_counter() - t0
        return n ** 3 * nsteps / el / 1e6, nsteps, el

    cores = oracle.num_threads()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    v, nsteps, el = rate(200)  # about seconds_target of work on all cores
    oracle.set_num_threads(1)
    v1, nsteps1, el1 = rate(3)
    oracle.set_num_threads(cores)
    return {"value": v, "unit": "Mcell-updates/s", "cores": cores, "cpu_model": model,
            "kind": "oracle",
            "sample": f"diagonal CPA {n}^3, {nsteps} RK3 steps after 1 warm-up step, FP64, "
                      f"OpenMP over z ({el:.1f} s)",
            "single_thread_value": v1,
            "single_thread_sample": f"same wave, {nsteps1} steps on 1 thread ({el1:.1f} s)"}


def _newton_row(d):
    h = d["newton_hist"]
    tot = max(sum(h), 1)
    cdf, acc = [], 0
    for c in h:
        acc += c
        cdf.append(acc / tot)
    return {"mean_iters": round(d["newton_iters"] / max(d["newton_calls"], 1), 3),
            "p50": next(i for i, c in enumerate(cdf) if c >= 0.5),
            "p99": next(i for i, c in enumerate(cdf) if c >= 0.99),
            "fallback_rate": round(d["mlp_fallbacks"] / max(d["newton_calls"], 1), 5),
            "c2p_failures": d["c2p_failures"], "rc": d["rc"]}


def newton_report_turbulence(n, mlp, steps=4):
    """Newton iterations per inversion on the turbulence set-up at n^3
    (sigma0 = 10, Gamma up to 5), all from the same state (2 steps in).
    Warm, over `steps` steps: the previous-step W, the learned guess where no
    usable previous W exists ("mlp": the previous W everywhere here), the
    network first in every cell ("mlp_all"), and a cold start (W0 = U);
    mean/p50/p99 iterations, fallback rate, k_c2p ms, and each run's L1
    difference from the previous-W run.  Restart, the inversion of the
    conserved state alone (no W): the method without the network (a start
    from U) and the learned guess."""
    import torch
    from paper_2401_03008_amd import inputs
    from paper_2401_03008_amd.solver import Solver
    prim5, bf = inputs.turbulence(n, sigma0=10.0, gamma_max=5.0, device="cuda")
    rows, ref = {}, None
    runs = [(g, False, steps) for g in ("prev", "mlp", "mlp_all", "cold")] + \
        [(g, True, 0) for g in ("prev", "mlp")]
    for guess, restart, nst in runs:
        S = Solver(n, pfloor=1e-10, collect_stats=True)
        S.init(prim5, bf)
        S.step(2)
        if restart:
            st = S.get_state()
            S.set_state(st["cons"], st["bface"], None, st["t"], st["step"])
            del st
        S.set_mlp(mlp)
        S.set_guess(guess)
        S.reset_counters()
        S.kernel_timing(True)
        if restart:
            S.primitives()  # one inversion of every cell
        else:
            S.step(nst)
        kt = S.kernel_times()
        S.kernel_timing(False)
        d = S.diagnostics(raise_on_error=False)
        S.set_guess("prev")
        row = _newton_row(d)
        row["c2p_ms"] = round(kt["c2p"][0] / max(kt["c2p"][1], 1), 4)
        if not restart:  # all kernels, per step (the fused updates invert too)
            row["step_ms"] = round(sum(v[0] for v in kt.values()) / nst, 3)
        key = ("restart_" if restart else "") + guess
        if not restart:
            P = S.primitives()
            if guess == "prev":
                ref = P
            else:
                row["l1_rel_vs_prev"] = float((P - ref).abs().sum() / ref.abs().sum())
                del P
        rows[key] = row
        S.close()
        del S
        torch.cuda.empty_cache()
    del ref, prim5, bf
    torch.cuda.empty_cache()
    rows["workload"] = (f"turbulence {n}^3, sigma0 = 10, Gamma <= 5: {steps} steps after 2 "
                        "(warm), or one inversion after 2 steps of the conserved state "
                        "without W (restart_*)")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--stats", action="store_true", help="collect Newton statistics while timed")
    ap.add_argument("--high-order", action="store_true",
                    help="HO: sixth-order INT and DER, point-value MP5 (the timed run; with "
                         "this or --recon mc the roofline's flop counts stay those of the "
                         "default scheme)")
    ap.add_argument("--recon", default="mp5", choices=["mp5", "mc"])
    ap.add_argument("--time-order", type=int, default=3, choices=[2, 3])
    ap.add_argument("--guess", default="prev", choices=["prev", "mlp", "mlp_all"],
                    help="Newton guess of the timed run: the previous W, or the learned "
                         "network (trained first by the library's kernels) where no usable "
                         "previous W exists / first in every cell")
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
              "multi-GPU domain decomposition is not implemented.", file=sys.stderr)
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
    workload = workload_label(n, args.precision, args.high_order, args.recon, args.time_order,
                              args.guess)
    print(f"[bench] building the {n}^3 diagonal CPA", file=sys.stderr, flush=True)
    prim5, bf, _ = inputs.cpa(n, diagonal=True, device="cuda")
    step_bytes = STEP_BYTES if args.time_order == 3 else STEP_BYTES_RK2
    S = Solver(n, precision=args.precision, collect_stats=args.stats, recon=args.recon,
               time_order=args.time_order, high_order=args.high_order)
    S.init(prim5, bf)
    del prim5, bf
    if args.guess in ("mlp", "mlp_all"):
        from paper_2401_03008_amd.learned import train_default
        net = train_default()[0]
        S.set_mlp(net)
        S.set_guess(args.guess)
        print("[bench] learned guess trained and set", file=sys.stderr, flush=True)
    S.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # the timed region: K steps between HIP events on the library's stream,
    # three times; the median run is the value
    stream = S.stream
    runs = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        S.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1))
    ms = sorted(runs)[1]
    ms_per_step = ms / args.steps
    value = n ** 3 * args.steps / (ms / 1e3) / 1e6
    diag = S.diagnostics()
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} Mcell/s",
          file=sys.stderr, flush=True)

    roof = None
    floor = None
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
        fused = "update_c2p" in kernels
        b64, bmx, fl = (KERNEL_UNITS_FUSED_UPDATE if (fused and dom == "update")
                        else KERNEL_UNITS[dom])
        units = n ** 3
        avg_s = kernels[dom]["avg_ms"] / 1e3
        bytes_with_inter = (bmx if args.precision == "mixed" else b64) * units
        sb = STATE_BYTES_FUSED_UPDATE if (fused and dom == "update") else STATE_BYTES[dom]
        bytes_per = sb * units
        flops_per = fl * units
        gbs = bytes_per / avg_s / 1e9
        gbs_inter = bytes_with_inter / avg_s / 1e9
        tfl = flops_per / avg_s / 1e12
        fpeak = FP32_PEAK_TFLOPS if (args.precision == "mixed" and dom.startswith("flux")) else FP64_PEAK_TFLOPS
        # the roof that binds is the one with the larger minimum time for the
        # kernel's algorithmic bytes (the state arrays it must touch) and its
        # algorithmic flops; a pass whose operands are all intermediates (the
        # face fluxes) is bound by its arithmetic
        if bytes_per / (HBM_PEAK_GBS * 1e9) >= flops_per / (fpeak * 1e12):
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
        else:
            roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": fpeak,
                    "unit": "TFLOP/s", "frac": round(tfl / fpeak, 4), "traffic": None}
        default_scheme = (not args.high_order and args.recon == "mp5" and args.time_order == 3
                          and args.guess == "prev")
        if default_scheme:
            roof["traffic"] = profiled_traffic(dom, f"cpa{n} {args.precision}")
        roof.update({"kernel": dom, "avg_ms": round(kernels[dom]["avg_ms"], 4),
                     "alg_bytes_per_launch": bytes_per, "state_bytes_per_cell": sb,
                     "alg_flops_per_launch": flops_per,
                     "alu_tflops": round(tfl, 3), "hbm_gbs": round(gbs, 1),
                     "bytes_with_intermediates_per_launch": bytes_with_inter,
                     "achieved_with_intermediates_gbs": round(gbs_inter, 1),
                     "frac_with_intermediates": round(gbs_inter / HBM_PEAK_GBS, 4)})
        if default_scheme:
            floor = {"bytes_per_cell_step":
                     round(step_bytes_with_intermediates(kernels, args.steps, args.precision), 1)}
        print(f"[bench] kernel timing: {json.dumps(kernels)}", file=sys.stderr, flush=True)
    S.close()
    copy_gbs = stream_copy_gbs()
    print(f"[bench] plain device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    if floor is not None:
        fms = floor["bytes_per_cell_step"] * n ** 3 / (copy_gbs * 1e9) * 1e3
        floor.update({"copy_ms_per_step": round(fms, 3),
                      "frac_of_step": round(fms / ms_per_step, 4)})

    forms = None
    if not args.no_forms:
        from paper_2401_03008_amd.learned import train_default
        forms = {}
        for prec in ("fp64", "mixed"):
            print(f"[bench] form {prec} at {args.forms_n}^3", file=sys.stderr, flush=True)
            forms[prec] = run_form(args.forms_n, prec, max(5, args.steps // 2), 2)
        # the paper's two other configurations: HO = YES (with UCT), and
        # second-order time stepping with linear reconstruction
        for prec in ("fp64", "mixed"):
            for key, form_scheme in (("ho", dict(high_order=True)),
                                     ("mc+rk2", dict(recon="mc", time_order=2))):
                name = f"{prec}+{key}"
                print(f"[bench] form {name} at {args.forms_n}^3", file=sys.stderr, flush=True)
                forms[name] = run_form(args.forms_n, prec, max(5, args.steps // 2), 2,
                                       **form_scheme)
        print("[bench] training the learned guess", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        mlp, hist, npairs = train_default()
        train_s = time.perf_counter() - t0
        for prec in ("fp64", "mixed"):
            for key, gmode in ((f"{prec}+learned", "mlp"), (f"{prec}+learned_all", "mlp_all")):
                print(f"[bench] form {key} at {args.forms_n}^3", file=sys.stderr, flush=True)
                forms[key] = run_form(args.forms_n, prec, max(5, args.steps // 2), 2, mlp=mlp,
                                      guess=gmode)
        forms["learned_training"] = {"pairs": npairs, "adam_steps": 1500, "batch": 4096,
                                     "final_loss": hist[-1][1], "seconds": round(train_s, 2)}
        print(f"[bench] Newton report, turbulence {args.forms_n}^3", file=sys.stderr, flush=True)
        forms["newton_turbulence"] = newton_report_turbulence(args.forms_n, mlp)

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
        "ms_per_step_runs": [round(r / args.steps, 4) for r in runs],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 state + f32 REC/flux",
        "data": "synthetic",
        "config": {"workload": workload,
                   "cells": n ** 3, "precision": args.precision, "guess": args.guess,
                   "newton_stats": bool(args.stats)},
        "hbm_roofline_frac_step": round(value * 1e6 * step_bytes / (HBM_PEAK_GBS * 1e9), 4),
        "stream_copy_gbs": round(copy_gbs, 1),
        "hbm_roofline_frac_step_vs_copy": round(value * 1e6 * step_bytes / (copy_gbs * 1e9), 4),
        "roofline": roof,
        "copy_floor": floor,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "forms": forms,
        "final_step_dt": diag["dt"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
