"""Long-run driver for the decaying-turbulence set-up: steps the solver in one
form (FP64 or mixed, previous-step or learned Newton guess) and logs
max|div_h B|, Newton statistics and shell-binned spectra of v and B.

The spectra are diagnostics off the hot path (torch FFT on the primitives the
library returns); every step of the solver runs in libsrmhd.
"""
from __future__ import annotations

import math
import time

import torch

from . import inputs
from .solver import Solver


def shell_spectrum(fields, nbins=None, groups=4096):
    """E(k) = sum over |k| in [k - 1/2, k + 1/2) of |FFT(f)|^2 / N^2, summed
    over the components in `fields` (list of (nz, ny, nx) tensors); k in units
    of the box wave number.  The shell sums are accumulated into `groups`
    interleaved copies of the bins (mode index mod groups) and then added,
    so that no bin takes more than ~N/groups atomic additions."""
    nz, ny, nx = fields[0].shape
    dev = fields[0].device
    kx = torch.fft.rfftfreq(nx, d=1.0 / nx, device=dev)
    ky = torch.fft.fftfreq(ny, d=1.0 / ny, device=dev)
    kz = torch.fft.fftfreq(nz, d=1.0 / nz, device=dev)
    nbins = nbins or int(min(m for m in (nx, ny, nz) if m > 1) // 2)
    K = torch.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    gid = torch.round(K).long().clamp_(max=nbins).reshape(-1)
    del K
    gid.add_(torch.arange(gid.numel(), device=dev).remainder_(groups).mul_(nbins + 1))
    # rfft keeps half the x spectrum: weight the doubled modes
    w = torch.full((nx // 2 + 1,), 2.0, device=dev, dtype=torch.float64)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    N = float(nx * ny * nz)
    E = torch.zeros(groups * (nbins + 1), dtype=torch.float64, device=dev)
    for f in fields:
        F = torch.fft.rfftn(f - f.mean())
        P = (F.real ** 2 + F.imag ** 2) * w[None, None, :] / (N * N)
        del F
        E.index_add_(0, gid, P.reshape(-1))
        del P
    del gid
    return E.view(groups, nbins + 1).sum(0)[1:nbins].cpu()


def turbulence_run(n, steps, precision="fp64", mlp=None, sigma0=10.0, gamma_max=5.0,
                   log_every=10, spectrum_every=100, device="cuda", verbose=True):
    """Run the turbulence set-up at n^3; returns a dict of logs."""
    prim5, bf = inputs.turbulence(n, sigma0=sigma0, gamma_max=gamma_max, device=device)
    torch.cuda.empty_cache()  # the generator's temporaries, before the solver's large blocks
    S = Solver(n, precision=precision, pfloor=1e-10, collect_stats=True, device=device)
    S.init(prim5, bf)
    del prim5, bf
    torch.cuda.empty_cache()
    if mlp is not None:
        S.set_mlp(mlp)
        S.set_guess("mlp")
    log = {"n": n, "precision": precision, "learned": mlp is not None, "divb": [], "spectra": [],
           "newton": None}
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        if done % spectrum_every == 0:
            P = S.primitives()
            ev = shell_spectrum([P[1], P[2], P[3]])
            eb = shell_spectrum([P[5], P[6], P[7]])
            t, _, _ = S.time()
            log["spectra"].append({"step": done, "t": t, "E_v": ev.tolist(), "E_B": eb.tolist()})
            del P
        k = min(log_every, steps - done)
        S.step(k)
        done += k
        d = S.diagnostics(raise_on_error=False)
        log["divb"].append((done, d["t"], d["divb_max"] / n))
        if verbose:
            print(f"[run] {precision}{'+learned' if mlp else ''} {n}^3 step {done} t={d['t']:.4f} "
                  f"divB*dx={d['divb_max'] / n:.2e} rc={d['rc']}", flush=True)
        if d["rc"] != 0:
            log["error"] = d["rc"]
            break
    torch.cuda.synchronize()
    log["seconds"] = time.perf_counter() - t0
    if "error" not in log:
        P = S.primitives()
        t, _, _ = S.time()
        log["spectra"].append({"step": done, "t": t, "E_v": shell_spectrum([P[1], P[2], P[3]]).tolist(),
                               "E_B": shell_spectrum([P[5], P[6], P[7]]).tolist()})
        del P
    d = S.diagnostics(raise_on_error=False)
    h = d["newton_hist"]
    tot = max(sum(h), 1)
    cdf, acc = [], 0
    for c in h:
        acc += c
        cdf.append(acc / tot)
    log["newton"] = {"mean": d["newton_iters"] / max(d["newton_calls"], 1),
                     "p50": next(i for i, c in enumerate(cdf) if c >= 0.5),
                     "p99": next(i for i, c in enumerate(cdf) if c >= 0.99),
                     "mlp_fallback_rate": d["mlp_fallbacks"] / max(d["newton_calls"], 1),
                     "floors": d["floors"], "c2p_failures": d["c2p_failures"],
                     "recon_fallbacks": d["recon_fallbacks"]}
    log["Mcell_updates_per_s"] = n ** 3 * done / log["seconds"] / 1e6
    P = S.primitives()
    log["final_prims"] = P
    S.close()
    return log


def turbulence2d_run(n, t_end, precision="fp64", high_order=True, log_every=200,
                     wall_limit=None, device="cuda", verbose=True):
    """The 2D set-up of Sec. 5 on an n x n x 1 box (side 2 pi) up to t_end
    (or until wall_limit seconds have passed): logs div B, the time per
    simulation time unit, and the shell spectra of the perpendicular (x, y)
    and parallel (z) components of v and B at the start and the end."""
    prim5, bf, L = inputs.turbulence2d(n, device=device)
    torch.cuda.empty_cache()
    S = Solver(n, n, 1, L=L, precision=precision, high_order=high_order, collect_stats=False,
               device=device)
    S.init(prim5, bf)
    del prim5, bf

    def spectra(tag):
        P = S.primitives()
        t, st, _ = S.time()
        out = {"tag": tag, "t": t, "step": st,
               "E_v_perp": shell_spectrum([P[1], P[2]]).tolist(),
               "E_v_par": shell_spectrum([P[3]]).tolist(),
               "E_B_perp": shell_spectrum([P[5], P[6]]).tolist(),
               "E_B_par": shell_spectrum([P[7]]).tolist()}
        del P
        return out

    log = {"n": n, "precision": precision, "high_order": high_order, "spectra": [spectra("start")],
           "divb": [], "divb0": S.diagnostics()["divb_max"] * L[0] / n}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, steps = 0.0, 0
    while t < t_end:
        S.step(log_every)
        steps += log_every
        t, _, dt = S.time()
        d = S.diagnostics(raise_on_error=False)
        wall = time.perf_counter() - t0
        log["divb"].append((steps, t, d["divb_max"] * L[0] / n))
        if verbose:
            print(f"[run2d] {n}^2 {precision}{'+HO' if high_order else ''} step {steps} t={t:.3f} "
                  f"dt={dt:.2e} wall={wall:.0f}s divB*dx={d['divb_max'] * L[0] / n:.1e} "
                  f"rc={d['rc']}", flush=True)
        if d["rc"] != 0:
            log["error"] = d["rc"]
            break
        if wall_limit is not None and wall > wall_limit:
            log["stopped_by_wall_limit"] = True
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log.update({"t_final": t, "steps": steps, "seconds": wall,
                "seconds_per_time_unit": wall / max(t, 1e-300),
                "Mcell_updates_per_s": n * n * steps / wall / 1e6})
    log["spectra"].append(spectra("end"))
    end = log["spectra"][-1]
    log["slopes_end"] = {key: {f"{a}-{b}": spectral_slope(end[key], a, b)
                               for a, b in ((4, 32), (8, 128), (16, 512)) if b <= len(end[key])}
                         for key in ("E_v_perp", "E_B_perp")}
    S.close()
    return log


def spectral_slope(E, kmin=3, kmax=None):
    """Least-squares slope of log E against log k over [kmin, kmax]."""
    kmax = kmax or len(E)
    ks = torch.arange(1, len(E) + 1, dtype=torch.float64)
    sel = (ks >= kmin) & (ks <= kmax) & (torch.as_tensor(E) > 0)
    x = torch.log(ks[sel])
    y = torch.log(torch.as_tensor(E, dtype=torch.float64)[sel])
    A = torch.stack([x, torch.ones_like(x)], 1)
    sol = torch.linalg.lstsq(A, y[:, None]).solution
    return float(sol[0, 0])


def compare_runs(a, b, scale=1.0):
    """Per-variable L1 relative difference of two runs' final primitives."""
    out = []
    for q in range(8):
        d = (a["final_prims"][q] - b["final_prims"][q]).abs().sum().item()
        r = max(b["final_prims"][q].abs().sum().item(), b["final_prims"][q].numel() * scale)
        out.append(d / r)
    return out


def _summary(log):
    """JSON-ready digest of a turbulence_run log (no tensors)."""
    out = {k: log[k] for k in ("n", "precision", "learned", "seconds", "Mcell_updates_per_s",
                               "newton") if k in log}
    if "error" in log:
        out["error"] = log["error"]
    out["divb_max_dx"] = max(x[2] for x in log["divb"]) if log["divb"] else None
    out["divb"] = log["divb"]
    out["t_final"] = log["divb"][-1][1] if log["divb"] else 0.0
    out["spectra"] = log["spectra"]
    out["slopes_v_B"] = [(s["step"], spectral_slope(s["E_v"]), spectral_slope(s["E_B"]))
                         for s in log["spectra"]]
    return out


def main(argv=None):
    """Long run of the 3D turbulence set-up: plain FP64 first, then the mixed
    form with the learned guess from the same initial state, and the
    per-variable L1 difference of their final primitives.  With --2d: the
    2D set-up of Sec. 5 up to --t-end in one form."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--n", type=int, default=768)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--log-every", type=int, default=10)
    ap.add_argument("--spectrum-every", type=int, default=100)
    ap.add_argument("--out", default=None, help="write the JSON summary here")
    ap.add_argument("--2d", dest="two_d", action="store_true")
    ap.add_argument("--t-end", type=float, default=20.0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-ho", action="store_true")
    ap.add_argument("--wall-limit", type=float, default=None)
    args = ap.parse_args(argv)
    if args.two_d:
        log = turbulence2d_run(args.n, args.t_end, args.precision, not args.no_ho,
                               log_every=args.log_every, wall_limit=args.wall_limit)
        print("[run2d] done:", {k: log[k] for k in ("t_final", "steps", "seconds",
                                                    "seconds_per_time_unit",
                                                    "Mcell_updates_per_s", "slopes_end")},
              flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(log, f)
        return log
    from .learned import train_default
    mlp, hist, npairs = train_default()
    print(f"[run] learned guess trained on {npairs} pairs, loss {hist[-1][1]:.2e}", flush=True)
    res = {"workload": f"turbulence {args.n}^3, sigma0 = 10, Gamma <= 5, {args.steps} steps"}
    a = turbulence_run(args.n, args.steps, "fp64", None, log_every=args.log_every,
                       spectrum_every=args.spectrum_every)
    a["final_prims"] = a["final_prims"].cpu()
    torch.cuda.empty_cache()
    b = turbulence_run(args.n, args.steps, "mixed", mlp, log_every=args.log_every,
                       spectrum_every=args.spectrum_every)
    b["final_prims"] = b["final_prims"].cpu()
    res["fp64"] = _summary(a)
    res["mixed+learned"] = _summary(b)
    res["l1_rel_mixed_learned_vs_fp64"] = compare_runs(b, a)
    print("[run] L1 rel (rho, vx, vy, vz, p, Bx, By, Bz):",
          ["%.2e" % d for d in res["l1_rel_mixed_learned_vs_fp64"]], flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    return res


if __name__ == "__main__":
    main()
