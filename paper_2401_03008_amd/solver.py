"""Torch-owned device buffers around the C ABI.

PyTorch supplies device memory and the stream; every step of the solver runs
in libsrmhd's HIP kernels.  State tensors (float64, shape (n, nz, ny, nx)):
``cons`` = D, Sx, Sy, Sz, U; ``bface`` = face B_x, B_y, B_z; ``W`` = Newton
guess.  They are the caller-owned buffers of the C ABI, so copying them (plus
``time()``) is a checkpoint.
"""
from __future__ import annotations

import torch

from . import binding as B

_PREC = {"fp64": B.SRMHD_FP64, "mixed": B.SRMHD_MIXED}
_RIEM = {"hll": B.SRMHD_HLL, "llf": B.SRMHD_LLF}
_GUESS = {"prev": B.SRMHD_GUESS_PREV, "mlp": B.SRMHD_GUESS_MLP, "cold": B.SRMHD_GUESS_COLD}
_REC = {"mp5": B.SRMHD_REC_MP5, "mc": B.SRMHD_REC_MC}


class Solver:
    def __init__(self, nx, ny=None, nz=None, L=(1.0, 1.0, 1.0), gamma_ad=4.0 / 3.0, cfl=0.5,
                 dt_fixed=0.0, riemann="hll", precision="fp64", guess="prev",
                 newton_maxit=50, newton_tol=1e-14, pfloor=0.0, collect_stats=True,
                 recon="mp5", time_order=3, high_order=False, device="cuda:0", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device (torch.cuda.is_available() is False)")
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.device = torch.device(device)
        cfg = B.srmhd_config_default()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.lx, cfg.ly, cfg.lz = L
        cfg.gamma_ad, cfg.cfl, cfg.dt_fixed = gamma_ad, cfl, dt_fixed
        cfg.riemann = _RIEM[riemann]
        cfg.precision = _PREC[precision]
        cfg.guess = _GUESS[guess]
        cfg.newton_maxit, cfg.newton_tol, cfg.pfloor = newton_maxit, newton_tol, pfloor
        cfg.collect_stats = 1 if collect_stats else 0
        cfg.recon = _REC[recon]
        cfg.time_order = int(time_order)
        cfg.high_order = 1 if high_order else 0
        self.cfg = cfg
        self.shape = (nz, ny, nx)
        wb = B.srmhd_work_bytes(cfg)
        f64 = dict(dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self.cons = torch.zeros((5,) + self.shape, **f64)
            self.bface = torch.zeros((3,) + self.shape, **f64)
            self.W = torch.zeros(self.shape, **f64)
            self.work = torch.empty(wb + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            base = self.work.data_ptr()
            aligned = (base + 255) // 256 * 256
            self._amax = torch.zeros(1, **f64)
            self.ctx = B.srmhd_create(cfg, [a.data_ptr() for a in self.cons],
                                      [b.data_ptr() for b in self.bface], self.W.data_ptr(),
                                      aligned, wb, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            B.srmhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
        assert tuple(t.shape[-3:]) == self.shape
        return t

    # ------------------------------------------------------------------ ABI
    def init(self, prim5, bface):
        """prim5: rho, vx, vy, vz, p at centres; bface: face B (arrays or tensors)."""
        p = [self._dev(a) for a in prim5]
        b = [self._dev(a) for a in bface]
        B.srmhd_init_from_prims(self.ctx, [a.data_ptr() for a in p], [a.data_ptr() for a in b])
        self.stream.synchronize()  # inputs may be temporaries

    def step(self, nsteps=1):
        B.srmhd_step(self.ctx, nsteps)

    def primitives(self):
        out = torch.empty((8,) + self.shape, dtype=torch.float64, device=self.device)
        B.srmhd_get_primitives(self.ctx, [out[n].data_ptr() for n in range(8)])
        return out

    def rhs(self):
        out = torch.empty((8,) + self.shape, dtype=torch.float64, device=self.device)
        B.srmhd_rhs(self.ctx, [out[n].data_ptr() for n in range(8)], self._amax.data_ptr())
        return out, self._amax

    def diagnostics(self, raise_on_error=True):
        d, rc = B.srmhd_get_diagnostics(self.ctx, raise_on_error)
        out = d.as_dict()
        out["rc"] = rc
        return out

    def reset_counters(self):
        B.srmhd_reset_counters(self.ctx)

    def set_mlp(self, mlp):
        """Use a trained learned.Mlp for the Newton guess (kept by reference)."""
        self._mlp = mlp
        B.srmhd_set_mlp(self.ctx, mlp.params.data_ptr(), mlp.w.data_ptr(), mlp.norm)

    def set_guess(self, guess):
        B.srmhd_set_guess(self.ctx, _GUESS[guess])

    def harvest(self, cap, frac, seed=1):
        """(features (n, 5), targets (n, 2)) float32 device tensors."""
        f = torch.empty((cap, 5), dtype=torch.float32, device=self.device)
        t = torch.empty((cap, 2), dtype=torch.float32, device=self.device)
        n = B.srmhd_harvest(self.ctx, f.data_ptr(), t.data_ptr(), cap, frac, seed)
        return f[:n], t[:n]

    def kernel_timing(self, enable=True):
        B.srmhd_kernel_timing(self.ctx, enable)

    def kernel_times(self):
        """{class: (total ms, launches)} since timing was enabled."""
        return B.srmhd_get_kernel_times(self.ctx)

    def time(self):
        return B.srmhd_get_time(self.ctx)

    def set_time(self, t, step):
        B.srmhd_set_time(self.ctx, t, step)

    def checkpoint(self):
        t, st, dt = self.time()
        return {"cons": self.cons.clone(), "bface": self.bface.clone(), "W": self.W.clone(),
                "t": t, "step": st}

    def restore(self, ck):
        self.cons.copy_(ck["cons"])
        self.bface.copy_(ck["bface"])
        self.W.copy_(ck["W"])
        self.set_time(ck["t"], ck["step"])
