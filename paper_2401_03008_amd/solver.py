"""Torch-owned device buffers around the C ABI.

PyTorch supplies device memory and the stream; every step of the solver runs
in libsrmhd's HIP kernels.  State tensors (float64, shape (n, nz, ny, nx)):
``cons`` = D, Sx, Sy, Sz, U; ``bface`` = face B_x, B_y, B_z; ``W`` = Newton
guess: the caller-owned buffers of the C ABI.  ``checkpoint``/``restore`` go
through srmhd_get_state / srmhd_set_state.

With ``ghost_z = G > 0`` the solver is one z-slab of a larger periodic box
(nz interior planes of length L[2], plus G ghost planes below and above: the
tensors have nz + 2G planes); it advances with ``stage_begin`` /
``stage_end`` and a ghost exchange (``halo_pack`` / ``halo_unpack``) after
every stage.
"""
from __future__ import annotations

import torch

from . import binding as B

_PREC = {"fp64": B.SRMHD_FP64, "mixed": B.SRMHD_MIXED}
_RIEM = {"hll": B.SRMHD_HLL, "llf": B.SRMHD_LLF}
_GUESS = {"prev": B.SRMHD_GUESS_PREV, "mlp": B.SRMHD_GUESS_MLP, "cold": B.SRMHD_GUESS_COLD,
          "mlp_all": B.SRMHD_GUESS_MLP_ALL}
_REC = {"mp5": B.SRMHD_REC_MP5, "mc": B.SRMHD_REC_MC}


class Solver:
    def __init__(self, nx, ny=None, nz=None, L=(1.0, 1.0, 1.0), gamma_ad=4.0 / 3.0, cfl=0.5,
                 dt_fixed=0.0, riemann="hll", precision="fp64", guess="prev",
                 newton_maxit=50, newton_tol=1e-14, pfloor=0.0, collect_stats=True,
                 recon="mp5", time_order=3, high_order=False, ghost_z=0, device="cuda:0",
                 stream=None):
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
        cfg.ghost_z = int(ghost_z)
        self.cfg = cfg
        self.ghost_z = int(ghost_z)
        self.shape = (nz + 2 * self.ghost_z, ny, nx)
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

    def get_state(self):
        """The state through srmhd_get_state: new tensors cons (5, ...),
        bface (3, ...), W, and host t, step."""
        cons = torch.empty_like(self.cons)
        bface = torch.empty_like(self.bface)
        W = torch.empty_like(self.W)
        t, st = B.srmhd_get_state(self.ctx, [a.data_ptr() for a in cons],
                                  [b.data_ptr() for b in bface], W.data_ptr())
        return {"cons": cons, "bface": bface, "W": W, "t": t, "step": st}

    def set_state(self, cons, bface, W=None, t=0.0, step=0):
        """srmhd_set_state from device tensors (W None: no previous W)."""
        c = [self._dev(a) for a in cons]
        b = [self._dev(a) for a in bface]
        w = self._dev(W) if W is not None else None
        B.srmhd_set_state(self.ctx, [a.data_ptr() for a in c], [a.data_ptr() for a in b],
                          w.data_ptr() if w is not None else 0, t, step)
        self.stream.synchronize()  # inputs may be temporaries

    def checkpoint(self):
        return self.get_state()

    def restore(self, ck):
        self.set_state(ck["cons"], ck["bface"], ck["W"], ck["t"], ck["step"])

    def mlp_guess(self):
        """(out (2, ...) float32: log(p/D), log Gamma; W0 (...) float64) of
        the learned guess on the current state (srmhd_mlp_guess)."""
        out = torch.empty((2,) + self.shape, dtype=torch.float32, device=self.device)
        w0 = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        B.srmhd_mlp_guess(self.ctx, out.data_ptr(), w0.data_ptr())
        return out, w0

    # ------------------------------------------------- stages and ghost planes
    def stage_begin(self, stage):
        B.srmhd_stage_begin(self.ctx, stage)

    def local_amax(self):
        """This slab's speed maximum (a 1-element device tensor) after
        stage_begin(1)."""
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        B.srmhd_local_amax(self.ctx, out.data_ptr())
        return out

    def stage_end(self, stage, amax=None):
        """amax: 1-element device tensor with the maximum over all slabs
        (stage 1), or None for this slab's own."""
        B.srmhd_stage_end(self.ctx, stage, amax.data_ptr() if amax is not None else 0)

    def halo_pack(self, side):
        """New device tensor with the G edge planes of side 0 (bottom) or 1
        (top) of the 9 exchanged arrays."""
        buf = torch.empty(B.srmhd_halo_count(self.ctx), dtype=torch.float64, device=self.device)
        B.srmhd_halo_pack(self.ctx, side, buf.data_ptr())
        return buf

    def halo_unpack(self, side, buf):
        B.srmhd_halo_unpack(self.ctx, side, buf.data_ptr())
