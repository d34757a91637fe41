"""ctypes wrapper of the FP64 CPU oracle (``srmhd_oracle.c``) and of the
FP64 MLP reference (``mlp_oracle.py``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the CPU-baseline leg of ``bench.py``; the product path never imports
it.  The oracle shares no code with the HIP library.

Grid arrays are numpy float64, C-contiguous, shape (nz, ny, nx) (x fastest).
Primitive vectors are (rho, vx, vy, vz, p, Bx, By, Bz); conserved vectors are
(D, Sx, Sy, Sz, U, Bx, By, Bz).  Face field bf[d] holds B_d at the +d face of
each cell; edge field E[k] holds E_k at the edge that is +1/2 in the two other
directions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srmhd_oracle.c")
_LIB = os.environ.get("SRMHD_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("gam", C.c_double), ("cfl", C.c_double), ("dt_fixed", C.c_double),
                ("riemann", C.c_int), ("maxit", C.c_int), ("tol", C.c_double),
                ("pfloor", C.c_double), ("recon", C.c_int), ("time_order", C.c_int),
                ("ho", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_long), ("newton_hist", C.c_long * 32),
                ("c2p_fail", C.c_long), ("recon_fallbacks", C.c_long),
                ("floors", C.c_long)]

    def as_dict(self) -> dict:
        return {"newton_iters": self.newton_iters,
                "newton_hist": list(self.newton_hist),
                "c2p_fail": self.c2p_fail,
                "recon_fallbacks": self.recon_fallbacks,
                "floors": self.floors}


_lib = None
_D = C.c_double
_PD = C.POINTER(C.c_double)
_PP = C.POINTER(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.orc_prim2cons.argtypes = [_D, _PD, _PD]
        L.orc_flux.argtypes = [_D, _PD, C.c_int, _PD]
        L.orc_speeds.argtypes = [_D, _PD, C.c_int, _PD, _PD]
        L.orc_con2prim.argtypes = [_D, _PD, _PD, C.c_int, _D, _D, _PD,
                                   C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_con2prim.restype = C.c_int
        L.orc_mp5.argtypes = [_PD]
        L.orc_mp5.restype = _D
        L.orc_riemann.argtypes = [C.c_int, _D, _PD, _PD, C.c_int, _PD, _PD, _PD]
        L.orc_uct_formula.argtypes = [_PD] + [_D] * 8
        L.orc_uct_formula.restype = _D
        cp = C.POINTER(_Cfg)
        L.orc_init.argtypes = [cp, _PP, _PP, _PP, C.c_void_p]
        L.orc_c2p.argtypes = [cp, _PP, _PP, C.c_void_p, _PP, C.c_void_p,
                              C.POINTER(Stats)]
        L.orc_c2p.restype = C.c_int
        L.orc_rhs.argtypes = [cp, _PP, _PP, _PP, _PD, _PP, _PP, _PP, _PP,
                              C.POINTER(Stats)]
        L.orc_rhs_cells.argtypes = [cp, _PP, _PP, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [cp, _PP, _PP, C.c_void_p, C.c_int, _PD, _PD,
                               C.POINTER(Stats)]
        L.orc_step.restype = C.c_int
        L.orc_divb_max.argtypes = [cp, _PP]
        L.orc_divb_max.restype = _D
        L.orc_sums.argtypes = [cp, _PP, _PP, _PD]
        L.orc_num_threads.restype = C.c_int
        for name in ("orc_mc", "orc_int_ho", "orc_der_ho", "orc_mp5_point"):
            getattr(L, name).argtypes = [_PD]
            getattr(L, name).restype = _D
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a, a.ctypes.data_as(_PD)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- point ops
def prim2cons(pr, gam=4.0 / 3.0):
    a, pa = _vec(pr, 8)
    u = np.zeros(8)
    lib().orc_prim2cons(gam, pa, u.ctypes.data_as(_PD))
    return u


def flux(pr, d, gam=4.0 / 3.0):
    a, pa = _vec(pr, 8)
    f = np.zeros(8)
    lib().orc_flux(gam, pa, d, f.ctypes.data_as(_PD))
    return f


def speeds(pr, d, gam=4.0 / 3.0):
    a, pa = _vec(pr, 8)
    lm, lp = _D(), _D()
    lib().orc_speeds(gam, pa, d, C.byref(lm), C.byref(lp))
    return lm.value, lp.value


def con2prim(u, W, gam=4.0 / 3.0, maxit=50, tol=1e-14, pfloor=0.0):
    """Returns (status, prim[8], W, iterations, floored)."""
    a, pa = _vec(u, 8)
    w = _D(W)
    pr = np.zeros(8)
    it, fl = C.c_int(), C.c_int()
    rc = lib().orc_con2prim(gam, pa, C.byref(w), maxit, tol, pfloor,
                            pr.ctypes.data_as(_PD), C.byref(it), C.byref(fl))
    return rc, pr, w.value, it.value, fl.value


def mp5(s):
    a, pa = _vec(s, 5)
    return lib().orc_mp5(pa)


def mp5_point(s):
    """MP5 limiter around the 5-point interpolation of point values (the
    HO scheme's REC)."""
    a, pa = _vec(s, 5)
    return lib().orc_mp5_point(pa)


def mc(s):
    """Left-biased linear MC value at x_{i+1/2} from (v_{i-1}, v_i, v_{i+1})."""
    a, pa = _vec(s, 3)
    return lib().orc_mc(pa)


def int_ho(b):
    """Sixth-order centre value from the six face values b_{i-5/2..i+5/2}."""
    a, pa = _vec(b, 6)
    return lib().orc_int_ho(pa)


def der_ho(f):
    """Fhat(i+1/2) - Fhat(i-1/2) from point fluxes f_{i-5/2..i+5/2} (times
    1/dx this is the sixth-order derivative at x_i)."""
    a, pa = _vec(f, 6)
    return lib().orc_der_ho(pa)


def riemann(prL, prR, d, kind=0, gam=4.0 / 3.0):
    a, pa = _vec(prL, 8)
    b, pb = _vec(prR, 8)
    f = np.zeros(8)
    ap, am = _D(), _D()
    lib().orc_riemann(kind, gam, pa, pb, d, f.ctypes.data_as(_PD),
                      C.byref(ap), C.byref(am))
    return f, ap.value, am.value


def uct_formula(Eab, axp, axm, ayp, aym, byL, byR, bxL, bxR):
    a, pa = _vec(Eab, 4)
    return lib().orc_uct_formula(pa, axp, axm, ayp, aym, byL, byR, bxL, bxR)


# ----------------------------------------------------------------- grid ops
def _ptrs(arrs):
    arr = (C.c_void_p * len(arrs))()
    for n, a in enumerate(arrs):
        if a is None:
            arr[n] = None
        else:
            assert a.dtype == np.float64 and a.flags.c_contiguous
            arr[n] = a.ctypes.data
    return arr


class Grid:
    """One periodic box: configuration plus the oracle's grid operations."""

    def __init__(self, nx, ny=None, nz=None, lx=1.0, ly=1.0, lz=1.0,
                 gam=4.0 / 3.0, cfl=0.5, dt_fixed=0.0, riemann=0, maxit=50,
                 tol=1e-14, pfloor=0.0, recon=0, time_order=3, ho=0):
        """recon: 0 = MP5, 1 = linear MC; time_order: 3 (SSP-RK3) or 2
        (SSP-RK2); ho: 1 = sixth-order INT and DER corrections."""
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.shape = (nz, ny, nx)
        self.cfg = _Cfg(nx, ny, nz, lx, ly, lz, gam, cfl, dt_fixed, riemann,
                        maxit, tol, pfloor, recon, time_order, ho)
        self.stats = Stats()

    def _z(self, n):
        return [np.zeros(self.shape) for _ in range(n)]

    def init(self, prim5, bf):
        """cons (5 arrays) and W from cell-centred rho, v, p and face B."""
        cons = self._z(5)
        W = np.zeros(self.shape)
        prim5 = [np.ascontiguousarray(a, dtype=np.float64) for a in prim5]
        bf = [np.ascontiguousarray(a, dtype=np.float64) for a in bf]
        lib().orc_init(C.byref(self.cfg), _ptrs(prim5), _ptrs(bf), _ptrs(cons),
                       W.ctypes.data)
        return cons, W

    def c2p(self, cons, bf, W):
        """(prim[8], iters, nfail); W is updated in place."""
        prim = self._z(8)
        it = np.zeros(self.shape, dtype=np.int32)
        nfail = lib().orc_c2p(C.byref(self.cfg), _ptrs(cons), _ptrs(bf), W.ctypes.data,
                              _ptrs(prim), it.ctypes.data, C.byref(self.stats))
        return prim, it, nfail

    def rhs(self, prim, bf, detail=False):
        rhs = self._z(8)
        amax = _D()
        if detail:
            fh, apm, fv, ee = self._z(15), self._z(6), self._z(18), self._z(3)
            lib().orc_rhs(C.byref(self.cfg), _ptrs(prim), _ptrs(bf), _ptrs(rhs),
                          C.byref(amax), _ptrs(fh), _ptrs(apm), _ptrs(fv), _ptrs(ee),
                          C.byref(self.stats))
            return rhs, amax.value, {"fhat": fh, "apm": apm, "face_v": fv, "edge_e": ee}
        lib().orc_rhs(C.byref(self.cfg), _ptrs(prim), _ptrs(bf), _ptrs(rhs),
                      C.byref(amax), None, None, None, None, C.byref(self.stats))
        return rhs, amax.value

    def rhs_cells(self, prim, bf, cells):
        """L(U) at the linear cell indices `cells` only: array (len(cells), 8)."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((len(cells), 8))
        lib().orc_rhs_cells(C.byref(self.cfg), _ptrs(prim), _ptrs(bf), len(cells),
                            cells.ctypes.data, out.ctypes.data)
        return out

    def step(self, cons, bf, W, nsteps, t=0.0):
        """Advance in place; returns (t, dt_last, nfail)."""
        tt, dt = _D(t), _D()
        nfail = lib().orc_step(C.byref(self.cfg), _ptrs(cons), _ptrs(bf), W.ctypes.data,
                               nsteps, C.byref(tt), C.byref(dt), C.byref(self.stats))
        return tt.value, dt.value, nfail

    def divb_max(self, bf):
        return lib().orc_divb_max(C.byref(self.cfg), _ptrs(bf))

    def sums(self, cons, bf):
        s = np.zeros(8)
        lib().orc_sums(C.byref(self.cfg), _ptrs(cons), _ptrs(bf), s.ctypes.data_as(_PD))
        return s
