"""ctypes binding of libsrmhd.so: the entry points of include/srmhd.h with
the same names, argument marshalling only.  Every computation runs in the
HIP library; if the library is missing this module raises instead of falling
back to anything else.

Pointers passed to the device-side entry points are integers (device
addresses, e.g. ``tensor.data_ptr()``) or sequences of them.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsrmhd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "srmhd.h")

SRMHD_OK = 0
SRMHD_E_INVAL = -1
SRMHD_E_HIP = -2
SRMHD_E_C2P = -3
SRMHD_E_NONFINITE = -4
SRMHD_E_STATE = -5
SRMHD_HLL, SRMHD_LLF = 0, 1
SRMHD_FP64, SRMHD_MIXED = 0, 1
SRMHD_GUESS_PREV, SRMHD_GUESS_MLP, SRMHD_GUESS_COLD, SRMHD_GUESS_MLP_ALL = 0, 1, 2, 3
SRMHD_REC_MP5, SRMHD_REC_MC = 0, 1
ERRBIT_C2P, ERRBIT_NONFINITE, ERRBIT_DT, ERRBIT_PRESSURE = 1, 2, 4, 8


class SrmhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"srmhd error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("gamma_ad", C.c_double), ("cfl", C.c_double), ("dt_fixed", C.c_double),
                ("riemann", C.c_int), ("precision", C.c_int), ("guess", C.c_int),
                ("newton_maxit", C.c_int), ("newton_tol", C.c_double),
                ("pfloor", C.c_double), ("collect_stats", C.c_int),
                ("recon", C.c_int), ("time_order", C.c_int), ("high_order", C.c_int),
                ("ghost_z", C.c_int)]


class Buffers(C.Structure):
    _fields_ = [("cons", C.c_void_p * 5), ("bface", C.c_void_p * 3),
                ("guess_w", C.c_void_p), ("work", C.c_void_p), ("work_bytes", C.c_size_t)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("step", C.c_long),
                ("amax", C.c_double), ("divb_max", C.c_double), ("sums", C.c_double * 8),
                ("newton_iters", C.c_long), ("newton_calls", C.c_long),
                ("newton_hist", C.c_long * 32), ("c2p_failures", C.c_long),
                ("recon_fallbacks", C.c_long), ("floors", C.c_long),
                ("mlp_fallbacks", C.c_long), ("error_word", C.c_uint)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["sums"] = list(self.sums)
        d["newton_hist"] = list(self.newton_hist)
        return d


_lib = None
_VP = C.c_void_p
_CTX = C.c_void_p


def check_build_id(L, root=None):
    """Raise unless the library L was built from the sources under root (the
    repository this binding sits in by default)."""
    from .build import ROOT, source_id
    want = source_id(root or ROOT)
    L.srmhd_build_id.restype = C.c_char_p
    got = (L.srmhd_build_id() or b"").decode()
    if got != want:
        raise RuntimeError(
            f"{LIB_PATH} was built from other sources (build id {got}, sources {want}): "
            "rebuild it (python -c 'import __graft_entry__ as g; g.build()')")


def lib():
    """Load libsrmhd.so (built by ``paper_2401_03008_amd.build``); refuses a
    library built from sources other than those beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        check_build_id(L)
        L.srmhd_config_default.argtypes = [C.POINTER(Config)]
        L.srmhd_work_bytes.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.srmhd_create.argtypes = [C.POINTER(Config), C.POINTER(Buffers), _VP, C.POINTER(_CTX)]
        L.srmhd_init_from_prims.argtypes = [_CTX, C.POINTER(_VP), C.POINTER(_VP)]
        L.srmhd_step.argtypes = [_CTX, C.c_int]
        L.srmhd_rhs.argtypes = [_CTX, C.POINTER(_VP), _VP]
        L.srmhd_get_primitives.argtypes = [_CTX, C.POINTER(_VP)]
        L.srmhd_get_diagnostics.argtypes = [_CTX, C.POINTER(Diag)]
        L.srmhd_reset_counters.argtypes = [_CTX]
        L.srmhd_get_time.argtypes = [_CTX, C.POINTER(C.c_double), C.POINTER(C.c_long),
                                     C.POINTER(C.c_double)]
        L.srmhd_set_time.argtypes = [_CTX, C.c_double, C.c_long]
        L.srmhd_get_state.argtypes = [_CTX, C.POINTER(_VP), C.POINTER(_VP), _VP,
                                      C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.srmhd_set_state.argtypes = [_CTX, C.POINTER(_VP), C.POINTER(_VP), _VP, C.c_double,
                                      C.c_long]
        L.srmhd_mlp_guess.argtypes = [_CTX, _VP, _VP]
        L.srmhd_stage_begin.argtypes = [_CTX, C.c_int]
        L.srmhd_local_amax.argtypes = [_CTX, _VP]
        L.srmhd_stage_end.argtypes = [_CTX, C.c_int, _VP]
        L.srmhd_halo_count.argtypes = [_CTX, C.POINTER(C.c_size_t)]
        L.srmhd_halo_pack.argtypes = [_CTX, C.c_int, _VP]
        L.srmhd_halo_unpack.argtypes = [_CTX, C.c_int, _VP]
        L.srmhd_set_mlp.argtypes = [_CTX, _VP, _VP, C.POINTER(C.c_float)]
        L.srmhd_set_guess.argtypes = [_CTX, C.c_int]
        L.srmhd_harvest.argtypes = [_CTX, _VP, _VP, C.c_int, C.c_double, C.c_uint,
                                    C.POINTER(C.c_int)]
        L.srmhd_mlp_cache_bytes.argtypes = [C.c_int]
        L.srmhd_mlp_cache_bytes.restype = C.c_size_t
        L.srmhd_mlp_quantize.argtypes = [_VP, _VP, C.c_int, _VP]
        L.srmhd_mlp_forward.argtypes = [_VP, _VP, _VP, _VP, _VP, C.c_int, _VP]
        L.srmhd_mlp_forward_noalloc.argtypes = [_VP, _VP, _VP, _VP, C.c_int, _VP]
        L.srmhd_mlp_loss_grad.argtypes = [_VP, _VP, _VP, _VP, C.c_int, _VP]
        L.srmhd_mlp_backward.argtypes = [_VP, _VP, _VP, C.c_int, _VP]
        L.srmhd_mlp_adam.argtypes = [_VP, _VP, _VP, _VP, _VP, C.c_int, C.c_float, C.c_float,
                                     C.c_float, C.c_float, C.c_int, _VP]
        L.srmhd_kernel_timing.argtypes = [_CTX, C.c_int]
        L.srmhd_get_kernel_times.argtypes = [_CTX, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.srmhd_last_error.argtypes = [_CTX]
        L.srmhd_last_error.restype = C.c_char_p
        L.srmhd_strerror.argtypes = [C.c_int]
        L.srmhd_strerror.restype = C.c_char_p
        L.srmhd_destroy.argtypes = [_CTX]
        L.srmhd_destroy.restype = None
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/srmhd.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(srmhd_\w+)\s*\(", txt)))


def _check(rc, ctx=None):
    if rc != SRMHD_OK:
        msg = lib().srmhd_last_error(ctx)
        raise SrmhdError(rc, (msg or b"").decode() or lib().srmhd_strerror(rc).decode())
    return rc


def _ptrs(seq, n):
    if len(seq) != n:
        raise ValueError(f"expected {n} pointers, got {len(seq)}")
    return (_VP * n)(*[int(p) for p in seq])


# ---------------------------------------------------------------- entry points
def srmhd_config_default():
    cfg = Config()
    _check(lib().srmhd_config_default(C.byref(cfg)))
    return cfg


def srmhd_work_bytes(cfg):
    n = C.c_size_t()
    _check(lib().srmhd_work_bytes(C.byref(cfg), C.byref(n)))
    return n.value


def srmhd_create(cfg, cons, bface, guess_w, work, work_bytes, stream=0):
    buf = Buffers()
    buf.cons = (_VP * 5)(*[int(p) for p in cons])
    buf.bface = (_VP * 3)(*[int(p) for p in bface])
    buf.guess_w = int(guess_w)
    buf.work = int(work)
    buf.work_bytes = int(work_bytes)
    ctx = _CTX()
    _check(lib().srmhd_create(C.byref(cfg), C.byref(buf), _VP(int(stream) or None), C.byref(ctx)))
    return ctx


def srmhd_init_from_prims(ctx, prim5, bface):
    _check(lib().srmhd_init_from_prims(ctx, _ptrs(prim5, 5), _ptrs(bface, 3)), ctx)


def srmhd_step(ctx, nsteps):
    _check(lib().srmhd_step(ctx, int(nsteps)), ctx)


def srmhd_rhs(ctx, rhs, amax_dev):
    _check(lib().srmhd_rhs(ctx, _ptrs(rhs, 8), _VP(int(amax_dev))), ctx)


def srmhd_get_primitives(ctx, prim):
    _check(lib().srmhd_get_primitives(ctx, _ptrs(prim, 8)), ctx)


def srmhd_get_diagnostics(ctx, raise_on_error=True):
    d = Diag()
    rc = lib().srmhd_get_diagnostics(ctx, C.byref(d))
    if raise_on_error:
        _check(rc, ctx)
    return d, rc


def srmhd_reset_counters(ctx):
    _check(lib().srmhd_reset_counters(ctx), ctx)


def srmhd_get_time(ctx):
    t, st, dt = C.c_double(), C.c_long(), C.c_double()
    _check(lib().srmhd_get_time(ctx, C.byref(t), C.byref(st), C.byref(dt)), ctx)
    return t.value, st.value, dt.value


def srmhd_set_time(ctx, t, step):
    _check(lib().srmhd_set_time(ctx, float(t), int(step)), ctx)


def srmhd_get_state(ctx, cons, bface, w):
    """cons (5 device pointers or None), bface (3 or None), w (pointer or 0);
    returns (t, step)."""
    t, st = C.c_double(), C.c_long()
    pc = _ptrs(cons, 5) if cons is not None else None
    pb = _ptrs(bface, 3) if bface is not None else None
    _check(lib().srmhd_get_state(ctx, pc, pb, _VP(int(w) or None), C.byref(t), C.byref(st)),
           ctx)
    return t.value, st.value


def srmhd_set_state(ctx, cons, bface, w, t, step):
    """w: device pointer, or 0/None for no previous W."""
    _check(lib().srmhd_set_state(ctx, _ptrs(cons, 5), _ptrs(bface, 3), _VP(int(w or 0) or None),
                                 float(t), int(step)), ctx)


def srmhd_mlp_guess(ctx, out, w0=0):
    _check(lib().srmhd_mlp_guess(ctx, _VP(int(out)), _VP(int(w0 or 0) or None)), ctx)


def srmhd_stage_begin(ctx, stage):
    _check(lib().srmhd_stage_begin(ctx, int(stage)), ctx)


def srmhd_local_amax(ctx, amax_dev):
    _check(lib().srmhd_local_amax(ctx, _VP(int(amax_dev))), ctx)


def srmhd_stage_end(ctx, stage, amax_dev=0):
    """amax_dev: device pointer to the speed maximum over all slabs, or 0."""
    _check(lib().srmhd_stage_end(ctx, int(stage), _VP(int(amax_dev or 0) or None)), ctx)


def srmhd_halo_count(ctx):
    n = C.c_size_t()
    _check(lib().srmhd_halo_count(ctx, C.byref(n)), ctx)
    return n.value


def srmhd_halo_pack(ctx, side, buf):
    _check(lib().srmhd_halo_pack(ctx, int(side), _VP(int(buf))), ctx)


def srmhd_halo_unpack(ctx, side, buf):
    _check(lib().srmhd_halo_unpack(ctx, int(side), _VP(int(buf))), ctx)


def srmhd_build_id():
    return (lib().srmhd_build_id() or b"").decode()


MLP_NPARAM = 4674
MLP_OFF = {"W1": 0, "b1": 320, "W2": 384, "b2": 4480, "W3": 4544, "b3": 4672}


def _vp(x):
    return _VP(int(x) or None)


def srmhd_set_mlp(ctx, params, w_bf16, norm):
    arr = (C.c_float * 14)(*[float(v) for v in norm])
    _check(lib().srmhd_set_mlp(ctx, _vp(params), _vp(w_bf16), arr), ctx)


def srmhd_set_guess(ctx, guess):
    _check(lib().srmhd_set_guess(ctx, int(guess)), ctx)


def srmhd_harvest(ctx, feats, targets, cap, frac, seed):
    n = C.c_int()
    _check(lib().srmhd_harvest(ctx, _vp(feats), _vp(targets), int(cap), float(frac),
                               int(seed), C.byref(n)), ctx)
    return n.value


def srmhd_mlp_cache_bytes(batch):
    return lib().srmhd_mlp_cache_bytes(int(batch))


def srmhd_mlp_quantize(params, w_bf16, n, stream=0):
    _check(lib().srmhd_mlp_quantize(_vp(params), _vp(w_bf16), int(n), _vp(stream)))


def srmhd_mlp_forward(params, w_bf16, x, y, cache, batch, stream=0):
    _check(lib().srmhd_mlp_forward(_vp(params), _vp(w_bf16), _vp(x), _vp(y), _vp(cache),
                                   int(batch), _vp(stream)))


MLP_NOALLOC_MAX_BATCH = 65536


def srmhd_mlp_forward_noalloc(params, w_bf16, x, y, batch, stream=0):
    _check(lib().srmhd_mlp_forward_noalloc(_vp(params), _vp(w_bf16), _vp(x), _vp(y),
                                           int(batch), _vp(stream)))


def srmhd_mlp_loss_grad(y, t, cache, loss, batch, stream=0):
    _check(lib().srmhd_mlp_loss_grad(_vp(y), _vp(t), _vp(cache), _vp(loss), int(batch),
                                     _vp(stream)))


def srmhd_mlp_backward(w_bf16, cache, grad, batch, stream=0):
    _check(lib().srmhd_mlp_backward(_vp(w_bf16), _vp(cache), _vp(grad), int(batch), _vp(stream)))


def srmhd_mlp_adam(params, w_bf16, m, v, grad, n, lr, beta1, beta2, eps, t, stream=0):
    _check(lib().srmhd_mlp_adam(_vp(params), _vp(w_bf16), _vp(m), _vp(v), _vp(grad), int(n),
                                float(lr), float(beta1), float(beta2), float(eps), int(t),
                                _vp(stream)))


NKCLASS = 9
KCLASS_NAMES = ["c2p", "flux_xy", "flux_z", "uct_x", "uct_y", "uct_z", "update", "dt",
                "update_c2p"]


def srmhd_kernel_timing(ctx, enable):
    _check(lib().srmhd_kernel_timing(ctx, 1 if enable else 0), ctx)


def srmhd_get_kernel_times(ctx):
    ms = (C.c_double * NKCLASS)()
    n = (C.c_long * NKCLASS)()
    _check(lib().srmhd_get_kernel_times(ctx, ms, n), ctx)
    return {KCLASS_NAMES[k]: (ms[k], n[k]) for k in range(NKCLASS)}


def srmhd_last_error(ctx=None):
    return (lib().srmhd_last_error(ctx) or b"").decode()


def srmhd_strerror(code):
    return lib().srmhd_strerror(int(code)).decode()


def srmhd_destroy(ctx):
    lib().srmhd_destroy(ctx)
