"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/srmhd.h declares, and validates configurations on the
host before touching a device."""
import ctypes as C
import os

import pytest

from paper_2401_03008_amd import binding as B


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_2401_03008_amd.build import build
        build()
    return B.lib()


def test_exports_every_declared_symbol(L):
    names = B.header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_defaults_and_work_bytes(L):
    cfg = B.srmhd_config_default()
    assert (cfg.nx, cfg.ny, cfg.nz) == (32, 32, 32)
    assert cfg.gamma_ad == pytest.approx(4.0 / 3.0)
    assert cfg.cfl == 0.5 and cfg.newton_maxit == 50 and cfg.newton_tol == 1e-14
    w64 = B.srmhd_work_bytes(cfg)
    n = 32 ** 3
    # RK register 8 + edge fields 3 + primitives 8 + per direction 5 fluxes,
    # a+-, 4 face velocities (33) arrays of n cells
    assert w64 >= (8 + 3 + 8 + 33) * 8 * n
    cfg.precision = B.SRMHD_MIXED
    wmx = B.srmhd_work_bytes(cfg)
    assert (8 + 3) * 8 * n + 41 * 4 * n <= wmx < w64


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("nz", -1), ("gamma_ad", 1.0), ("gamma_ad", 2.5), ("cfl", 0.0), ("cfl", 1.5),
    ("riemann", 5), ("precision", 7), ("guess", 9), ("newton_maxit", 0),
    ("newton_tol", 0.0), ("newton_tol", 0.5), ("pfloor", -1.0), ("lx", 0.0),
    ("dt_fixed", -1.0), ("recon", 2), ("time_order", 1), ("time_order", 4), ("high_order", 2),
])
def test_invalid_configs_rejected(L, field, value):
    cfg = B.srmhd_config_default()
    setattr(cfg, field, value)
    with pytest.raises(B.SrmhdError) as e:
        B.srmhd_work_bytes(cfg)
    assert e.value.code == B.SRMHD_E_INVAL
    assert B.srmhd_last_error(None)


def test_huge_grid_rejected(L):
    cfg = B.srmhd_config_default()
    cfg.nx = cfg.ny = cfg.nz = 1300
    with pytest.raises(B.SrmhdError):
        B.srmhd_work_bytes(cfg)


def test_create_rejects_bad_buffers_on_host(L):
    cfg = B.srmhd_config_default()
    with pytest.raises(B.SrmhdError) as e:
        B.srmhd_create(cfg, [0] * 5, [0] * 3, 0, 0, 0)
    assert e.value.code == B.SRMHD_E_INVAL
    # work too small
    with pytest.raises(B.SrmhdError) as e:
        B.srmhd_create(cfg, [256] * 5, [256] * 3, 256, 256, 16)
    assert "work" in str(e.value)
    # misaligned work
    with pytest.raises(B.SrmhdError) as e:
        B.srmhd_create(cfg, [256] * 5, [256] * 3, 256, 257, 1 << 40)
    assert "aligned" in str(e.value)


def test_null_context_calls(L):
    assert L.srmhd_step(None, 1) == B.SRMHD_E_INVAL
    assert L.srmhd_get_diagnostics(None, None) == B.SRMHD_E_INVAL
    assert B.srmhd_strerror(B.SRMHD_E_C2P) == "Newton inversion failed"


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libsrmhd.so")
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()


def test_null_state_calls(L):
    assert L.srmhd_get_state(None, None, None, None, None, None) == B.SRMHD_E_INVAL
    assert L.srmhd_set_state(None, None, None, None, 0.0, 0) == B.SRMHD_E_INVAL
    assert L.srmhd_mlp_guess(None, None, None) == B.SRMHD_E_INVAL


def test_library_matches_its_sources(L):
    from paper_2401_03008_amd.build import source_id
    assert B.srmhd_build_id() == source_id()


def test_stale_library_rejected(L, tmp_path):
    """A library whose build id differs from the sources beside it is refused:
    a copy of the sources with one kernel file edited gives another id."""
    import shutil
    from paper_2401_03008_amd.build import ROOT, source_files, source_id
    for f in source_files(ROOT):
        rel = os.path.relpath(f, ROOT)
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(f, tmp_path / rel)
    B.check_build_id(L, str(tmp_path))  # identical copy: accepted
    k = tmp_path / "paper_2401_03008_amd" / "csrc" / "srmhd_kernels.hip"
    k.write_text(k.read_text() + "\n// edited\n")
    assert source_id(str(tmp_path)) != source_id()
    with pytest.raises(RuntimeError, match="other sources"):
        B.check_build_id(L, str(tmp_path))


def test_struct_layouts_match_the_header(L, tmp_path):
    """The ctypes mirrors of srmhd_config, srmhd_buffers and srmhd_diag have
    the C structs' sizes and field offsets (a C program compiled against
    include/srmhd.h prints them)."""
    import subprocess
    fields = {"srmhd_config": B.Config, "srmhd_buffers": B.Buffers, "srmhd_diag": B.Diag}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "srmhd.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(B.HEADER))
    subprocess.run(["gcc", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        name, f, v = line.split()
        got[(name, f)] = int(v)
    for cname, py in fields.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_header_constants_match_the_binding():
    import re
    txt = open(B.HEADER).read()
    defs = dict(re.findall(r"#define (SRMHD_\w+) \(?(-?\w+)\)?", txt))
    assert int(defs["SRMHD_NKCLASS"]) == B.NKCLASS == len(B.KCLASS_NAMES)
    assert int(defs["SRMHD_MLP_NPARAM"]) == B.MLP_NPARAM
    assert int(defs["SRMHD_MLP_NOALLOC_MAX_BATCH"]) == B.MLP_NOALLOC_MAX_BATCH
    for k, v in B.MLP_OFF.items():
        assert int(defs["SRMHD_MLP_OFF_" + k.upper()]) == v
    for code in ("OK", "E_INVAL", "E_HIP", "E_C2P", "E_NONFINITE", "E_STATE"):
        assert int(defs["SRMHD_" + code]) == getattr(B, "SRMHD_" + code)
    enums = dict(re.findall(r"(SRMHD_GUESS_\w+) = (\d+)", txt))
    assert {k: int(v) for k, v in enums.items()} == {
        "SRMHD_GUESS_PREV": B.SRMHD_GUESS_PREV, "SRMHD_GUESS_MLP": B.SRMHD_GUESS_MLP,
        "SRMHD_GUESS_COLD": B.SRMHD_GUESS_COLD, "SRMHD_GUESS_MLP_ALL": B.SRMHD_GUESS_MLP_ALL}


@pytest.mark.parametrize("kw", [{"ghost_z": 3}, {"ghost_z": 7, "high_order": 1},
                                {"ghost_z": 4, "nz": 3}, {"ghost_z": 65}, {"ghost_z": -1}])
def test_invalid_slab_configs_rejected(L, kw):
    cfg = B.srmhd_config_default()
    for k, v in kw.items():
        setattr(cfg, k, v)
    with pytest.raises(B.SrmhdError) as e:
        B.srmhd_work_bytes(cfg)
    assert e.value.code == B.SRMHD_E_INVAL and "ghost" in B.srmhd_last_error(None)


def test_slab_work_covers_the_ghost_planes(L):
    cfg = B.srmhd_config_default()
    cfg.nz, cfg.ghost_z = 16, 4
    w = B.srmhd_work_bytes(cfg)
    cfg2 = B.srmhd_config_default()
    cfg2.nz = 24
    assert w == B.srmhd_work_bytes(cfg2)


def test_null_context_stage_and_halo_calls(L):
    n = C.c_size_t()
    assert L.srmhd_stage_begin(None, 1) == B.SRMHD_E_INVAL
    assert L.srmhd_stage_end(None, 1, None) == B.SRMHD_E_INVAL
    assert L.srmhd_local_amax(None, None) == B.SRMHD_E_INVAL
    assert L.srmhd_halo_count(None, C.byref(n)) == B.SRMHD_E_INVAL
    assert L.srmhd_halo_pack(None, 0, None) == B.SRMHD_E_INVAL
    assert L.srmhd_halo_unpack(None, 0, None) == B.SRMHD_E_INVAL


def test_noalloc_forward_checks_before_any_launch(L):
    """Batch limits and null pointers are refused on the host (no device call:
    this runs without a GPU)."""
    p = 256
    for batch in (0, B.MLP_NOALLOC_MAX_BATCH + 1):
        rc = L.srmhd_mlp_forward_noalloc(C.c_void_p(p), C.c_void_p(p), C.c_void_p(p),
                                         C.c_void_p(p), batch, None)
        assert rc == B.SRMHD_E_INVAL
        assert "65536" in B.srmhd_last_error(None)
    rc = L.srmhd_mlp_forward_noalloc(None, C.c_void_p(p), C.c_void_p(p), C.c_void_p(p), 8, None)
    assert rc == B.SRMHD_E_INVAL
