"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol include/lbm_vans.h declares, sizes its work buffer, and rejects invalid
parameters before touching the device."""
import ctypes
import math
import os
import re

import pytest

from paper_1406_6438_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_vans.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_vans_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(lbm.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lbm.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert lbm.load().lbm_vans_abi_version() == lbm.ABI_VERSION


def test_header_constants_match_binding():
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(LBM_\w+)\s+\(?(-?\d+)\)?", src))
    assert int(consts["LBM_VANS_ABI_VERSION"]) == lbm.ABI_VERSION
    assert int(consts["LBM_VANS_EINVAL"]) == lbm.EINVAL
    assert int(consts["LBM_VANS_ENONFINITE"]) == lbm.ENONFINITE
    assert int(consts["LBM_VANS_ENOTIMPL"]) == lbm.ENOTIMPL
    assert int(consts["LBM_F32_SHIFTED"]) == lbm.F32_SHIFTED
    assert int(consts["LBM_F16_SHIFTED"]) == lbm.F16_SHIFTED
    assert int(consts["LBM_BC_BOUNCEBACK"]) == lbm.BC_BOUNCEBACK
    assert int(consts["LBM_DRAG_CONST"]) == lbm.DRAG_CONST
    assert int(consts["LBM_VANS_NDIAG"]) == lbm.NDIAG
    assert int(consts["LBM_VANS_DIAG_RING"]) == lbm.DIAG_RING
    assert int(consts["LBM_BC_OPEN"]) == lbm.BC_OPEN
    assert int(consts["LBM_OBJ_OUTLET_FLUX"]) == lbm.OBJ_OUTLET_FLUX
    assert int(consts["LBM_BC_INOUT"]) == lbm.BC_INOUT
    assert int(consts["LBM_VANS_WMACH"]) == lbm.WMACH
    assert float(re.search(r"#define\s+LBM_VANS_MACH_WARN\s+([0-9.]+)", src).group(1)) == lbm.MACH_WARN
    m = re.search(r"#define\s+LBM_VANS_GRAD_STATIC_BYTES\s+\(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == lbm.GRAD_STATIC_BYTES


def test_work_bytes_scale_with_storage():
    p32 = lbm.Params(Lx=4096, Ly=4096, tau=0.6, storage=lbm.F32_SHIFTED, d_p=13.0)
    p16 = lbm.Params(Lx=4096, Ly=4096, tau=0.6, storage=lbm.F16_SHIFTED, d_p=13.0)
    p64 = lbm.Params(Lx=4096, Ly=4096, tau=0.6, storage=lbm.F64, d_p=13.0)
    cells = 4096 * 4096
    n32, n16, n64 = (lbm.lbm_vans_work_bytes(p) for p in (p32, p16, p64))
    # two population buffers + porosity + small partial/diagnostic areas
    assert 2 * 9 * 4 * cells + 4 * cells <= n32 < 2 * 9 * 4 * cells + 4 * cells + 8 << 20
    assert 2 * 9 * 2 * cells + 4 * cells <= n16 < 2 * 9 * 2 * cells + 4 * cells + 8 << 20
    assert 2 * 9 * 8 * cells + 8 * cells <= n64 < 2 * 9 * 8 * cells + 8 * cells + 8 << 20


@pytest.mark.parametrize("bad", [
    dict(Lx=0), dict(Ly=-3), dict(tau=0.5), dict(tau=math.nan), dict(d_p=0.0),
    dict(d_p=-1.0), dict(storage=7), dict(bc_x=4), dict(bc_y=2), dict(bc_y=3), dict(bc_y=5),
    dict(drag=3), dict(bc_x=2, Lx=1), dict(bc_x=2, rho_in=0.0), dict(bc_x=2, u_out=math.inf),
    dict(bc_x=3, Lx=1), dict(bc_x=3, rho_out=0.0), dict(bc_x=3, u_in=math.nan),
    dict(drag=lbm.DRAG_CONST, K=0.0), dict(drag=lbm.DRAG_CONST, K=1.0, F_eps=-1.0),
    dict(rho0=0.0), dict(G=(math.inf, 0.0)), dict(u0=(0.0, math.nan)),
    dict(storage=lbm.F16_SHIFTED, fp16_scale_log2=30), dict(diag_every=-1),
    dict(Lx=65536, Ly=65536), dict(u_wall=(0.01, 0.0)), dict(bc_y=1, u_wall=(math.nan, 0.0)),
    dict(sweep_vec=3), dict(sweep_vec=4, storage=lbm.F64), dict(sweep_vec=2),
    dict(steps_per_pass=5), dict(steps_per_pass=-1), dict(steps_per_pass=4, storage=lbm.F16_SHIFTED),
    dict(steps_per_pass=4, storage=lbm.F64),
    dict(pass_rows=16), dict(pass_rows=-24), dict(pass_rows=28, storage=lbm.F16_SHIFTED),
    dict(pass_rows=12, storage=lbm.F16_SHIFTED), dict(pass_rows=12, storage=lbm.F64),
    dict(pass_rows=6, storage=lbm.F16_SHIFTED), dict(pass_rows=8),
    dict(pass_rows=24, storage=lbm.F64),
])
def test_invalid_params_rejected_without_gpu(bad):
    kw = dict(Lx=16, Ly=8, tau=0.7, d_p=10.0)
    kw.update(bad)
    p = lbm.Params(**kw)
    with pytest.raises(lbm.LbmVansError) as ei:
        lbm.lbm_vans_work_bytes(p)
    assert ei.value.code == lbm.EINVAL
    L = lbm.load()
    h = ctypes.c_void_p()
    rc = L.lbm_vans_init(ctypes.byref(p.c()), 256, 256, 1 << 30, None, ctypes.byref(h))
    assert rc == lbm.EINVAL and not h.value
    assert L.lbm_vans_last_error()


def test_init_rejects_short_or_misaligned_work_without_gpu():
    p = lbm.Params(Lx=16, Ly=8, tau=0.7, d_p=10.0)
    need = lbm.lbm_vans_work_bytes(p)
    L = lbm.load()
    h = ctypes.c_void_p()
    assert L.lbm_vans_init(ctypes.byref(p.c()), 256, 256, need - 1, None, ctypes.byref(h)) == lbm.EINVAL
    assert b"needed" in L.lbm_vans_last_error()
    assert L.lbm_vans_init(ctypes.byref(p.c()), 256, 260, need, None, ctypes.byref(h)) == lbm.EINVAL
    assert b"aligned" in L.lbm_vans_last_error()
    assert L.lbm_vans_init(ctypes.byref(p.c()), None, 256, need, None, ctypes.byref(h)) == lbm.EINVAL


def test_null_handle_calls_fail_cleanly():
    L = lbm.load()
    assert L.lbm_vans_step(None, 1) == lbm.EINVAL
    assert L.lbm_vans_moments(None, None, None, None, None, None) == lbm.EINVAL
    assert L.lbm_vans_step_count(None) == -1
    L.lbm_vans_destroy(None)
    assert L.lbm_vans_grad(None, 0, 1, 1, None, 0, None, None) == lbm.EINVAL
    p = lbm.Params(Lx=16, Ly=8, tau=0.7, d_p=10.0)
    assert L.lbm_vans_grad_work_bytes(ctypes.byref(p.c()), 1, 10, 5) == 0   # unknown objective
    assert L.lbm_vans_grad_work_bytes(ctypes.byref(p.c()), 0, 10, 0) == 0   # ckpt_every < 1
    n1 = lbm.lbm_vans_grad_work_bytes(p, 0, 100, 10)
    n2 = lbm.lbm_vans_grad_work_bytes(p, 0, 100, 50)
    n3 = lbm.lbm_vans_grad_work_bytes(p, 0, 40, 50)
    pop = 9 * 8 * 256 * 4
    # checkpoints + two sets of segment buffers when there are two or more segments
    # (one recomputed beside the reverse steps of the next), one set otherwise
    assert n1 >= (10 + 2 * 10) * pop and n2 >= (2 + 2 * 50) * pop
    assert (1 + 50) * pop <= n3 < (1 + 2 * 50) * pop


def test_null_batch_calls_fail_cleanly():
    L = lbm.load()
    out = ctypes.c_void_p()
    assert L.lbm_vans_batch_work_bytes(None, 0) == 0
    assert L.lbm_vans_batch_create(None, 0, None, 0, None, ctypes.byref(out)) == lbm.EINVAL
    assert out.value is None
    no_members = (ctypes.c_void_p * 2)(None, None)
    assert L.lbm_vans_batch_work_bytes(no_members, 2) == 0
    assert L.lbm_vans_batch_create(no_members, 2, None, 0, None, ctypes.byref(out)) == lbm.EINVAL
    assert b"NULL" in L.lbm_vans_last_error()
    cfg = lbm.LbmVansBatchConfig(4, 0, 16, 0, 0, 0.0)
    assert L.lbm_vans_batch_configure(None, ctypes.byref(cfg)) == lbm.EINVAL
    assert L.lbm_vans_batch_get_config(None, ctypes.byref(cfg)) == lbm.EINVAL
    assert L.lbm_vans_batch_tune(None, 3, None, None, 0, None) == lbm.EINVAL
    assert L.lbm_vans_batch_step(None, 1) == lbm.EINVAL
    assert L.lbm_vans_batch_grad_work_bytes(None, 0, 10, 5) == 0
    assert L.lbm_vans_batch_grad(None, 0, 10, 5, None, 0, None, None) == lbm.EINVAL
    assert L.lbm_vans_pass_plan(None, None, None) == lbm.EINVAL
    assert L.lbm_vans_batch_pass_plan(None, None, None) == lbm.EINVAL
    L.lbm_vans_batch_destroy(None)


def test_binding_fails_loudly_when_library_missing(tmp_path):
    import importlib
    mod = importlib.import_module("paper_1406_6438_amd.lbm")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(ImportError):
            mod.load(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved


@pytest.mark.parametrize("cname, pystruct", [("lbm_vans_params", "LbmVansParams"),
                                             ("lbm_vans_batch_config", "LbmVansBatchConfig")])
def test_struct_layouts_match_header(tmp_path, cname, pystruct):
    """The ctypes mirrors of the header's structs have the same size and the same
    offset for every field (a C program built against include/lbm_vans.h prints
    them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    S = getattr(lbm, pystruct)
    names = [f[0] for f in S._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm_vans.h"',
             'int main(void) {',
             f'  printf("size %zu\\n", sizeof({cname}));']
    lines += [f'  printf("{n} %zu\\n", offsetof({cname}, {n}));' for n in names]
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(out["size"]) == ctypes.sizeof(S)
    for n in names:
        assert int(out[n]) == getattr(S, n).offset, n
