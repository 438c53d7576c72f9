"""Host-side checks of the C ABI library: it loads, exports every entry point
the header declares, and validates configurations without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sdmd_pic.h")).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.load()
    names = _declared()
    assert set(names) == set(B.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_strerror_texts():
    L = B.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert L.pic_strerror(code) and L.pic_strerror(code) != b"unknown error"
    assert B.PIC_E_OVERFLOW == -8
    assert L.pic_strerror(-99) == b"unknown error"


def _cfg(**over):
    wl = WL.thermal_2d(n=(32, 32), ppc=1)
    for k, v in over.items():
        setattr(wl, k, v)
    return wl


@pytest.mark.parametrize("change,msg", [
    (dict(patch=(3, 8)), "patch size must be >= 4"),
    (dict(patch=(6, 8)), "divide"),
    (dict(patch=(64, 8)), "<= 32"),
    (dict(dt=1.0), "dt must satisfy"),
    (dict(nreg=(3, 1)), "whole patches"),
    (dict(dims=4), "dims must be 2 or 3"),
    (dict(filter=5), "filter_passes"),
    (dict(solver="psatd", nreg=(2, 1)), "one region"),
    (dict(solver="psatd", n=(48, 32)), "powers of two"),
    (dict(solver="psatd", dt=0.2), "dt must satisfy 0 < dt < min d"),
    (dict(seg_cap=100), "seg_cap"),
    (dict(seg_cap=70000), "seg_cap"),
    (dict(tile_x=24), "field_tile_x"),
])
def test_config_validation(change, msg):
    wl = _cfg(**change)
    with pytest.raises(B.PicError) as e:
        B.mem_bytes(wl)
    assert e.value.code == B.PIC_E_CONFIG
    assert msg in str(e.value)


def test_spectral_solver_accepts_dt_beyond_the_yee_limit():
    """The spectral step has no Courant limit; dt only has to keep particles
    under a cell per step (dt < min d)."""
    wl = _cfg(solver="psatd", dt=0.09)      # Yee limit here: 0.1/sqrt(2) = 0.0707
    assert B.mem_bytes(wl) > B.mem_bytes(_cfg())
    with pytest.raises(B.PicError):
        B.mem_bytes(_cfg(dt=0.09))


def test_mem_bytes_scales_with_particles():
    a = B.mem_bytes(WL.thermal_2d(n=(64, 64), ppc=4, patch=(8, 8)))
    b = B.mem_bytes(WL.thermal_2d(n=(64, 64), ppc=16, patch=(8, 8)))
    assert b > a > 64 * 64 * 18 * 8


def test_init_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = B.load()
    ctx = C.c_void_p()
    rc = L.pic_init(None, 0, None, C.byref(ctx))
    assert rc == B.PIC_E_DEVICE


def _instantiations(src, macro):
    txt = open(os.path.join(ROOT, "paper_1912_04064_amd", "csrc", src)).read()
    out = set()
    for args in re.findall(macro + r"\(([^)]*)\)", txt):
        a = [x.strip() for x in args.split(",")]
        if not a[0].isdigit():
            continue        # the macro's own definition
        out.add(tuple(int(x) if x.lstrip("-").isdigit() else {"true": True, "false": False}.get(x, x) for x in a))
    return out


def test_paths_table_names_every_kernel_instantiation():
    """The oracle-compared path cases (tests/test_gpu_paths.py) cover every
    particle-kernel and field-kernel instantiation compiled into the
    library, and name none that is not compiled."""
    from tests import test_gpu_paths as T
    push = _instantiations("k_push.hip", "PUSH_CASE")
    yee = _instantiations("k_fields.hip", "YEE_CASE")
    assert len(push) >= 15 and len(yee) >= 24
    assert T.push_instantiations() == push
    assert T.yee_instantiations() == yee


def test_3d_filter_takes_the_narrow_field_tile_only():
    wl = WL.cylinder_3d(n=(16, 16, 16), radius=3.0, ppc_bg=1, ppc_cyl=2, patch=(8, 8, 8))
    wl.filter = 1
    wl.tile_x = 16
    with pytest.raises(B.PicError) as e:
        B.mem_bytes(wl)
    assert e.value.code == B.PIC_E_CONFIG and "field_tile_x" in str(e.value)
    wl.tile_x = 8
    assert B.mem_bytes(wl) > 0


def test_mem_bytes_bounds_the_autotuners_choices():
    """With the patch left to the autotuner, pic_mem_bytes is the most any
    candidate (patch edge x segment capacity) can take."""
    auto = WL.thermal_2d(n=(128, 64), ppc=8, patch=(0, 0))
    worst = 0
    for p in (8, 16, 32):
        for cap in (1024, 2048, 4096):
            wl = WL.thermal_2d(n=(128, 64), ppc=8, patch=(p, p))
            wl.seg_cap = cap
            worst = max(worst, B.mem_bytes(wl))
    assert B.mem_bytes(auto) == worst
