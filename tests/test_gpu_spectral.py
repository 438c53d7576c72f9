"""Parity of the spectral (PSATD) field phase on the GPU with the oracle:
lattice plane waves against their closed form at a time step beyond the Yee
limit, full steps with particles against the oracle's spectral step, and
the Gauss law on the GPU's own data."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle as O
from oracle import psatd as PS
from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL
from tests.helpers import family_errors
from tests.test_oracle_pins import _lattice_wave, _thermal_parts

pytestmark = pytest.mark.gpu

MASK = B.F_E | B.F_B | B.F_BH | B.F_J


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_fields(wl, steps):
    with B.Context([wl], track_ids=True) as ctx:
        if steps:
            ctx.step(steps)
        F = ctx.fields(0, MASK)
        parts = B.sort_by_id(ctx.particles(0)) if wl.n_particles else None
    return {"E": F[0:3], "Bm": F[3:6], "B": F[6:9], "J": F[9:12]}, parts


def oracle_psatd(wl, steps):
    g = O.Grid(wl.dims, wl.n, wl.d, wl.dt, q=wl.q, m=wl.m, patch=wl.patch, filter=wl.filter)
    F = g.zeros_fields()
    if wl.E0 is not None:
        F[0:3] = wl.E0
        F[3:6] = wl.Bm0 if (wl.field_kind == 1 and wl.Bm0 is not None) else wl.B0
    PS.init_fields(F)
    p = wl.parts
    P = O.Particles(x=p["x"], y=p["y"], z=p["z"], ux=p["ux"], uy=p["uy"], uz=p["uz"], w=p["w"])
    for _ in range(steps):
        PS.step(g, F, P)
    return {"E": F[0:3], "Bm": F[6:9], "B": F[3:6], "J": F[9:12]}, P, g


def fam_err(a, b):
    out = {}
    for k in ("E", "B", "J"):
        nb = np.linalg.norm(b[k])
        out[k] = float(np.abs(a[k]).max()) if nb == 0 else max(family_errors(a[k], b[k]))
    return out


@pytest.mark.parametrize("dims,m,e_dir", [(2, (3, 2, 0), (0, 0, 1)), (2, (1, 4, 0), (1, 0, 0)),
                                          (3, (2, 1, 3), (1, -1, 0.5))])
def test_spectral_vacuum_wave_exact_on_gpu(dims, m, e_dir):
    say(f"case: spectral vacuum wave dims={dims}")
    n = (64, 32) if dims == 2 else (16, 8, 32)
    d = (0.1, 0.15) if dims == 2 else (0.2, 0.1, 0.15)
    dt = 0.95 * min(d)                          # beyond the Yee limit
    g = O.Grid(dims, n, d, dt)
    F, w = _lattice_wave(g, m, e_dir, 0.0)
    parts = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    parts["id"] = np.zeros(0, np.uint32)
    wl = WL.Workload(name="wave", dims=dims, n=n, d=d, dt=dt, patch=(8,) * dims, nreg=(1,) * dims, steps=0,
                     precision="fp64", parts=parts, E0=F[0:3], B0=F[3:6], Bm0=F[6:9], field_kind=1, solver="psatd")
    Fg, _ = gpu_fields(wl, 30)
    ref, _ = _lattice_wave(g, m, e_dir, 30 * dt)
    err = max(np.abs(Fg["E"] - ref[0:3]).max(), np.abs(Fg["B"] - ref[3:6]).max())
    say(f"max error after 30 steps: {err:.3e}")
    assert err < 1e-11


@pytest.mark.parametrize("dims,n", [(2, (32, 16)), (3, (8, 16, 8)), (2, (16, 512)), (3, (4, 8, 512))])
def test_spectral_white_noise_fields_match_oracle(dims, n):
    """Random E, B (no particles) carry every wavevector at full amplitude,
    the Nyquist planes of each axis included.  The oracle steps every
    wavevector of each component's full spectrum and keeps the real part of
    the inverse; the GPU transforms the real components two to a complex
    array, steps k and obtains -k by conjugation, so this checks the
    splitting, the repacking and the symmetry of the step everywhere.  The
    512-node last axes take the separate k-space launch."""
    say(f"case: spectral white noise dims={dims} n={n}")
    d = (0.1, 0.15, 0.12)[:dims]
    dt = 0.9 * min(d)
    rng = np.random.default_rng(11 + dims)
    g = O.Grid(dims, n, d, dt)
    F = g.zeros_fields()
    F[0:6] = rng.standard_normal(F[0:6].shape)
    E0, B0 = F[0:3].copy(), F[3:6].copy()
    PS.init_fields(F)
    for _ in range(4):
        PS.step_fields(g, F)
    parts = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    parts["id"] = np.zeros(0, np.uint32)
    wl = WL.Workload(name="noise", dims=dims, n=n, d=d, dt=dt, patch=(4,) * dims, nreg=(1,) * dims, steps=0,
                     precision="fp64", parts=parts, E0=E0, B0=B0, Bm0=B0, field_kind=1, solver="psatd")
    Fg, _ = gpu_fields(wl, 4)
    err = max(np.abs(Fg["E"] - F[0:3]).max(), np.abs(Fg["B"] - F[3:6]).max(), np.abs(Fg["Bm"] - F[6:9]).max())
    say(f"max error after 4 steps: {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("prec,tol1,tol20", [("fp64", 1e-12, 1e-9), ("fp32s", 1e-5, 1e-3)])
def test_spectral_steps_match_oracle(prec, tol1, tol20):
    say(f"case: spectral thermal {prec}")
    wl = dataclasses.replace(WL.thermal_2d(n=(64, 32), ppc=4, vth=0.05, patch=(8, 8), precision=prec),
                             solver="psatd", dt=0.09)
    Fo, P, g = oracle_psatd(wl, 1)
    Fg, gp = gpu_fields(wl, 1)
    e1 = fam_err(Fg, Fo)
    Fo20, P20, _ = oracle_psatd(wl, 20)
    Fg20, gp20 = gpu_fields(wl, 20)
    e20 = fam_err(Fg20, Fo20)
    say(f"{prec}: 1-step {e1}; 20-step {e20}")
    assert max(e1.values()) < tol1
    assert max(e20.values()) < tol20
    if prec == "fp64":
        L = wl.n[0] * wl.d[0]
        dx = np.abs(gp["x"] - P.x)
        assert np.minimum(dx, L - dx).max() < 1e-13


def test_spectral_long_last_axis_matches_oracle():
    """Lines along the last axis longer than the fused line kernel takes
    (512 > 256 nodes) go through separate transform and k-space launches;
    both routes must give the oracle's step."""
    say("case: spectral thermal 16x512 fp64 (unfused last axis)")
    wl = dataclasses.replace(WL.thermal_2d(n=(16, 512), ppc=2, vth=0.05, patch=(8, 8), precision="fp64"),
                             solver="psatd", dt=0.09)
    Fo, _, _ = oracle_psatd(wl, 5)
    Fg, _ = gpu_fields(wl, 5)
    e = fam_err(Fg, Fo)
    say(f"5-step {e}")
    assert max(e.values()) < 1e-10


def test_spectral_3d_and_filter_match_oracle():
    say("case: spectral 3D fp64 with filter")
    wl = dataclasses.replace(WL.cylinder_3d(n=(16, 16, 16), radius=3.0, ppc_bg=2, ppc_cyl=16, patch=(4, 4, 4),
                                            precision="fp64"), solver="psatd", filter=2)
    Fo, _, _ = oracle_psatd(wl, 3)
    Fg, _ = gpu_fields(wl, 3)
    e = fam_err(Fg, Fo)
    say(f"3-step {e}")
    assert max(e.values()) < 1e-11


def test_spectral_3d_anisotropic_split_form_matches_oracle():
    """A 3D grid with three different sizes (32 x 8 x 16: adjacent-pair and
    leftover line groups, transforms of three lengths) in the FP32 split
    form against the FP64 oracle."""
    say("case: spectral 3D 32x8x16 fp32s")
    wl = dataclasses.replace(WL.cylinder_3d(n=(32, 8, 16), radius=2.0, ppc_bg=2, ppc_cyl=8, patch=(4, 4, 4),
                                            precision="fp32s"), solver="psatd")
    Fo, _, _ = oracle_psatd(wl, 2)
    Fg, _ = gpu_fields(wl, 2)
    e = fam_err(Fg, Fo)
    say(f"2-step {e}")
    assert max(e.values()) < 1e-5   # measured 1.5e-7: FP32 particles, FP64 fields


def test_spectral_gauss_law_on_gpu_data():
    say("case: spectral gauss fp64")
    wl = dataclasses.replace(WL.thermal_2d(n=(64, 64), ppc=4, vth=0.1, precision="fp64"), solver="psatd")
    with B.Context([wl]) as ctx:
        r0 = ctx.fields(0, B.F_RHO)[0]
        ctx.step(20)
        F = ctx.fields(0, B.F_RHO | B.F_E)
    E, r1 = F[0:3], F[3]
    dx, dy = wl.d
    divE = (E[0] - np.roll(E[0], 1, axis=2)) / dx + (E[1] - np.roll(E[1], 1, axis=1)) / dy
    scale = np.abs(r0).max()
    say(f"gauss residual: {np.abs(divE - (r1 - r0)).max() / scale:.3e}")
    assert np.abs(divE - (r1 - r0)).max() < 1e-11 * scale


def test_spectral_and_yee_runs_in_one_batch():
    """A spectral run and a Yee run stepped together (separate field classes
    in one context) give what each gives alone."""
    say("case: batch spectral + yee")
    a = dataclasses.replace(WL.thermal_2d(n=(64, 32), ppc=4, vth=0.05, patch=(8, 8), precision="fp64"),
                            solver="psatd", dt=0.09)
    b = WL.thermal_2d(n=(32, 32), ppc=4, vth=0.05, patch=(8, 8), precision="fp64")
    with B.Context([a, b]) as ctx:
        ctx.step(5)
        Fa, Fb = ctx.fields(0, MASK), ctx.fields(1, MASK)
    for wl, F in ((a, Fa), (b, Fb)):
        with B.Context([wl]) as ctx:
            ctx.step(5)
            G = ctx.fields(0, MASK)
        assert np.abs(F - G).max() <= 1e-12 * max(np.abs(G).max(), 1e-30)
