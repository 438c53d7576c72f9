"""Seeded synthetic inputs for the SDMD PIC step.

This module only draws initial states: grids, particle sets and initial
fields.  It holds none of the method's arithmetic (no shape functions, no
push, no deposition, no Maxwell solve) and is the one module that both the
HIP path and the CPU oracle tests consume.

The paper's own workload (a laser-wakefield run in azimuthal-mode geometry,
section 3.1-3.2) is not reproducible here; these Cartesian inputs take its
shapes instead: a vacuum region, a linear density up-ramp then a plateau
(section 3.1), regularly placed cold macro-particles (section 3.2), and
density contrasts that make patches uneven (the high-density spot of
section 3.1 that drives the load imbalance).

Every generator is deterministic in its seed.  Positions, momenta and weights
are float64 arrays; ``id`` is uint32 (the particle's index at creation).
Units are normalised (c = 1).  A particle's weight ``w`` is its share of the
local density: the density of a cell divided by its particles per cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 1912040640


def seed_for(cfg_index: int, run: int = 0) -> int:
    return SEED_BASE + cfg_index * 1000 + run


def cfl_dt(d, frac=0.95) -> float:
    return frac / math.sqrt(sum(1.0 / (x * x) for x in d))


@dataclasses.dataclass
class Workload:
    name: str
    dims: int
    n: tuple                      # cells (nx, ny[, nz])
    d: tuple                      # cell sizes
    dt: float
    patch: tuple                  # cells per patch per axis (0 = autotune)
    nreg: tuple                   # regions per axis
    steps: int
    precision: str                # "fp64" or "fp32s"
    parts: dict                   # x y z ux uy uz w (float64), id (uint32)
    # initial fields, float64 (3, nz, ny, nx) each, or None for zero fields.
    # kind 0: E and B at t=0; kind 1: E at t=0, B at t=+dt/2 and Bm at t=0.
    E0: Optional[np.ndarray] = None
    B0: Optional[np.ndarray] = None
    Bm0: Optional[np.ndarray] = None
    field_kind: int = 0
    q: float = -1.0
    m: float = 1.0
    seed: int = 0
    filter: int = 0               # binomial current filter passes (0 = off)
    solver: str = "yee"           # field solver: "yee" or "psatd"
    seg_cap: int = 0              # particles per segment (0 = library default / autotuner)
    tile_x: int = 0               # field-kernel tile width (0 = library default / autotuner)

    @property
    def n_particles(self) -> int:
        return int(len(self.parts["x"]))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0])


def _empty_parts():
    return {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")} | {"id": np.zeros(0, np.uint32)}


def uniform_random_plasma(n, d, ppc, density, vth, rng, dims=2):
    """`ppc` particles per cell at uniform random in-cell positions, Maxwellian
    momenta of standard deviation `vth` per component, weight density/ppc.
    `ppc` and `density` may be scalars or per-cell arrays of shape n[::-1].
    Particles are in cell order (x fastest)."""
    shape = tuple(n[::-1])
    ppc_a = np.broadcast_to(np.asarray(ppc, dtype=np.int64), shape).reshape(-1)
    den_a = np.broadcast_to(np.asarray(density, dtype=np.float64), shape).reshape(-1)
    # per-cell indices, repeated per particle (no per-particle division)
    ix_c = np.broadcast_to(np.arange(n[0], dtype=np.int32)[None, :], (int(np.prod(n[1:])), n[0])).reshape(-1)
    iy_c = np.broadcast_to(np.arange(n[1], dtype=np.int32)[:, None], (n[1], n[0])).reshape(-1)
    if dims == 3:
        iy_c = np.tile(iy_c, n[2])
    N = int(ppc_a.sum())
    out = {
        "x": (np.repeat(ix_c, ppc_a) + rng.random(N)) * d[0],
        "y": (np.repeat(iy_c, ppc_a) + rng.random(N)) * d[1],
    }
    if dims == 3:
        iz_c = np.repeat(np.arange(n[2], dtype=np.int32), n[0] * n[1])
        out["z"] = (np.repeat(iz_c, ppc_a) + rng.random(N)) * d[2]
    else:
        out["z"] = np.zeros(N)
    u = rng.standard_normal((3, N), dtype=np.float32).astype(np.float64) * vth
    out["ux"], out["uy"], out["uz"] = u[0], u[1], u[2]
    out["w"] = np.repeat(den_a / np.maximum(ppc_a, 1), ppc_a)
    out["id"] = np.arange(N, dtype=np.uint32)
    return out


def regular_cold_plasma(n, d, per_axis, density):
    """per_axis^2 particles per cell on a regular lattice (2D), zero momentum,
    only in cells of positive density; weight density/ppc."""
    nx, ny = n
    den = np.asarray(density, dtype=np.float64).reshape(ny, nx)
    jj, ii = np.nonzero(den > 0)
    ppc = per_axis * per_axis
    sub = (np.arange(per_axis) + 0.5) / per_axis
    sx, sy = np.meshgrid(sub, sub, indexing="xy")
    sx, sy = sx.reshape(-1), sy.reshape(-1)
    # cell-major order: all particles of one cell are consecutive
    x = (ii[:, None] + sx[None, :]).reshape(-1) * d[0]
    y = (jj[:, None] + sy[None, :]).reshape(-1) * d[1]
    w = np.repeat(den[jj, ii] / ppc, ppc)
    N = len(x)
    return {"x": x, "y": y, "z": np.zeros(N), "ux": np.zeros(N), "uy": np.zeros(N), "uz": np.zeros(N),
            "w": w, "id": np.arange(N, dtype=np.uint32)}


# --------------------------------------------------------------------------
# C1: small thermal plasma, FP64
# --------------------------------------------------------------------------
def thermal_2d(seed=None, n=(64, 64), d=(0.1, 0.1), ppc=4, vth=0.01, patch=(8, 8), nreg=(1, 1), steps=100,
               precision="fp64", density=1.0, name="thermal64"):
    seed = seed_for(0) if seed is None else seed
    rng = np.random.default_rng(seed)
    parts = uniform_random_plasma(n, d, ppc, density, vth, rng, dims=2)
    return Workload(name=name, dims=2, n=tuple(n), d=tuple(d), dt=cfl_dt(d), patch=tuple(patch),
                    nreg=tuple(nreg), steps=steps, precision=precision, parts=parts, seed=seed)


# --------------------------------------------------------------------------
# C2: laser-wakefield-shaped 2D run
# --------------------------------------------------------------------------
def lwfa_density(nx, ny, vac_end=1088, ramp=256, n0=0.005):
    """vacuum for cells [0, vac_end), linear up-ramp over `ramp` cells (value at
    the cell centre), plateau n0 afterwards."""
    i = np.arange(nx, dtype=np.float64)
    prof = np.where(i < vac_end, 0.0, np.where(i < vac_end + ramp, n0 * (i - vac_end + 0.5) / ramp, n0))
    return np.broadcast_to(prof[None, :], (ny, nx)).copy()


def laser_profile(x, y, a0, y0, waist, x0, duration):
    """Gaussian pulse: transverse 1/e field radius `waist`, intensity FWHM
    `duration` (field envelope exp(-2 ln2 (x-x0)^2 / duration^2)), carrier
    cos(x - x0) (k0 = 1); cut to zero where the envelope is below 1e-3."""
    env_x = np.exp(-2.0 * math.log(2.0) * (x - x0) ** 2 / duration ** 2)
    env_x = np.where(np.abs(x - x0) > 67.0, 0.0, env_x)
    return a0 * np.exp(-((y - y0) ** 2) / waist ** 2) * env_x * np.cos(x - x0)


def lwfa_2d(n=(2048, 256), d=(0.125, 0.5), patch=(16, 16), nreg=(4, 1), steps=1000, precision="fp32s",
            a0=2.0, waist=40.0, duration=30.0, per_axis=4, vac_end=1088, ramp=256, n0=0.005, x0=68.0,
            seed=None, name="lwfa2048x256"):
    seed = seed_for(1) if seed is None else seed
    nx, ny = n
    dt = cfl_dt(d)
    den = lwfa_density(nx, ny, vac_end, ramp, n0)
    parts = regular_cold_plasma(n, d, per_axis, den)
    y0 = 0.5 * ny * d[1]
    shape = (1, ny, nx)
    E = np.zeros((3,) + shape)
    B = np.zeros((3,) + shape)
    Bm = np.zeros((3,) + shape)
    ii = np.arange(nx, dtype=np.float64)[None, :]
    jj = np.arange(ny, dtype=np.float64)[:, None]
    # Ey sits at (i, j+1/2); Bz at (i+1/2, j+1/2).  +x propagation: Bz = Ey(x - t).
    E[1, 0] = laser_profile(ii * d[0], (jj + 0.5) * d[1], a0, y0, waist, x0, duration)
    xb = (ii + 0.5) * d[0]
    yb = (jj + 0.5) * d[1]
    B[2, 0] = laser_profile(xb - 0.5 * dt, yb, a0, y0, waist, x0, duration)
    Bm[2, 0] = laser_profile(xb, yb, a0, y0, waist, x0, duration)
    return Workload(name=name, dims=2, n=tuple(n), d=tuple(d), dt=dt, patch=tuple(patch), nreg=tuple(nreg),
                    steps=steps, precision=precision, parts=parts, E0=E, B0=B, Bm0=Bm, field_kind=1, seed=seed)


# --------------------------------------------------------------------------
# C3: 3D thermal plasma with a dense cylinder along x
# --------------------------------------------------------------------------
def cylinder_3d(n=(512, 128, 128), d=(0.2, 0.2, 0.2), ppc_bg=8, ppc_cyl=128, radius=16.0, vth=0.05,
                patch=(8, 8, 8), steps=200, precision="fp32s", seed=None, name="cyl512x128x128"):
    seed = seed_for(2) if seed is None else seed
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    jc, kc = 0.5 * ny, 0.5 * nz
    jj = np.arange(ny)[None, :] + 0.5 - jc
    kk = np.arange(nz)[:, None] + 0.5 - kc
    inside = (jj ** 2 + kk ** 2) < radius ** 2          # (nz, ny)
    ppc = np.where(inside[:, :, None], ppc_cyl, ppc_bg) * np.ones((nz, ny, nx), dtype=np.int64)
    w_bg = 1.0 / ppc_bg
    # every particle carries the background weight: the cylinder is 16x denser
    density = ppc * w_bg
    parts = uniform_random_plasma(n, d, ppc, density, vth, rng, dims=3)
    return Workload(name=name, dims=3, n=tuple(n), d=tuple(d), dt=cfl_dt(d), patch=tuple(patch),
                    nreg=(1, 1, 1), steps=steps, precision=precision, parts=parts, seed=seed)


# --------------------------------------------------------------------------
# C4: batched parameter scan
# --------------------------------------------------------------------------
C4_GRIDS = [(64, 64), (128, 128), (256, 256), (512, 128)]


def scan_run(run: int, steps=500, patch=(0, 0), precision="fp32s", cfg_index=3):
    seed = seed_for(cfg_index, run)
    rng = np.random.default_rng(seed)
    n = C4_GRIDS[int(rng.integers(0, len(C4_GRIDS)))]
    ppc = int(rng.integers(4, 33))
    vth = float(10 ** rng.uniform(-3, -1))
    d = (0.1, 0.1)
    parts = uniform_random_plasma(n, d, ppc, 1.0, vth, rng, dims=2)
    return Workload(name=f"scan{run}", dims=2, n=n, d=d, dt=cfl_dt(d), patch=tuple(patch), nreg=(1, 1),
                    steps=steps, precision=precision, parts=parts, seed=seed)


def scan_batch(n_runs=256, steps=500, patch=(0, 0), precision="fp32s"):
    return [scan_run(r, steps=steps, patch=patch, precision=precision) for r in range(n_runs)]


# --------------------------------------------------------------------------
# C5: served request stream
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival: float     # seconds after stream start
    n: tuple
    ppc: int
    vth: float
    ramp: bool
    steps: int
    seed: int


def request_stream(rate, window_s=60.0, seed=None, max_requests=None, steps_range=(200, 2000),
                   nx_pow=(6, 10), ny_pow=(6, 8)):
    """Poisson arrivals at `rate` runs/s over `window_s` seconds."""
    seed = seed_for(4) if seed is None else seed
    rng = np.random.default_rng(seed + int(rate * 1000))
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= window_s:
            break
        nx = 2 ** int(rng.integers(nx_pow[0], nx_pow[1] + 1))
        ny = 2 ** int(rng.integers(ny_pow[0], ny_pow[1] + 1))
        out.append(Request(rid=len(out), arrival=t, n=(nx, ny), ppc=int(rng.integers(4, 33)),
                           vth=float(10 ** rng.uniform(-3, -1)), ramp=bool(rng.random() < 0.5),
                           steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
                           seed=seed_for(4, len(out))))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out


def request_workload(req: Request, patch=(0, 0), precision="fp32s"):
    rng = np.random.default_rng(req.seed)
    nx, ny = req.n
    d = (0.1, 0.1)
    if req.ramp:
        i = np.arange(nx, dtype=np.float64)
        ramp_end = nx // 4
        prof = np.where(i < ramp_end, (i + 0.5) / ramp_end, 1.0)
        dens = np.broadcast_to(prof[None, :], (ny, nx))
    else:
        dens = np.ones((ny, nx))
    parts = uniform_random_plasma(req.n, d, req.ppc, dens, req.vth, rng, dims=2)
    return Workload(name=f"req{req.rid}", dims=2, n=req.n, d=d, dt=cfl_dt(d), patch=tuple(patch), nreg=(1, 1),
                    steps=req.steps, precision=precision, parts=parts, seed=req.seed)


# --------------------------------------------------------------------------
# small fixtures for tests
# --------------------------------------------------------------------------
def single_particle(x, y, z=0.0, ux=0.0, uy=0.0, uz=0.0, w=1.0):
    return {"x": np.array([x], float), "y": np.array([y], float), "z": np.array([z], float),
            "ux": np.array([ux], float), "uy": np.array([uy], float), "uz": np.array([uz], float),
            "w": np.array([w], float), "id": np.zeros(1, np.uint32)}


def concat_parts(*ps):
    out = {k: np.concatenate([p[k] for p in ps]) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    out["id"] = np.arange(len(out["x"]), dtype=np.uint32)
    return out
