"""FP64 CPU oracle of the SDMD particle-in-cell step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links or calls
it, and it shares no code with the HIP path; both sides only share the seeded
input generators, which hold none of the method's arithmetic.

The arithmetic lives in ``pic_oracle.c`` (plain C, FP64, single thread); this
module is argument marshalling through ctypes.  See that file's header for the
equations, the staggering and the readings taken where the paper is silent.

Field arrays are numpy float64 of shape ``(12, nz, ny, nx)`` with components
``Ex Ey Ez Bx By Bz Bmx Bmy Bmz Jx Jy Jz`` (B at t^{n+1/2}, Bm at t^n).
Particle sets are dicts of float64 arrays ``x y z ux uy uz w`` (``z`` ignored in
2D).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EX, EY, EZ, BX, BY, BZ, BMX, BMY, BMZ, JX, JY, JZ = range(12)
NCOMP = 12


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, -O2, no fast-math, no contraction):
    the parity build (single thread), and a timing build of the same source
    with OpenMP, which only the CPU-baseline leg of the benchmark loads."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", *_FLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    if force or not os.path.exists(_LIB_OMP):
        subprocess.check_call(["gcc", *_FLAGS, "-fopenmp", "-o", _LIB_OMP + ".tmp", _SRC, "-lm"])
        os.replace(_LIB_OMP + ".tmp", _LIB_OMP)
    return _LIB


class OCfg(C.Structure):
    _fields_ = [
        ("dims", C.c_int32),
        ("n", C.c_int32 * 3),
        ("d", C.c_double * 3),
        ("dt", C.c_double),
        ("q", C.c_double),
        ("m", C.c_double),
        ("patch", C.c_int32 * 3),
        ("nreg", C.c_int32 * 3),
        ("filter", C.c_int32),
    ]


class OParts(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
        ("ux", C.POINTER(C.c_double)), ("uy", C.POINTER(C.c_double)), ("uz", C.POINTER(C.c_double)),
        ("w", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_S.restype = C.c_double
        L.oracle_S.argtypes = [C.c_double]
        L.oracle_interp.argtypes = [C.POINTER(OCfg), dp, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_boris.argtypes = [C.c_double, C.c_double, dp, dp]
        L.oracle_gamma.restype = C.c_double
        L.oracle_gamma.argtypes = [dp]
        L.oracle_deposit_one.argtypes = [C.POINTER(OCfg), dp, dp, dp, C.c_double, C.c_double]
        L.oracle_yee.argtypes = [C.POINTER(OCfg), dp]
        L.oracle_init_fields.argtypes = [C.POINTER(OCfg), dp]
        L.oracle_filter.argtypes = [C.POINTER(OCfg), dp, C.c_int32, C.c_int32]
        L.oracle_wrap.restype = C.c_double
        L.oracle_wrap.argtypes = [C.c_double, C.c_double]
        L.oracle_cell.restype = C.c_int64
        L.oracle_cell.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.oracle_bin.argtypes = [C.POINTER(OCfg), C.POINTER(OParts), C.POINTER(C.c_int32)]
        L.oracle_split.argtypes = [C.c_double, C.c_double, C.c_int64, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_float)]
        L.oracle_particles_sdsd.restype = C.c_double
        L.oracle_particles_sdsd.argtypes = [C.POINTER(OCfg), dp, C.POINTER(OParts)]
        L.oracle_push_only.argtypes = [C.POINTER(OCfg), dp, C.POINTER(OParts)]
        L.oracle_step_sdsd.restype = C.c_double
        L.oracle_step_sdsd.argtypes = [C.POINTER(OCfg), dp, C.POINTER(OParts)]
        L.oracle_step_sdmd.restype = C.c_int
        L.oracle_step_sdmd.argtypes = [C.POINTER(OCfg), dp, C.POINTER(OParts), C.c_int32]
        L.oracle_deposit_moves.restype = C.c_int
        L.oracle_deposit_moves.argtypes = [C.POINTER(OCfg), C.c_int32, C.c_int64, dp, dp, dp, dp, dp, dp,
                                           dp, dp, dp]
        L.oracle_rho.argtypes = [C.POINTER(OCfg), C.POINTER(OParts), dp]
        L.oracle_divE.argtypes = [C.POINTER(OCfg), dp, dp]
        L.oracle_energy.argtypes = [C.POINTER(OCfg), dp, C.POINTER(OParts), dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Grid:
    """Grid/decomposition description handed to every oracle call."""

    def __init__(self, dims, n, d, dt, q=-1.0, m=1.0, patch=(8, 8, 8), nreg=(1, 1, 1), filter=0):
        n = list(n) + [1] * (3 - len(n))
        d = list(d) + [1.0] * (3 - len(d))
        patch = list(patch) + [1] * (3 - len(patch))
        nreg = list(nreg) + [1] * (3 - len(nreg))
        if dims == 2:
            n[2], d[2], patch[2], nreg[2] = 1, 1.0, 1, 1
        self.dims, self.n, self.d, self.dt, self.q, self.m = dims, n, d, dt, q, m
        self.patch, self.nreg, self.filter = patch, nreg, filter
        self.c = OCfg(dims, (C.c_int32 * 3)(*n), (C.c_double * 3)(*d), dt, q, m,
                      (C.c_int32 * 3)(*patch), (C.c_int32 * 3)(*nreg), int(filter))

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def zeros_fields(self):
        return np.zeros((NCOMP,) + self.shape, dtype=np.float64)


class Particles:
    """float64 SoA particle set that the oracle updates in place."""

    KEYS = ("x", "y", "z", "ux", "uy", "uz", "w")

    def __init__(self, **arrs):
        n = len(arrs["x"])
        for k in self.KEYS:
            a = arrs.get(k)
            if a is None:
                a = np.zeros(n)
            setattr(self, k, np.ascontiguousarray(a, dtype=np.float64).copy())
        self.n = n

    def c(self):
        return OParts(self.n, *[_dp(getattr(self, k)) for k in self.KEYS])

    def copy(self):
        return Particles(**{k: getattr(self, k) for k in self.KEYS})


def S(s: float) -> float:
    return lib().oracle_S(float(s))


def interp(g: Grid, F: np.ndarray, x, y, z=0.0) -> np.ndarray:
    out = np.zeros(6)
    lib().oracle_interp(C.byref(g.c), _dp(F), float(x), float(y), float(z), _dp(out))
    return out


def boris(qm, dt, EB, u) -> np.ndarray:
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().oracle_boris(float(qm), float(dt), _dp(EB), _dp(u))
    return u


def gamma(u) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().oracle_gamma(_dp(u))


def deposit_one(g: Grid, J: np.ndarray, x0, x1, w, vz=0.0):
    x0 = np.array(list(x0) + [0.0] * (3 - len(x0)), dtype=np.float64)
    x1 = np.array(list(x1) + [0.0] * (3 - len(x1)), dtype=np.float64)
    lib().oracle_deposit_one(C.byref(g.c), _dp(J), _dp(x0), _dp(x1), float(w), float(vz))


def yee(g: Grid, F: np.ndarray):
    lib().oracle_yee(C.byref(g.c), _dp(F))


def filter_arrays(g: Grid, a: np.ndarray, passes: int) -> np.ndarray:
    """Binomial filter (``passes`` passes) of a stack of global arrays,
    shape (k, nz, ny, nx) or (nz, ny, nx); returns a filtered copy."""
    out = np.ascontiguousarray(a, dtype=np.float64).copy()
    k = 1 if out.ndim == 3 else out.shape[0]
    lib().oracle_filter(C.byref(g.c), _dp(out), int(k), int(passes))
    return out


def init_fields(g: Grid, F: np.ndarray):
    lib().oracle_init_fields(C.byref(g.c), _dp(F))


def wrap(x, L) -> float:
    return lib().oracle_wrap(float(x), float(L))


def cell(x, d, n) -> int:
    return lib().oracle_cell(float(x), float(d), int(n))


def bin_patches(g: Grid, P: Particles) -> np.ndarray:
    out = np.zeros(max(P.n, 1), dtype=np.int32)
    pc = P.c()
    lib().oracle_bin(C.byref(g.c), C.byref(pc), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out[:P.n]


def split(x, d, n):
    ci = C.c_int32()
    xi = C.c_float()
    lib().oracle_split(float(x), float(d), int(n), C.byref(ci), C.byref(xi))
    return ci.value, np.float32(xi.value)


def particles_sdsd(g: Grid, F: np.ndarray, P: Particles) -> float:
    pc = P.c()
    return lib().oracle_particles_sdsd(C.byref(g.c), _dp(F), C.byref(pc))


def push_only(g: Grid, F: np.ndarray, P: Particles):
    pc = P.c()
    lib().oracle_push_only(C.byref(g.c), _dp(F), C.byref(pc))


def step_sdsd(g: Grid, F: np.ndarray, P: Particles) -> float:
    pc = P.c()
    return lib().oracle_step_sdsd(C.byref(g.c), _dp(F), C.byref(pc))


_lib_omp = None


def step_sdmd_threads(g: Grid, F: np.ndarray, P: Particles, threads: int) -> int:
    """One SDMD step from the OpenMP timing build with `threads` threads over
    the patches (dynamic schedule).  Same arithmetic, same result bit for bit
    as step_sdmd; used only to time the CPU baseline."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB_OMP)
        L.oracle_step_sdmd.restype = C.c_int
        L.oracle_step_sdmd.argtypes = [C.POINTER(OCfg), C.POINTER(C.c_double), C.POINTER(OParts), C.c_int32]
        L.omp_set_num_threads.argtypes = [C.c_int]
        _lib_omp = L
    _lib_omp.omp_set_num_threads(int(threads))
    pc = P.c()
    rc = _lib_omp.oracle_step_sdmd(C.byref(g.c), _dp(F), C.byref(pc), 0)
    if rc != 0:
        raise ValueError("invalid decomposition")
    return rc


def step_sdmd(g: Grid, F: np.ndarray, P: Particles | None, fields_only: bool = False) -> int:
    if P is None:
        P = Particles(x=np.zeros(0))
        fields_only = True
    pc = P.c()
    rc = lib().oracle_step_sdmd(C.byref(g.c), _dp(F), C.byref(pc), int(fields_only))
    if rc != 0:
        raise ValueError("invalid decomposition")
    return rc


def deposit_moves(g: Grid, mode: int, x0, y0, z0, x1, y1, z1, w, vz=None) -> np.ndarray:
    n = len(x0)
    arrs = [np.ascontiguousarray(a if a is not None else np.zeros(n), dtype=np.float64)
            for a in (x0, y0, z0, x1, y1, z1, w)]
    vz_a = np.ascontiguousarray(vz if vz is not None else np.zeros(n), dtype=np.float64)
    J = np.zeros((3,) + g.shape)
    rc = lib().oracle_deposit_moves(C.byref(g.c), int(mode), n, *[_dp(a) for a in arrs], _dp(vz_a), _dp(J))
    if rc != 0:
        raise ValueError("invalid decomposition")
    return J


def rho(g: Grid, P: Particles) -> np.ndarray:
    out = np.zeros(g.shape)
    pc = P.c()
    lib().oracle_rho(C.byref(g.c), C.byref(pc), _dp(out))
    return out


def divE(g: Grid, F: np.ndarray) -> np.ndarray:
    out = np.zeros(g.shape)
    lib().oracle_divE(C.byref(g.c), _dp(F), _dp(out))
    return out


def energy(g: Grid, F: np.ndarray, P: Particles) -> np.ndarray:
    out = np.zeros(3)
    pc = P.c()
    lib().oracle_energy(C.byref(g.c), _dp(F), C.byref(pc), _dp(out))
    return out
