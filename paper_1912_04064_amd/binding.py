"""Thin ctypes binding of the HIP library ``libsdmd.so`` (C ABI in
``include/sdmd_pic.h``).

Argument marshalling only: every step of the PIC path runs in the library's
gfx950 kernels.  PyTorch supplies device memory (its caching allocator, passed
as the library's alloc/free callbacks) and the stream (the current torch
stream).  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdmd.so")

PIC_OK = 0
PIC_E_INVAL = -1
PIC_E_CONFIG = -2
PIC_E_NOMEM = -3
PIC_E_DEVICE = -4
PIC_E_NUMERIC = -5
PIC_E_CAPACITY = -6
PIC_E_STATE = -7
PIC_E_OVERFLOW = -8
PIC_FP64 = 0
PIC_FP32_SPLIT = 1
PIC_RT_NO_GRAPH = 1

F_EX, F_EY, F_EZ = 1 << 0, 1 << 1, 1 << 2
F_BX, F_BY, F_BZ = 1 << 3, 1 << 4, 1 << 5
F_BHX, F_BHY, F_BHZ = 1 << 6, 1 << 7, 1 << 8
F_JX, F_JY, F_JZ = 1 << 9, 1 << 10, 1 << 11
F_RHO = 1 << 12
SOLVERS = {"yee": 0, "psatd": 1}
F_E = F_EX | F_EY | F_EZ
F_B = F_BX | F_BY | F_BZ
F_BH = F_BHX | F_BHY | F_BHZ
F_J = F_JX | F_JY | F_JZ
F_ALL = F_E | F_B | F_BH | F_J

EXPORTED = ["pic_init", "pic_step", "pic_fields", "pic_diag", "pic_diag_noalloc", "pic_particles", "pic_mem_bytes",
            "pic_admit", "pic_retire", "pic_run_steps", "pic_time_phases", "pic_free", "pic_strerror",
            "pic_last_error"]

_dp = C.POINTER(C.c_double)


class PicParticlesIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", _dp), ("y", _dp), ("z", _dp), ("ux", _dp), ("uy", _dp), ("uz", _dp),
                ("w", _dp), ("id", C.POINTER(C.c_uint32))]


class PicFieldsIn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("E", _dp), ("B", _dp), ("Bm", _dp)]


class PicConfig(C.Structure):
    _fields_ = [("dims", C.c_int32), ("n_cells", C.c_int32 * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("patch", C.c_int32 * 3), ("n_regions", C.c_int32 * 3), ("shape_order", C.c_int32),
                ("precision", C.c_int32), ("bc", C.c_int32 * 3), ("track_ids", C.c_int32),
                ("filter_passes", C.c_int32), ("field_solver", C.c_int32), ("q", C.c_double),
                ("m", C.c_double), ("max_steps", C.c_int64), ("seg_cap", C.c_int32), ("field_tile_x", C.c_int32),
                ("particles", C.POINTER(PicParticlesIn)),
                ("fields", C.POINTER(PicFieldsIn))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class PicRuntime(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("stream", C.c_void_p), ("user", C.c_void_p),
                ("hbm_budget", C.c_size_t), ("max_runs", C.c_int32), ("flags", C.c_int32),
                ("deterministic", C.c_int32), ("reserved", C.c_int32)]


class PicDiag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("n_particles", C.c_int64), ("patch_min", C.c_int64),
                ("patch_max", C.c_int64), ("patch_mean", C.c_double), ("U_E", C.c_double), ("U_B", C.c_double),
                ("K", C.c_double), ("t_ms", C.c_double * 4), ("n_relayout", C.c_int64), ("n_spill", C.c_int64),
                ("err_flags", C.c_int32), ("patch", C.c_int32 * 3), ("gauss_residual", C.c_double),
                ("kernel_path", C.c_int32 * 4), ("device_bytes", C.c_int64), ("device_bytes_peak", C.c_int64),
                ("det_quantum", C.c_double * 2), ("seg_cap", C.c_int32), ("reserved", C.c_int32),
                ("t_push_kernel_ms", C.c_double)]


class PicParticlesOut(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n", C.c_int64), ("x", _dp), ("y", _dp), ("z", _dp), ("ux", _dp),
                ("uy", _dp), ("uz", _dp), ("w", _dp), ("id", C.POINTER(C.c_uint32)),
                ("patch", C.POINTER(C.c_int32))]


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Open the library (no GPU call).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    # One HIP runtime per process: torch carries its own libamdhip64, so load
    # torch first and let this library bind to that copy by soname.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    L.pic_init.argtypes = [C.POINTER(PicConfig), C.c_int32, C.POINTER(PicRuntime), C.POINTER(C.c_void_p)]
    L.pic_step.argtypes = [C.c_void_p, C.c_int32]
    L.pic_fields.argtypes = [C.c_void_p, C.c_int32, C.c_uint32, _dp, C.c_size_t, C.c_int32]
    L.pic_diag.argtypes = [C.c_void_p, C.c_int32, C.POINTER(PicDiag)]
    L.pic_diag_noalloc.argtypes = [C.c_void_p, C.c_int32, C.POINTER(PicDiag)]
    L.pic_particles.argtypes = [C.c_void_p, C.c_int32, C.POINTER(PicParticlesOut)]
    L.pic_mem_bytes.argtypes = [C.POINTER(PicConfig), C.POINTER(C.c_size_t)]
    L.pic_admit.argtypes = [C.c_void_p, C.POINTER(PicConfig), C.POINTER(C.c_int32)]
    L.pic_retire.argtypes = [C.c_void_p, C.c_int32]
    L.pic_run_steps.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
    L.pic_time_phases.argtypes = [C.c_void_p, C.c_int32]
    L.pic_free.argtypes = [C.c_void_p]
    L.pic_free.restype = None
    L.pic_strerror.argtypes = [C.c_int]
    L.pic_strerror.restype = C.c_char_p
    L.pic_last_error.argtypes = [C.c_void_p]
    L.pic_last_error.restype = C.c_char_p
    for name in ("pic_init", "pic_step", "pic_fields", "pic_diag", "pic_diag_noalloc", "pic_particles",
                 "pic_mem_bytes", "pic_admit", "pic_retire", "pic_run_steps", "pic_time_phases"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ptr(a: Optional[np.ndarray], ctype=C.c_double):
    if a is None:
        return C.POINTER(ctype)()
    return a.ctypes.data_as(C.POINTER(ctype))


class _CfgHolder:
    """A PicConfig plus the numpy arrays its pointers refer to."""

    def __init__(self, wl, track_ids=False, patch=None, max_steps=0):
        self.keep = []
        p = wl.parts
        n = len(p["x"])

        def arr(k, dt=np.float64):
            a = np.ascontiguousarray(p[k] if k in p else np.zeros(n), dtype=dt)
            self.keep.append(a)
            return a

        self.pin = PicParticlesIn(n, _ptr(arr("x")), _ptr(arr("y")), _ptr(arr("z")), _ptr(arr("ux")),
                                  _ptr(arr("uy")), _ptr(arr("uz")), _ptr(arr("w")),
                                  _ptr(arr("id", np.uint32), C.c_uint32))
        self.fin = None
        if wl.E0 is not None:
            E = np.ascontiguousarray(wl.E0, dtype=np.float64)
            B = np.ascontiguousarray(wl.B0, dtype=np.float64)
            Bm = np.ascontiguousarray(wl.Bm0, dtype=np.float64) if wl.Bm0 is not None else None
            self.keep += [E, B, Bm]
            self.fin = PicFieldsIn(int(wl.field_kind), 0, _ptr(E), _ptr(B), _ptr(Bm))
        dims = wl.dims
        nc = list(wl.n) + [1] * (3 - len(wl.n))
        d = list(wl.d) + [1.0] * (3 - len(wl.d))
        pt = list(patch if patch is not None else wl.patch) + [0] * 3
        nr = list(wl.nreg) + [1] * 3
        if dims == 2:
            nc[2], pt[2], nr[2] = 1, 0, 1
        prec = PIC_FP64 if wl.precision == "fp64" else PIC_FP32_SPLIT
        self.cfg = PicConfig(dims, (C.c_int32 * 3)(*nc[:3]), (C.c_double * 3)(*d[:3]), wl.dt,
                             (C.c_int32 * 3)(*pt[:3]), (C.c_int32 * 3)(*nr[:3]), 2, prec, (C.c_int32 * 3)(0, 0, 0),
                             1 if track_ids else 0, int(wl.filter), SOLVERS[wl.solver], wl.q, wl.m,
                             int(max_steps), int(wl.seg_cap), int(wl.tile_x),
                             C.pointer(self.pin),
                             C.pointer(self.fin) if self.fin is not None else C.POINTER(PicFieldsIn)())


def _check(L, ctx, rc, what):
    if rc != PIC_OK:
        msg = (L.pic_last_error(ctx) or b"").decode()
        raise PicError(rc, f"{what}: {L.pic_strerror(rc).decode()}: {msg}")


def mem_bytes(wl, patch=None) -> int:
    L = load()
    h = _CfgHolder(wl, patch=patch)
    out = C.c_size_t()
    _check(L, None, L.pic_mem_bytes(C.byref(h.cfg), C.byref(out)), "pic_mem_bytes")
    return int(out.value)


class Context:
    """A live set of runs on cuda:0.  Workloads come from ``workloads``."""

    def __init__(self, workloads: Sequence, track_ids=False, use_torch=True, graph=True, max_runs=0,
                 hbm_budget=0, patch=None, max_steps=None, deterministic=False):
        self.L = load()
        self._torch = None
        self._cbs = None
        stream_ptr = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU: the SDMD library needs a HIP device")
            self._torch = torch
            self.stream = torch.cuda.current_stream()
            stream_ptr = self.stream.cuda_stream
            dev = torch.cuda.current_device()

            def _alloc(nbytes, stream, user):
                try:
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream))
                except Exception:
                    return None

            def _free(ptr, nbytes, stream, user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
        self.track_ids = track_ids
        ms = max_steps if max_steps is not None else [0] * len(workloads)
        if isinstance(ms, int):
            ms = [ms] * len(workloads)
        self._holders = [_CfgHolder(w, track_ids, patch, m) for w, m in zip(workloads, ms)]
        cfgs = (PicConfig * max(1, len(workloads)))(*[h.cfg for h in self._holders])
        rt = PicRuntime()
        if self._cbs:
            rt.alloc, rt.free = self._cbs
        rt.stream = stream_ptr
        rt.hbm_budget = hbm_budget
        rt.max_runs = max_runs
        rt.flags = 0 if graph else PIC_RT_NO_GRAPH
        rt.deterministic = 1 if deterministic else 0
        self._rt = rt
        ctx = C.c_void_p()
        rc = self.L.pic_init(cfgs, len(workloads), C.byref(rt), C.byref(ctx))
        _check(self.L, None, rc, "pic_init")
        self.ctx = ctx
        self.workloads = {i: w for i, w in enumerate(workloads)}
        self._holders = None

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.L.pic_free(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        import sys as _sys
        if _sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------
    def step(self, n: int = 1):
        _check(self.L, self.ctx, self.L.pic_step(self.ctx, int(n)), "pic_step")

    def time_phases(self, n: int = 1):
        """Take n steps timed phase by phase; diag()["t_ms"] then holds the
        per-step average of each phase over them."""
        _check(self.L, self.ctx, self.L.pic_time_phases(self.ctx, int(n)), "pic_time_phases")

    def fields(self, run: int = 0, mask: int = F_ALL, check=True) -> np.ndarray:
        w = self.workloads[run]
        shape = w.shape
        ncomp = bin(mask).count("1")
        out = np.zeros((ncomp,) + shape, dtype=np.float64)
        rc = self.L.pic_fields(self.ctx, run, mask, _ptr(out), out.size, 0)
        if check:
            _check(self.L, self.ctx, rc, "pic_fields")
        return out

    def diag(self, run: int = 0, check=True, noalloc=False) -> dict:
        """pic_diag, or with noalloc=True pic_diag_noalloc (no device
        allocation: its scratch is the library's static per-GPU array)."""
        d = PicDiag()
        fn = self.L.pic_diag_noalloc if noalloc else self.L.pic_diag
        rc = fn(self.ctx, run, C.byref(d))
        if check:
            _check(self.L, self.ctx, rc, "pic_diag_noalloc" if noalloc else "pic_diag")
        arrays = ("t_ms", "patch", "kernel_path", "det_quantum")
        out = {k: getattr(d, k) for k, _ in PicDiag._fields_ if k not in arrays}
        for k in arrays:
            out[k] = list(getattr(d, k))
        out["rc"] = rc
        return out

    def particles(self, run: int = 0, check=True) -> dict:
        n = self.diag(run, check=False)["n_particles"]
        arrs = {k: np.zeros(n) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
        arrs["id"] = np.zeros(n, np.uint32)
        arrs["patch"] = np.zeros(n, np.int32)
        o = PicParticlesOut(n, 0, *[_ptr(arrs[k]) for k in ("x", "y", "z", "ux", "uy", "uz", "w")],
                            _ptr(arrs["id"], C.c_uint32), _ptr(arrs["patch"], C.c_int32))
        rc = self.L.pic_particles(self.ctx, run, C.byref(o))
        if check:
            _check(self.L, self.ctx, rc, "pic_particles")
        arrs = {k: v[: o.n] for k, v in arrs.items()}
        return arrs

    def admit(self, wl, max_steps=0, patch=None) -> int:
        h = _CfgHolder(wl, self.track_ids, patch, max_steps)
        rid = C.c_int32()
        _check(self.L, self.ctx, self.L.pic_admit(self.ctx, C.byref(h.cfg), C.byref(rid)), "pic_admit")
        self.workloads[rid.value] = wl
        return rid.value

    def retire(self, run: int):
        _check(self.L, self.ctx, self.L.pic_retire(self.ctx, run), "pic_retire")
        self.workloads.pop(run, None)

    def run_steps(self, run: int) -> int:
        s = C.c_int64()
        _check(self.L, self.ctx, self.L.pic_run_steps(self.ctx, run, C.byref(s)), "pic_run_steps")
        return s.value

    def checkpoint(self, run: int = 0):
        """The run's state as a resumable input: a copy of its workload whose
        initial fields are E^n, B^{n+1/2}, Bm^n (kind 1) and whose particles
        are the exported ones (with ids when the context tracks them).  A
        context made from it continues the run."""
        import dataclasses
        w = self.workloads[run]
        F = self.fields(run, F_E | F_BH | F_B)
        p = self.particles(run)
        parts = {k: p[k] for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
        if self.track_ids:
            parts["id"] = p["id"]
        return dataclasses.replace(w, parts=parts, E0=F[0:3].copy(), B0=F[6:9].copy(), Bm0=F[3:6].copy(),
                                   field_kind=1)

    def sync(self):
        if self._torch is not None:
            self._torch.cuda.synchronize()


def sort_by_id(parts: dict) -> dict:
    order = np.argsort(parts["id"], kind="stable")
    return {k: v[order] for k, v in parts.items()}
