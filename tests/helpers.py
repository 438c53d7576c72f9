"""Shared test helpers: workload -> oracle inputs, error metrics."""
import numpy as np

import oracle as O


def oracle_state(wl):
    """Oracle Grid, fields (initial half step applied) and particles of a workload."""
    g = O.Grid(wl.dims, wl.n, wl.d, wl.dt, q=wl.q, m=wl.m, patch=wl.patch, nreg=wl.nreg, filter=wl.filter)
    F = g.zeros_fields()
    if wl.E0 is not None:
        F[0:3] = wl.E0
        F[3:6] = wl.B0
        if wl.field_kind == 1:
            F[6:9] = wl.Bm0 if wl.Bm0 is not None else wl.B0
    if wl.E0 is None or wl.field_kind == 0:
        O.init_fields(g, F)
    p = wl.parts
    P = O.Particles(x=p["x"], y=p["y"], z=p["z"], ux=p["ux"], uy=p["uy"], uz=p["uz"], w=p["w"])
    return g, F, P


def family_errors(gpu, ref, floor=1e-3):
    """Relative L2 error per component; a component whose reference norm is
    below `floor` of its family's norm is measured against the family norm.
    gpu/ref: arrays (3, ...) of one family (E, B or J)."""
    fam = np.linalg.norm(ref)
    out = []
    for c in range(ref.shape[0]):
        nb = np.linalg.norm(ref[c])
        den = nb if nb >= floor * fam else fam
        out.append(np.linalg.norm(gpu[c] - ref[c]) / den if den > 0 else np.linalg.norm(gpu[c]))
    return out


def oracle_fields_view(F):
    """oracle 12-component array -> dict of families as pic_fields returns them"""
    return {"E": F[0:3], "Bm": F[6:9], "BH": F[3:6], "J": F[9:12]}
