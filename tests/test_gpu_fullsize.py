"""Parity at the benchmark's full size, in the benchmark's launch form.

The LWFA input at 2048 x 256 cells with 3,932,160 FP32 split particles,
16 x 16 patches and 4 regions, stepped with the captured hipGraph exactly
as ``bench.py`` times it, is stopped after 700 steps (the laser is in the
plasma, the wake is forming), and one more step is checked piece by piece
against the oracle, each piece from the GPU's own state at step n:

  * the particle push of every particle (interpolation from the GPU's E^n,
    Bm^n, Boris, move) -- oracle ``push_only``;
  * the current J^{n+1/2} of step n+1 against the oracle's deposition of the
    GPU's moves x^n -> x^{n+1} (summed globally in FP64);
  * E^{n+1}, B^{n+3/2}, Bm^{n+1} against the oracle's Yee step applied to the
    GPU's E^n, B^{n+1/2} and J^{n+1/2};
  * every particle's patch against the oracle's binning of its position,
    and the particle count.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL
from tests.helpers import family_errors

pytestmark = pytest.mark.gpu

MASK = B.F_E | B.F_B | B.F_BH | B.F_J


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wrapped(d, L):
    """Displacement folded into (-L/2, L/2]."""
    return d - L * np.round(d / L)


def test_lwfa_full_size_one_step_piecewise():
    say("case: LWFA 2048x256 full size, step 700 -> 701")
    wl = WL.lwfa_2d()
    n0 = 700
    with B.Context([wl], track_ids=True, graph=True) as ctx:
        ctx.step(n0)
        Fa = ctx.fields(0, MASK)
        Pa = B.sort_by_id(ctx.particles(0))
        ctx.step(1)
        Fb = ctx.fields(0, MASK)
        Pb = B.sort_by_id(ctx.particles(0))
        diag = ctx.diag(0)
    N = wl.n_particles
    assert diag["n_particles"] == N and len(Pb["x"]) == N
    assert np.array_equal(Pa["id"], Pb["id"])
    g = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch, nreg=wl.nreg)
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])

    # 1. particle push through the GPU's fields at step n
    F = g.zeros_fields()
    F[0:3], F[6:9], F[3:6] = Fa[0:3], Fa[3:6], Fa[6:9]
    P = O.Particles(x=Pa["x"], y=Pa["y"], ux=Pa["ux"], uy=Pa["uy"], uz=Pa["uz"], w=Pa["w"])
    O.push_only(g, F, P)
    # FP32 push against the FP64 oracle: errors scale with the momenta that
    # enter the step (a kick that nearly cancels u^{n-1/2} leaves a small
    # u^{n+1/2} with the absolute error of the larger terms)
    un = np.sqrt(P.ux ** 2 + P.uy ** 2 + P.uz ** 2)
    uo = np.sqrt(Pa["ux"] ** 2 + Pa["uy"] ** 2 + Pa["uz"] ** 2)
    du = np.max(np.abs(np.stack([Pb["ux"] - P.ux, Pb["uy"] - P.uy, Pb["uz"] - P.uz])), axis=0)
    rel_u = du / (un + uo + 1e-30)
    dx = np.abs(wrapped(Pb["x"] - P.x, L[0])) / wl.d[0]
    dy = np.abs(wrapped(Pb["y"] - P.y, L[1])) / wl.d[1]
    moving = un + uo > 0
    q = np.percentile(rel_u[moving], [50, 99, 99.99])
    say(f"push: {moving.sum()} moving particles, |du| / (|u_old| + |u_new|): median {q[0]:.2e}, "
        f"p99 {q[1]:.2e}, p99.99 {q[2]:.2e}, max {rel_u[moving].max():.2e}; "
        f"max position error {max(dx.max(), dy.max()):.3e} cells, max |u| {un.max():.3f}")
    assert moving.sum() > 0.05 * N
    assert rel_u[moving].max() < 1e-5
    if (~moving).any():
        assert np.abs(du[~moving]).max() == 0.0
    assert max(dx.max(), dy.max()) < 1e-5

    # 2. the current of step n+1 from the GPU's own moves
    mx = wrapped(Pb["x"] - Pa["x"], L[0])
    my = wrapped(Pb["y"] - Pa["y"], L[1])
    gam = np.sqrt(1 + Pb["ux"] ** 2 + Pb["uy"] ** 2 + Pb["uz"] ** 2)
    J = O.deposit_moves(g, 0, Pa["x"], Pa["y"], None, Pa["x"] + mx, Pa["y"] + my, None, Pa["w"],
                        vz=Pb["uz"] / gam)
    ej = family_errors(Fb[9:12], J)
    say(f"current of step n+1: family errors {ej}")
    assert max(ej) < 1e-5

    # 3. the field update from the GPU's state (FP64 both sides)
    G = g.zeros_fields()
    G[0:3], G[3:6], G[6:9], G[9:12] = Fa[0:3], Fa[6:9], Fa[3:6], Fb[9:12]
    O.yee(g, G)
    errs = [max(family_errors(Fb[0:3], G[0:3])), max(family_errors(Fb[6:9], G[3:6])),
            max(family_errors(Fb[3:6], G[6:9]))]
    say(f"field update E, B, Bm: {errs}")
    assert max(errs) < 1e-13

    # 4. binning of every particle
    Pn = O.Particles(x=Pb["x"], y=Pb["y"], w=Pb["w"])
    po = O.bin_patches(g, Pn)
    bad = np.nonzero(po != Pb["patch"])[0]
    if len(bad):
        # a position reconstructed from (cell, FP32 offset) can round onto a
        # cell face; such a particle is within round-off of its patch face
        fx = Pb["x"][bad] / (wl.patch[0] * wl.d[0])
        fy = Pb["y"][bad] / (wl.patch[1] * wl.d[1])
        near = np.minimum(np.abs(fx - np.round(fx)), np.abs(fy - np.round(fy)))
        assert near.max() < 1e-9
    say(f"binning: {len(bad)} of {N} particles on a patch face within round-off")
    assert len(bad) <= 1e-5 * N


def test_cylinder_3d_full_size_one_step():
    """The 3D cylinder at full size (512 x 128 x 128 cells, 116,998,144
    particles, 8^3 patches): after 60 steps, one step is checked -- the push
    of a sample of particles (ids divisible by 97) against the oracle, the
    discrete continuity of the GPU's own rho and J over every node, the field
    update against the oracle's Yee step on the GPU's state, and the binning
    of the sample."""
    say("case: cylinder 512x128x128 full size, step 60 -> 61")
    wl = WL.cylinder_3d()
    n0 = 60
    with B.Context([wl], track_ids=True, graph=True) as ctx:
        ctx.step(n0)
        Fa = ctx.fields(0, MASK | B.F_RHO)
        Pa = ctx.particles(0)
        ctx.step(1)
        Fb = ctx.fields(0, MASK | B.F_RHO)
        Pb = ctx.particles(0)
        diag = ctx.diag(0)
    N = wl.n_particles
    assert diag["n_particles"] == N and len(Pb["x"]) == N

    def sample(P):
        m = P["id"] % 97 == 0
        o = np.argsort(P["id"][m], kind="stable")
        return {k: v[m][o] for k, v in P.items()}

    Sa, Sb = sample(Pa), sample(Pb)
    del Pa, Pb
    assert np.array_equal(Sa["id"], Sb["id"]) and len(Sa["id"]) > N // 100
    g = O.Grid(3, wl.n, wl.d, wl.dt, patch=wl.patch)
    L = np.array([wl.n[a] * wl.d[a] for a in range(3)])

    # push of the sample through the GPU's fields at step n
    F = g.zeros_fields()
    F[0:3], F[6:9], F[3:6] = Fa[0:3], Fa[3:6], Fa[6:9]
    P = O.Particles(x=Sa["x"], y=Sa["y"], z=Sa["z"], ux=Sa["ux"], uy=Sa["uy"], uz=Sa["uz"], w=Sa["w"])
    O.push_only(g, F, P)
    un = np.sqrt(P.ux ** 2 + P.uy ** 2 + P.uz ** 2)
    uo = np.sqrt(Sa["ux"] ** 2 + Sa["uy"] ** 2 + Sa["uz"] ** 2)
    du = np.max(np.abs(np.stack([Sb["ux"] - P.ux, Sb["uy"] - P.uy, Sb["uz"] - P.uz])), axis=0)
    rel_u = du / (un + uo + 1e-30)
    dpos = max(np.abs(wrapped(Sb[k] - getattr(P, k), L[a])).max() / wl.d[a] for a, k in enumerate("xyz"))
    say(f"push sample {len(un)}: max |du| / (|u_old| + |u_new|) {rel_u.max():.2e}, position {dpos:.2e} cells")
    assert rel_u.max() < 1e-5
    assert dpos < 1e-5

    # continuity of the GPU's own charge and current over every node
    r0, r1 = Fa[12], Fb[12]
    J = Fb[9:12]
    dx, dy, dz = wl.d
    divJ = ((J[0] - np.roll(J[0], 1, axis=2)) / dx + (J[1] - np.roll(J[1], 1, axis=1)) / dy
            + (J[2] - np.roll(J[2], 1, axis=0)) / dz)
    res = np.abs((r1 - r0) / wl.dt + divJ).max() / (np.abs(r0).max() / wl.dt)
    say(f"continuity residual / (max rho / dt): {res:.2e}")
    assert res < 2e-6

    # field update from the GPU's state
    G = g.zeros_fields()
    G[0:3], G[3:6], G[6:9], G[9:12] = Fa[0:3], Fa[6:9], Fa[3:6], Fb[9:12]
    O.yee(g, G)
    errs = [max(family_errors(Fb[0:3], G[0:3])), max(family_errors(Fb[6:9], G[3:6])),
            max(family_errors(Fb[3:6], G[6:9]))]
    say(f"field update E, B, Bm: {errs}")
    assert max(errs) < 1e-13

    # binning of the sample
    po = O.bin_patches(g, O.Particles(x=Sb["x"], y=Sb["y"], z=Sb["z"], w=Sb["w"]))
    bad = int((po != Sb["patch"]).sum())
    say(f"binning: {bad} of {len(po)} sampled particles differ")
    assert bad <= 1e-5 * len(po)
