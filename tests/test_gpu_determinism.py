"""Deterministic mode (pic_runtime.deterministic) and checkpoint / resume.

SDMD re-decomposes one domain (paper section 2.2): the step's result does not
depend on how particles are split into patches and segments, on the region
layout, or on other runs sharing the GPU.  With FP64 atomics the current's
summation order is set by timing, so two executions agree only to
round-off; the deterministic mode sums fixed-point contributions in 64-bit
integers, and then every field and every particle is the same bit for bit:
  * the same input twice (with leavers, parked particles and re-layouts);
  * a run alone and inside a batch of unrelated runs;
  * one region, several regions and one region per patch (SDSD);
  * 50 steps, export (pic_fields + pic_particles), a new context from that
    state, 50 more steps -- against 100 steps straight.
Against the oracle the deterministic current is within half a quantum per
contribution of the FP64 sum.  Without the mode the resume agrees to
round-off.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle as O
from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL
from tests.helpers import family_errors, oracle_state

pytestmark = pytest.mark.gpu

MASK = B.F_E | B.F_B | B.F_BH | B.F_J | B.F_RHO
PKEYS = ("x", "y", "z", "ux", "uy", "uz", "w", "id")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state(ctx, run, steps=None):
    if steps:
        ctx.step(steps)
    return ctx.fields(run, MASK), B.sort_by_id(ctx.particles(run)), ctx.diag(run)


def run_alone(wl, steps, det=True):
    with B.Context([wl], track_ids=True, deterministic=det) as ctx:
        return state(ctx, 0, steps)


def assert_bitwise(a, b, what):
    Fa, pa, _ = a
    Fb, pb, _ = b
    names = ["Ex", "Ey", "Ez", "Bmx", "Bmy", "Bmz", "BHx", "BHy", "BHz", "Jx", "Jy", "Jz", "rho"]
    for c, nm in enumerate(names):
        if not np.array_equal(Fa[c], Fb[c]):
            d = np.abs(Fa[c] - Fb[c]).max()
            raise AssertionError(f"{what}: {nm} differs (max |diff| {d:.3e})")
    for k in PKEYS:
        assert np.array_equal(pa[k], pb[k]), f"{what}: particle {k} differs"


def stream_2d(prec):
    """Dense plasma streaming at ~0.9 c: leavers from every patch each step."""
    rng = np.random.default_rng(41)
    N = 32 * 32 * 24
    parts = {"x": rng.uniform(0, 32, N), "y": rng.uniform(0, 32, N), "z": np.zeros(N),
             "ux": 2.0 + rng.normal(0, 0.3, N), "uy": 0.7 + rng.normal(0, 0.3, N), "uz": rng.normal(0, 0.1, N),
             "w": rng.uniform(0.01, 0.03, N), "id": np.arange(N, dtype=np.uint32)}
    return WL.Workload(name="stream", dims=2, n=(32, 32), d=(1.0, 1.0), dt=0.6, patch=(8, 8), nreg=(2, 2),
                       steps=0, precision=prec, parts=parts, q=-1e-2)


def converge_2d(prec):
    """Particles streaming towards the centre: patches overflow their
    segments, particles are parked and the store is re-laid out."""
    rng = np.random.default_rng(42)
    N = 32 * 32 * 4
    x = rng.uniform(0, 32, N)
    y = rng.uniform(0, 32, N)
    parts = {"x": x, "y": y, "z": np.zeros(N), "ux": -0.6 * np.sign(x - 16) * (np.abs(x - 16) > 2),
             "uy": -0.6 * np.sign(y - 16) * (np.abs(y - 16) > 2), "uz": np.zeros(N), "w": np.full(N, 0.25),
             "id": np.arange(N, dtype=np.uint32)}
    return WL.Workload(name="conv", dims=2, n=(32, 32), d=(1.0, 1.0), dt=0.6, patch=(8, 8), nreg=(1, 1), steps=0,
                       precision=prec, parts=parts, q=-1e-6)


def cyl_3d(prec, nreg=(1, 1, 1)):
    wl = WL.cylinder_3d(n=(32, 16, 16), radius=4.0, ppc_bg=2, ppc_cyl=16, vth=0.1, patch=(4, 4, 4),
                        precision=prec, seed=43)
    return dataclasses.replace(wl, nreg=nreg)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("kind", ["stream2d", "converge2d", "cyl3d"])
def test_same_input_twice_is_bitwise_identical(kind, prec):
    say(f"case: deterministic twice {kind} {prec}")
    wl = {"stream2d": stream_2d, "converge2d": converge_2d, "cyl3d": cyl_3d}[kind](prec)
    steps = 24 if kind == "converge2d" else 20
    a = run_alone(wl, steps)
    b = run_alone(wl, steps)
    assert a[2]["kernel_path"][3] == 1 and a[2]["det_quantum"][0] > 0
    say(f"relayouts {a[2]['n_relayout']} spill {a[2]['n_spill']} quantum {a[2]['det_quantum']}")
    if kind == "converge2d":
        assert a[2]["n_relayout"] >= 3       # overflowing patches were re-laid out
    assert_bitwise(a, b, "second execution")


def _mix():
    return [
        WL.thermal_2d(n=(64, 64), ppc=4, vth=0.05, patch=(8, 8), precision="fp64", seed=11),
        WL.thermal_2d(n=(128, 64), ppc=9, vth=0.02, patch=(16, 16), precision="fp32s", seed=12),
        WL.thermal_2d(n=(64, 32), ppc=3, vth=0.08, patch=(32, 32), precision="fp32s", seed=13),
        WL.thermal_2d(n=(96, 64), ppc=5, vth=0.01, patch=(8, 8), nreg=(3, 2), precision="fp32s", seed=14),
        cyl_3d("fp32s"),
        stream_2d("fp64"),
    ]


def test_batch_equals_alone_bitwise():
    say("case: deterministic batch of 6 == each alone")
    wls = _mix()
    alone = [run_alone(w, 15) for w in wls]
    with B.Context(wls, track_ids=True, deterministic=True) as ctx:
        ctx.step(15)
        for i, w in enumerate(wls):
            assert_bitwise(state(ctx, i), alone[i], f"run {i} ({w.name}) in the batch")


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("dims", [2, 3])
def test_region_layouts_bitwise(dims, prec):
    """One region, several regions, and one region per patch (SDSD) give the
    same state bit for bit: the decompositions only re-group the sums."""
    say(f"case: deterministic region layouts {dims}D {prec}")
    if dims == 2:
        base = WL.thermal_2d(n=(64, 32), ppc=6, vth=0.1, patch=(8, 8), precision=prec, seed=45)
        layouts = [(1, 1), (4, 2), (8, 4)]
    else:
        base = cyl_3d(prec)
        layouts = [(1, 1, 1), (2, 2, 1), (8, 4, 4)]
    ref = run_alone(dataclasses.replace(base, nreg=layouts[0]), 12)
    for nr in layouts[1:]:
        assert_bitwise(run_alone(dataclasses.replace(base, nreg=nr), 12), ref, f"regions {nr}")


def _lwfa_small(prec):
    # cell sizes are powers of two, so the FP64 positions of the export hold
    # the split form's (cell, offset) exactly
    return WL.lwfa_2d(n=(256, 64), patch=(16, 16), nreg=(2, 1), vac_end=96, ramp=64, x0=17.0, waist=10.0,
                      duration=8.0, n0=0.02, precision=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_step_chunking_and_graphs_are_bitwise_identical(prec):
    """pic_step replays graphs of 2 and 8 steps and of a whole re-layout
    period (16 steps and the check) where the step count allows, and
    enqueues single steps otherwise.  Any split of the same 50 steps, with
    and without graphs, must give the same state: the re-layout checks fall
    on the same steps and every kernel sees the same parity."""
    say(f"case: step chunking and graphs, converging flow {prec}")
    wl = converge_2d(prec)
    ref = None
    for graph, chunks in ((False, [50]), (True, [50]), (True, [1, 7, 8, 16, 1, 17]), (True, [3, 2, 9, 36]),
                          (True, [16, 16, 16, 2])):
        assert sum(chunks) == 50
        with B.Context([wl], track_ids=True, deterministic=True, graph=graph) as ctx:
            for k in chunks:
                ctx.step(k)
            got = state(ctx, 0)
        say(f"graph={graph} chunks {chunks}: relayouts {got[2]['n_relayout']} spill {got[2]['n_spill']}")
        if ref is None:
            ref = got
            assert ref[2]["n_relayout"] >= 3   # the checks moved particles
        else:
            assert_bitwise(got, ref, f"graph={graph} chunks {chunks}")


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_checkpoint_resume_is_bitwise_in_deterministic_mode(prec):
    say(f"case: 50 + export/re-init + 50 == 100, deterministic {prec}")
    wl = _lwfa_small(prec)
    ref = run_alone(wl, 100)
    with B.Context([wl], track_ids=True, deterministic=True) as ctx:
        ctx.step(50)
        ck = ctx.checkpoint(0)
    with B.Context([ck], track_ids=True, deterministic=True) as ctx:
        got = state(ctx, 0, 50)
    say(f"quantum {ref[2]['det_quantum']} relayouts {ref[2]['n_relayout']}")
    assert_bitwise(got, ref, "resumed run")
    assert got[2]["n_particles"] == ref[2]["n_particles"] == wl.n_particles
    assert got[2]["K"] == pytest.approx(ref[2]["K"], rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_spectral_deterministic_twice_and_resume_bitwise(prec):
    """The spectral field phase uses no atomics, so with the deterministic
    current a spectral run is bitwise reproducible, and 50 steps, export,
    re-init and 50 more equal 100 steps bitwise (the state of the spectral
    solver is E^n and B^n, with Bm^n = B^n)."""
    say(f"case: spectral deterministic twice and resume {prec}")
    wl = dataclasses.replace(_lwfa_small(prec), nreg=(1, 1), solver="psatd", name="lwfa256x64_psatd")
    ref = run_alone(wl, 100)
    assert_bitwise(run_alone(wl, 100), ref, "second execution")
    with B.Context([wl], track_ids=True, deterministic=True) as ctx:
        ctx.step(50)
        ck = ctx.checkpoint(0)
    with B.Context([ck], track_ids=True, deterministic=True) as ctx:
        got = state(ctx, 0, 50)
    say(f"quantum {ref[2]['det_quantum']} relayouts {ref[2]['n_relayout']}")
    assert_bitwise(got, ref, "resumed run")


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_checkpoint_resume_matches_to_round_off(prec):
    say(f"case: 50 + export/re-init + 50 vs 100, plain mode {prec}")
    wl = _lwfa_small(prec)
    ref = run_alone(wl, 100, det=False)
    with B.Context([wl], track_ids=True) as ctx:
        ctx.step(50)
        ck = ctx.checkpoint(0)
    got = run_alone(ck, 50, det=False)
    tol = 1e-10 if prec == "fp64" else 1e-4
    for fam, sl in (("E", slice(0, 3)), ("Bm", slice(3, 6)), ("BH", slice(6, 9)), ("J", slice(9, 12))):
        e = max(family_errors(got[0][sl], ref[0][sl]))
        say(f"{prec} resume {fam}: {e:.2e}")
        assert e < tol, fam
    assert np.array_equal(got[1]["id"], ref[1]["id"])
    assert np.abs(got[1]["ux"] - ref[1]["ux"]).max() < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_deterministic_mode_matches_oracle(prec):
    """Deterministic current against the oracle: every contribution is
    rounded to a multiple of the quantum q_J, so a node holding k
    contributions may move by k q_J / 2 on top of the usual bar."""
    say(f"case: deterministic vs oracle {prec}")
    wl = WL.thermal_2d(n=(64, 64), ppc=4, vth=0.05, patch=(8, 8), nreg=(2, 2), precision=prec, seed=47)
    g, F, P = oracle_state(wl)
    with B.Context([wl], track_ids=True, deterministic=True) as ctx:
        res = {}
        for k in (1, 19):
            ctx.step(k)
            Fa = ctx.fields(0, B.F_E | B.F_B | B.F_BH | B.F_J)
            res[ctx.diag(0)["step"]] = (Fa, ctx.diag(0))
    done = 0
    for target, tol in ((1, 1e-12 if prec == "fp64" else 1e-5), (20, 1e-9 if prec == "fp64" else 1e-3)):
        while done < target:
            O.step_sdsd(g, F, P)
            done += 1
        Fa, d = res[target]
        qj = d["det_quantum"][0]
        Jo = F[9:12]
        # a node's current gathers at most 25 cells x ppc particle contributions
        slack = 25 * 4 * qj / 2
        dJ = np.abs(Fa[9:12] - Jo).max()
        say(f"{prec} step {target}: quantum {qj:.3e}, max |dJ| {dJ:.3e}, max |J| {np.abs(Jo).max():.3e}")
        assert dJ <= tol * np.abs(Jo).max() + slack
        for fam, a, b in (("E", Fa[0:3], F[0:3]), ("BH", Fa[6:9], F[3:6]), ("Bm", Fa[3:6], F[6:9])):
            assert max(family_errors(a, b)) < tol + 1e3 * slack / max(np.abs(b).max(), 1e-300), fam
