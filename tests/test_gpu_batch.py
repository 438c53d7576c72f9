"""Batched and served forms: every run gives the same result alone and inside
a batch or a continuously batched mix (within round-off; the LDS current
accumulation order is not fixed)."""
import sys

import numpy as np
import pytest

from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL
from tests.helpers import family_errors

pytestmark = pytest.mark.gpu
MASK = B.F_E | B.F_BH | B.F_J


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mix():
    return [
        WL.thermal_2d(n=(64, 64), ppc=4, vth=0.05, patch=(8, 8), precision="fp64", seed=11),
        WL.thermal_2d(n=(128, 64), ppc=9, vth=0.02, patch=(16, 16), precision="fp32s", seed=12),
        WL.thermal_2d(n=(64, 32), ppc=3, vth=0.08, patch=(32, 32), precision="fp32s", seed=13),
        WL.thermal_2d(n=(96, 64), ppc=5, vth=0.01, patch=(8, 8), nreg=(3, 2), precision="fp32s", seed=14),
        WL.cylinder_3d(n=(32, 16, 16), ppc_bg=2, ppc_cyl=8, radius=4.0, precision="fp32s", seed=15),
    ]


def alone(wl, steps):
    with B.Context([wl]) as c:
        c.step(steps)
        return c.fields(0, MASK)


def close(a, b, prec):
    tol = 1e-12 if prec == "fp64" else 2e-6
    for s in (slice(0, 3), slice(3, 6), slice(6, 9)):
        if np.linalg.norm(b[s]) == 0:
            assert np.abs(a[s]).max() == 0
        else:
            assert max(family_errors(a[s], b[s])) < tol


def test_batch_equals_alone():
    say("case: batch of 5 mixed runs, 12 steps")
    wls = mix()
    ref = [alone(w, 12) for w in wls]
    with B.Context(wls) as c:
        c.step(12)
        for i, w in enumerate(wls):
            close(c.fields(i, MASK), ref[i], w.precision)
            assert c.run_steps(i) == 12


def test_continuous_batching_equals_alone():
    """Runs admitted at different times with different step budgets: each
    stops on its own last step and matches the same run stepped alone."""
    say("case: continuous batching")
    wls = mix()
    budgets = [20, 7, 13, 5, 9]
    ref = [alone(w, s) for w, s in zip(wls, budgets)]
    with B.Context([wls[0]], max_runs=3, max_steps=[budgets[0]]) as c:
        c.step(3)
        r1 = c.admit(wls[1], max_steps=budgets[1])
        c.step(4)
        r2 = c.admit(wls[2], max_steps=budgets[2])
        c.step(5)
        # run 1 has taken its 7 steps; it stays frozen while the others go on
        close(c.fields(r1, MASK), ref[1], wls[1].precision)
        c.retire(r1)
        r3 = c.admit(wls[3], max_steps=budgets[3])
        with pytest.raises(B.PicError) as e:
            c.admit(wls[4], max_steps=budgets[4])
        assert e.value.code == B.PIC_E_CAPACITY
        c.step(20)
        close(c.fields(0, MASK), ref[0], wls[0].precision)
        close(c.fields(r2, MASK), ref[2], wls[2].precision)
        close(c.fields(r3, MASK), ref[3], wls[3].precision)
        assert c.run_steps(0) == 20 and c.run_steps(r2) == 13 and c.run_steps(r3) == 5
        c.retire(r2)
        r4 = c.admit(wls[4], max_steps=budgets[4])
        c.step(11)
        close(c.fields(r4, MASK), ref[4], wls[4].precision)


def test_autotuned_patch_is_valid_and_correct():
    """The autotuner's choices (patch edge, segment capacity, field tile
    width) are among its candidates, and the run gives what the same
    explicit configuration gives."""
    say("case: autotune")
    import dataclasses
    wl = WL.thermal_2d(n=(128, 64), ppc=8, vth=0.05, patch=(0, 0), precision="fp32s", seed=21)
    with B.Context([wl]) as c:
        c.step(5)
        d = c.diag(0)
        F = c.fields(0, MASK)
    say(f"autotuned: patch {d['patch']} seg_cap {d['seg_cap']} field tile {d['kernel_path'][2]}")
    assert d["patch"][0] in (8, 16, 32) and d["patch"][0] == d["patch"][1]
    assert d["seg_cap"] in (1024, 2048, 4096)
    assert d["kernel_path"][2] in (8, 16, 32, 64)
    wl2 = dataclasses.replace(wl, patch=tuple(d["patch"][:2]), seg_cap=d["seg_cap"], tile_x=d["kernel_path"][2])
    close(F, alone(wl2, 5), "fp32s")


def test_budget_admission_and_serving_loop():
    """The request loop on the GPU: small Poisson stream, budget for a few runs."""
    say("case: serving loop")
    from paper_1912_04064_amd import serving as S
    reqs = WL.request_stream(40.0, window_s=0.5, seed=3, steps_range=(20, 60), nx_pow=(6, 7), ny_pow=(6, 6))
    reqs = reqs[:12]
    mk = lambda r: WL.request_workload(r, patch=(16, 16))
    need = max(B.mem_bytes(mk(r)) for r in reqs)
    budget = 3 * need
    be = S.GpuBackend(max_runs=4, hbm_budget=budget)
    srv = S.Server(be, hbm_budget=budget, max_runs=4, steps_per_call=10)
    recs = srv.serve(reqs, mk)
    be.close()
    summ = S.summarize(recs)
    say("serving summary", summ, "library peak device bytes", be.peak_bytes, "budget", budget)
    assert len(recs) == len(reqs) and srv.max_active <= 4
    # the library's own count of every device byte it held (runs, set-up
    # staging, read-out scratch, patch autotuning, context tables) never
    # went above the budget, and at least two runs shared the GPU at once
    assert 0 < be.peak_bytes <= budget
    assert srv.max_active >= 2
    for r, q in zip(recs, reqs):
        assert r.result["step"] == q.steps and r.result["n_particles"] == mk(q).n_particles


def test_batched_scan_sample_against_oracle():
    """Runs of the parameter scan stepped together as a batch (autotuned
    patch, segment capacity and field tile; one launch per phase for all of
    them): the smaller runs of the sample (64 x 64 and 128 x 128 cells, 4 to
    10 particles per cell) against the oracle after 1 and 10 steps, FP32
    split form (1e-5 and 1e-4 relative per family)."""
    say("case: batched scan sample vs oracle")
    import oracle as O
    from tests.helpers import oracle_state
    wls = WL.scan_batch(n_runs=20, steps=10)
    picks = [2, 7, 16, 18]
    assert all(wls[i].n_particles <= 163840 for i in picks)
    res = {1: {}, 10: {}}
    with B.Context(wls) as c:
        for k in (1, 9):
            c.step(k)
            s = c.diag(0)["step"]
            for i in picks:
                res[s][i] = c.fields(i, B.F_E | B.F_B | B.F_J)
    for i in picks:
        g, F, P = oracle_state(wls[i])
        done = 0
        for s, tol in ((1, 1e-5), (10, 1e-4)):
            while done < s:
                O.step_sdsd(g, F, P)
                done += 1
            ref = np.concatenate([F[0:3], F[6:9], F[9:12]])
            errs = [max(family_errors(res[s][i][sl], ref[sl])) for sl in (slice(0, 3), slice(3, 6), slice(6, 9))]
            say(f"scan run {i} {wls[i].n} step {s}: E/Bm/J {errs}")
            assert max(errs) < tol, (i, s, errs)
