"""pic_diag_noalloc against pic_diag, through the C ABI.

The no-allocation variant runs the same kernels with their scratch (charge
density, Gauss residual, partial sums) in the library's static per-GPU
array instead of freshly allocated device memory.  Its output must equal
pic_diag's: counts and shapes exactly, the energies to round-off (1e-14
relative: the same kernels over the same state), the Gauss-law residual to
1e-10 (a round-off-level figure from a charge density that the kernels
deposit with atomics in no fixed order).  Two calls in a row, the second on
a smaller run, show that what the first leaves in the shared array does not
leak into the second.
"""
import sys

import pytest

from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL

pytestmark = pytest.mark.gpu

INT_KEYS = ("step", "n_particles", "patch_min", "patch_max", "n_relayout", "n_spill", "err_flags")
FLOAT_KEYS = ("t", "patch_mean", "U_E", "U_B", "K")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    for k in INT_KEYS:
        assert a[k] == b[k], k
    assert a["patch"] == b["patch"] and a["kernel_path"] == b["kernel_path"]
    for k in FLOAT_KEYS:
        assert a[k] == pytest.approx(b[k], rel=1e-14, abs=0.0), k
    assert abs(a["gauss_residual"] - b["gauss_residual"]) <= 1e-10, (a["gauss_residual"], b["gauss_residual"])


def test_noalloc_diag_matches_diag_on_two_calls_second_smaller():
    say("case: pic_diag_noalloc vs pic_diag, 256x128 fp32s then 32x32 fp64")
    big = WL.thermal_2d(n=(256, 128), ppc=8, vth=0.05, patch=(16, 16), nreg=(2, 1), precision="fp32s", seed=31)
    small = WL.thermal_2d(n=(32, 32), ppc=4, vth=0.05, patch=(8, 8), precision="fp64", seed=32)
    with B.Context([big, small]) as ctx:
        ctx.step(6)
        a_big = ctx.diag(0, noalloc=True)
        a_small = ctx.diag(1, noalloc=True)      # right after, a smaller run
        b_big = ctx.diag(0)
        b_small = ctx.diag(1)
        say(f"big: noalloc K {a_big['K']:.17g} diag K {b_big['K']:.17g}; "
            f"small: noalloc gauss {a_small['gauss_residual']:.3e} diag gauss {b_small['gauss_residual']:.3e}")
        _same(a_big, b_big)
        _same(a_small, b_small)
        assert a_big["n_particles"] == big.n_particles and a_small["n_particles"] == small.n_particles
        # and once more on the big run after the small one
        _same(ctx.diag(0, noalloc=True), b_big)


def test_noalloc_diag_allocates_no_device_memory():
    import torch
    say("case: pic_diag_noalloc allocates nothing")
    wl = WL.thermal_2d(n=(128, 64), ppc=4, vth=0.05, patch=(16, 16), precision="fp32s", seed=33)
    with B.Context([wl]) as ctx:
        ctx.step(3)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        m0 = torch.cuda.memory_allocated()
        d1 = ctx.diag(0, noalloc=True)
        d2 = ctx.diag(0, noalloc=True)
        assert torch.cuda.max_memory_allocated() == m0 and torch.cuda.memory_allocated() == m0
        # the library's own count agrees: nothing beyond what the runs hold
        assert d1["device_bytes"] == d2["device_bytes"] and d1["device_bytes_peak"] == d2["device_bytes_peak"]
        # pic_diag, by contrast, takes its scratch from the allocator
        torch.cuda.reset_peak_memory_stats()
        d3 = ctx.diag(0)
        assert torch.cuda.max_memory_allocated() > m0
        assert d3["device_bytes"] > d1["device_bytes"]
        _same(d1, d3)


def test_noalloc_diag_rejects_runs_beyond_the_static_scratch():
    say("case: pic_diag_noalloc on a 2048x2048 grid (beyond 64 MiB of scratch)")
    import numpy as np
    parts = {k: np.zeros(0) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
    wl = WL.Workload(name="huge", dims=2, n=(2048, 2048), d=(0.1, 0.1), dt=0.05, patch=(32, 32), nreg=(1, 1),
                     steps=0, precision="fp32s", parts=parts)
    with B.Context([wl]) as ctx:
        with pytest.raises(B.PicError) as e:
            ctx.diag(0, noalloc=True)
        assert e.value.code == B.PIC_E_NOMEM and "static scratch" in str(e.value)
        assert ctx.diag(0)["n_particles"] == 0
        # a small run in the same process still works afterwards
    with B.Context([WL.thermal_2d(n=(32, 32), ppc=2, patch=(8, 8), seed=34)]) as ctx:
        ctx.step(1)
        _same(ctx.diag(0, noalloc=True), ctx.diag(0))
