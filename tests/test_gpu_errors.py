"""Error paths of the C ABI on the GPU, each forced from the host with valid
kernels: non-finite particle values (PIC_E_NUMERIC), positions outside the
domain (PIC_E_CONFIG), an HBM budget below a run's need (PIC_E_NOMEM).  The
kernels guard every such value (a non-finite move is not applied, an
out-of-range position is binned at 0), so no launch touches memory outside
its buffers; the error surfaces at the next synchronising call."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_1912_04064_amd import binding as B
from paper_1912_04064_amd import workloads as WL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small(prec, **kw):
    return WL.thermal_2d(n=(32, 32), ppc=2, vth=0.05, patch=(8, 8), precision=prec, **kw)


def _with_parts(wl, **changes):
    parts = {k: np.array(v, copy=True) for k, v in wl.parts.items()}
    for k, (i, v) in changes.items():
        parts[k][i] = v
    return dataclasses.replace(wl, parts=parts)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_nonfinite_momentum_at_init_is_numeric(prec):
    say(f"case: NaN momentum at init {prec}")
    wl = _with_parts(_small(prec), uy=(17, np.nan))
    with pytest.raises(B.PicError) as e:
        B.Context([wl])
    assert e.value.code == B.PIC_E_NUMERIC and "non-finite" in str(e.value)


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_nonfinite_field_reaches_particles_as_numeric(prec):
    """A NaN in the initial E: the particles interpolating it get a
    non-finite momentum in the first step, which pic_diag reports."""
    say(f"case: NaN field {prec}")
    wl = _small(prec)
    E = np.zeros((3, 1, 32, 32))
    E[1, 0, 10, 12] = np.nan
    wl = dataclasses.replace(wl, E0=E, B0=np.zeros_like(E), field_kind=0)
    with B.Context([wl]) as ctx:
        ctx.step(1)
        d = ctx.diag(0, check=False)
        assert d["rc"] == B.PIC_E_NUMERIC and d["err_flags"] & 1
        with pytest.raises(B.PicError) as e:
            ctx.fields(0, B.F_E)
        assert e.value.code == B.PIC_E_NUMERIC


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("bad", ["at_L", "negative", "far"])
def test_position_outside_domain_is_config(prec, bad):
    say(f"case: position outside [0, L) {bad} {prec}")
    wl = _small(prec)
    L = wl.n[0] * wl.d[0]
    x = {"at_L": L, "negative": -1e-9, "far": 10 * L}[bad]
    wl = _with_parts(wl, x=(5, x))
    with pytest.raises(B.PicError) as e:
        B.Context([wl])
    assert e.value.code == B.PIC_E_CONFIG and "outside" in str(e.value)


def test_budget_below_need_is_nomem_and_context_survives():
    say("case: HBM budget")
    a, b = _small("fp32s", seed=5), WL.thermal_2d(n=(128, 128), ppc=8, patch=(16, 16), precision="fp32s")
    need_a, need_b = B.mem_bytes(a), B.mem_bytes(b)
    with pytest.raises(B.PicError) as e:
        B.Context([a], hbm_budget=need_a // 2)
    assert e.value.code == B.PIC_E_NOMEM
    budget = need_a + need_b // 2 + (1 << 20)
    with B.Context([a], hbm_budget=budget, max_runs=2) as ctx:
        with pytest.raises(B.PicError) as e:
            ctx.admit(b)
        assert e.value.code == B.PIC_E_NOMEM
        ctx.step(3)
        d = ctx.diag(0)
        say(f"device bytes {d['device_bytes']} peak {d['device_bytes_peak']} budget {budget} need {need_a}")
        assert d["step"] == 3 and d["device_bytes_peak"] <= budget
        assert d["device_bytes"] <= need_a + (1 << 20)
        # the refused admission left nothing behind: a run that fits is admitted
        r = ctx.admit(_small("fp64", seed=6))
        ctx.step(2)
        assert ctx.diag(r)["step"] == 2 and ctx.diag(r)["device_bytes_peak"] <= budget
