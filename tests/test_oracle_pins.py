"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Nothing here compares the oracle with itself: every expected value comes from
the mathematics of the method (B-spline identities, the discrete dispersion
relation of the Yee scheme, the exact gyration of the Boris rotation, the
discrete continuity equation that the Esirkepov scheme is built to satisfy)
or from an independent brute-force computation.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1912_04064_amd import workloads as WL


# --------------------------------------------------------------------------
# shape function
# --------------------------------------------------------------------------
def test_shape_values_match_golden_table():
    """Quadratic B-spline values at the tabulated points (tests/golden)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "quadratic_bspline.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 8
    for s, num, den in rows:
        assert O.S(float(s)) == pytest.approx(float(num) / float(den), abs=1e-15)


def test_shape_partition_of_unity_and_first_moment():
    rng = np.random.default_rng(1)
    for X in rng.uniform(-5, 5, 200):
        nodes = np.arange(math.floor(X) - 3, math.floor(X) + 4)
        w = np.array([O.S(X - k) for k in nodes])
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (w * nodes).sum() == pytest.approx(X, abs=1e-13)
        # second moment of the quadratic B-spline: X^2 + 1/4
        assert (w * nodes ** 2).sum() == pytest.approx(X * X + 0.25, abs=1e-12)
        assert (w > 0).sum() <= 3


# --------------------------------------------------------------------------
# interpolation
# --------------------------------------------------------------------------
STAG = {0: (1, 0, 0), 1: (0, 1, 0), 2: (0, 0, 1), 6: (0, 1, 1), 7: (1, 0, 1), 8: (1, 1, 0)}


@pytest.mark.parametrize("dims", [2, 3])
def test_interp_reproduces_constant_and_linear_fields(dims):
    n = (16, 12, 10) if dims == 3 else (16, 12)
    d = (0.3, 0.5, 0.7)[:dims]
    g = O.Grid(dims, n, d, 0.1)
    F = g.zeros_fields()
    nz, ny, nx = g.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    slopes = {0: (0.7, 0, 0), 1: (0, -0.3, 0), 2: (0, 0, 0.2) if dims == 3 else (0.1, 0.0, 0),
              6: (0.05, 0, 0), 7: (0, 0.4, 0), 8: (0, 0, -0.6) if dims == 3 else (0, 0.25, 0)}
    const = {0: 1.5, 1: -2.0, 2: 0.25, 6: 3.0, 7: -0.5, 8: 0.75}
    for comp, (sx, sy, sz) in STAG.items():
        xs = (ii + 0.5 * sx) * d[0]
        ys = (jj + 0.5 * sy) * d[1]
        zs = (kk + 0.5 * sz) * (d[2] if dims == 3 else 1.0)
        a, b, c = slopes[comp]
        F[comp] = const[comp] + a * xs + b * ys + (c * zs if dims == 3 else 0.0)
    rng = np.random.default_rng(2)
    Lx, Ly = n[0] * d[0], n[1] * d[1]
    Lz = n[2] * d[2] if dims == 3 else 1.0
    for _ in range(50):
        # keep the 3x3(x3) support away from the periodic seam of the linear ramp
        x = rng.uniform(2.5 * d[0], Lx - 2.5 * d[0])
        y = rng.uniform(2.5 * d[1], Ly - 2.5 * d[1])
        z = rng.uniform(2.5 * d[2], Lz - 2.5 * d[2]) if dims == 3 else 0.0
        out = O.interp(g, F, x, y, z)
        for slot, comp in enumerate([0, 1, 2, 6, 7, 8]):
            a, b, c = slopes[comp]
            exp = const[comp] + a * x + b * y + (c * z if dims == 3 else 0.0)
            assert out[slot] == pytest.approx(exp, abs=1e-12), (comp, x, y, z)


def test_interp_staggering_is_half_cell():
    """A field that is 1 on a single dual x node and 0 elsewhere is seen with
    weight S(X - i - 1/2): catches a primal/dual mix-up."""
    g = O.Grid(2, (16, 16), (1.0, 1.0), 0.1)
    F = g.zeros_fields()
    F[0, 0, 5, 7] = 1.0  # Ex at (7.5, 5)
    x, y = 7.9, 5.2
    out = O.interp(g, F, x, y)
    assert out[0] == pytest.approx(O.S(x - 7.5) * O.S(y - 5.0), abs=1e-15)
    F[0, 0, 5, 7] = 0.0
    F[8, 0, 5, 7] = 1.0  # Bmz at (7.5, 5.5)
    out = O.interp(g, F, x, y)
    assert out[5] == pytest.approx(O.S(x - 7.5) * O.S(y - 5.5), abs=1e-15)


# --------------------------------------------------------------------------
# Boris push
# --------------------------------------------------------------------------
def test_boris_pure_electric_kick_is_exact():
    for qm in (-1.0, 1.0, -2.5):
        u0 = np.array([0.1, -0.2, 0.3])
        E = np.array([0.3, -0.1, 0.05])
        dt = 0.07
        u = O.boris(qm, dt, np.r_[E, 0, 0, 0], u0)
        np.testing.assert_allclose(u, u0 + qm * E * dt, rtol=0, atol=1e-16)


def test_boris_gyration_angle_radius_and_sense():
    qm, dt, Bz = -1.0, 0.2, 1.3
    u = np.array([0.4, 0.0, 0.1])
    g = math.sqrt(1 + u @ u)
    theta = 2.0 * math.atan(abs(qm) * Bz * dt / (2.0 * g))
    EB = np.array([0, 0, 0, 0, 0, Bz], float)
    phase0 = math.atan2(u[1], u[0])
    uu = u.copy()
    for nstep in range(1, 301):
        uu = O.boris(qm, dt, EB, uu)
        assert math.sqrt(uu @ uu) == pytest.approx(math.sqrt(u @ u), rel=1e-14)
        assert uu[2] == u[2]
    # electron (q < 0) in B along +z turns counter-clockwise
    one = O.boris(qm, dt, EB, u)
    assert math.atan2(one[1], one[0]) == pytest.approx(theta, abs=1e-14)
    total = math.atan2(uu[1], uu[0]) - phase0
    expect = (300 * theta + math.pi) % (2 * math.pi) - math.pi
    assert total == pytest.approx(expect, abs=1e-11)
    # orbit radius of the position sequence x += dt u / gamma
    v = math.hypot(u[0], u[1]) / g
    R = (dt * v / 2.0) / math.sin(theta / 2.0)
    x = np.zeros(2)
    pts = []
    uu = u.copy()
    for _ in range(200):
        uu = O.boris(qm, dt, EB, uu)
        x = x + dt * uu[:2] / math.sqrt(1 + uu @ uu)
        pts.append(x.copy())
    pts = np.array(pts)
    # circumradius of three consecutive points
    a, b, c = pts[10], pts[11], pts[12]
    ab, bc, ca = np.linalg.norm(a - b), np.linalg.norm(b - c), np.linalg.norm(c - a)
    area = abs((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1])) / 2
    assert ab * bc * ca / (4 * area) == pytest.approx(R, rel=1e-10)


def test_boris_exb_drift():
    """Crossed fields, |E| << |B|: the guiding centre drifts at E x B / B^2."""
    qm, dt = -1.0, 0.05
    E = np.array([0.0, 0.01, 0.0])
    B = np.array([0.0, 0.0, 1.0])
    u = np.zeros(3)
    x = np.zeros(3)
    steps = int(round(40 * 2 * math.pi / dt))
    xs = []
    for _ in range(steps):
        u = O.boris(qm, dt, np.r_[E, B], u)
        x = x + dt * u / math.sqrt(1 + u @ u)
        xs.append(x.copy())
    vd = np.cross(E, B) / (B @ B)
    mean_v = (xs[-1] - xs[0]) / ((steps - 1) * dt)
    assert mean_v[0] == pytest.approx(vd[0], rel=2e-3)
    assert abs(mean_v[1]) < 1e-4


def _rodrigues(u, k, theta):
    """u rotated by theta about the unit vector k (right-hand rule)."""
    return u * math.cos(theta) + np.cross(k, u) * math.sin(theta) + k * (k @ u) * (1.0 - math.cos(theta))


@pytest.mark.parametrize("qm", [-1.0, 1.0, -3.0])
def test_boris_oblique_b_is_a_rotation_about_b(qm):
    """E = 0, B along a random oblique direction: one Boris step is the exact
    rotation of u about B by theta = 2 atan(|q/m| |B| dt / (2 gamma)), in the
    sense of d u/dt = (q/m) u x B / gamma (about +B for q < 0, about -B for
    q > 0).  Every component of t enters, so a wrong sign or index in any of
    the cross-product terms moves the result off the rotation."""
    rng = np.random.default_rng(11)
    dt = 0.17
    for _ in range(25):
        B = rng.normal(size=3) * rng.uniform(0.2, 3.0)
        Bn = math.sqrt(B @ B)
        b = B / Bn
        u = rng.normal(size=3) * rng.uniform(0.05, 2.0)
        g = math.sqrt(1 + u @ u)
        theta = 2.0 * math.atan(abs(qm) * Bn * dt / (2.0 * g))
        k = b if qm < 0 else -b
        expect = _rodrigues(u, k, theta)
        got = O.boris(qm, dt, np.r_[0.0, 0.0, 0.0, B], u)
        np.testing.assert_allclose(got, expect, rtol=0, atol=2e-15 * max(1.0, math.sqrt(u @ u)))
        # invariants: |u| and u . b
        assert math.sqrt(got @ got) == pytest.approx(math.sqrt(u @ u), rel=1e-14)
        assert got @ b == pytest.approx(u @ b, rel=1e-13, abs=1e-15)


def test_boris_parallel_momentum_grows_linearly_with_oblique_fields():
    """E with a component along an oblique B: the rotation leaves u . b
    unchanged and each half kick adds (q/m) (dt/2) E . b, so after n steps
    u . b = u0 . b + n (q/m) dt E . b (round-off only)."""
    qm, dt = -1.0, 0.09
    B = np.array([0.6, -0.8, 1.1])
    b = B / math.sqrt(B @ B)
    E = np.array([0.02, 0.05, -0.03])
    u0 = np.array([0.1, 0.2, -0.05])
    u = u0.copy()
    for n in range(1, 201):
        u = O.boris(qm, dt, np.r_[E, B], u)
        if n % 50 == 0:
            assert u @ b == pytest.approx(u0 @ b + n * qm * dt * (E @ b), rel=1e-12)


def test_boris_exb_drift_oblique():
    """E perpendicular to an oblique B, |E| << |B|: the guiding centre drifts
    at E x B / B^2 in all three components and not at all along B."""
    qm, dt = -1.0, 0.05
    B = np.array([0.3, -0.5, 0.8])
    B = B / math.sqrt(B @ B)
    e = np.cross(B, np.array([1.0, 0.0, 0.0]))
    E = 0.01 * e / math.sqrt(e @ e)
    u = np.zeros(3)
    x = np.zeros(3)
    steps = int(round(40 * 2 * math.pi / dt))
    for k in range(steps):
        u = O.boris(qm, dt, np.r_[E, B], u)
        x = x + dt * u / math.sqrt(1 + u @ u)
        if k == 0:
            x_first = x.copy()
    vd = np.cross(E, B) / (B @ B)
    mean_v = (x - x_first) / ((steps - 1) * dt)
    np.testing.assert_allclose(mean_v, vd, rtol=0, atol=2e-3 * math.sqrt(vd @ vd))
    assert abs(mean_v @ B) < 1e-6


# --------------------------------------------------------------------------
# Esirkepov deposition
# --------------------------------------------------------------------------
def _rho_single(g, x, w):
    P = O.Particles(x=[x[0]], y=[x[1]], z=[x[2] if len(x) > 2 else 0.0], w=[w])
    return O.rho(g, P)


def _divJ(g, J):
    dx, dy = g.d[0], g.d[1]
    out = (J[0] - np.roll(J[0], 1, axis=2)) / dx + (J[1] - np.roll(J[1], 1, axis=1)) / dy
    if g.dims == 3:
        out = out + (J[2] - np.roll(J[2], 1, axis=0)) / g.d[2]
    return out


@pytest.mark.parametrize("dims", [2, 3])
def test_esirkepov_discrete_continuity_and_sum_rules(dims):
    rng = np.random.default_rng(3 + dims)
    n = (12, 10, 8) if dims == 3 else (12, 10)
    d = (0.4, 0.25, 0.3)[:dims]
    dt = 0.11
    g = O.Grid(dims, n, d, dt, q=-1.0)
    L = np.array([n[a] * d[a] for a in range(dims)])
    for _ in range(40):
        x0 = rng.uniform(0, 1, dims) * L
        step = rng.uniform(-0.98, 0.98, dims) * np.array(d)
        x1 = x0 + step
        w, vz = rng.uniform(0.1, 2.0), rng.uniform(-0.5, 0.5)
        J = np.zeros((3,) + g.shape)
        O.deposit_one(g, J, list(x0), list(x1), w, vz)
        x1w = [O.wrap(x1[a], L[a]) for a in range(dims)]
        r0 = _rho_single(g, list(x0) + [0.0] * (3 - dims), w)
        r1 = _rho_single(g, list(x1w) + [0.0] * (3 - dims), w)
        resid = (r1 - r0) / dt + _divJ(g, J)
        assert np.abs(resid).max() <= 1e-13 * max(np.abs(r0).max(), 1e-300) / dt
        # sum rules: total current = q w displacement / dt (per cell volume unit)
        assert J[0].sum() == pytest.approx(-1.0 * w * step[0] / dt, rel=1e-12, abs=1e-14)
        assert J[1].sum() == pytest.approx(-1.0 * w * step[1] / dt, rel=1e-12, abs=1e-14)
        if dims == 2:
            assert J[2].sum() == pytest.approx(-1.0 * w * vz, rel=1e-12, abs=1e-14)
        else:
            assert J[2].sum() == pytest.approx(-1.0 * w * step[2] / dt, rel=1e-12, abs=1e-14)


def test_esirkepov_resting_particle_gives_zero_current():
    g = O.Grid(2, (8, 8), (1.0, 1.0), 0.5)
    J = np.zeros((3,) + g.shape)
    O.deposit_one(g, J, [3.3, 4.7], [3.3, 4.7], 1.0, 0.0)
    assert np.all(J == 0.0)


def test_esirkepov_motion_along_x_gives_no_y_current():
    g = O.Grid(2, (8, 8), (1.0, 1.0), 0.5)
    J = np.zeros((3,) + g.shape)
    O.deposit_one(g, J, [3.3, 4.7], [3.9, 4.7], 1.0, 0.0)
    assert np.all(J[1] == 0.0) and np.abs(J[0]).max() > 0


def test_esirkepov_brute_force_small_step_limit():
    """For a tiny move, Jx at (i+1/2, j) approaches q w v H(X - i - 1/2) S(Y - j)
    with H the linear hat: the derivative of the quadratic B-spline is a
    difference of hats, whose running sum telescopes to one hat."""
    g = O.Grid(2, (10, 10), (1.0, 1.0), 1.0)
    x0 = np.array([4.3, 5.6])
    eps = 1e-6
    J = np.zeros((3,) + g.shape)
    O.deposit_one(g, J, list(x0), [x0[0] + eps, x0[1]], 1.0, 0.0)
    for i in range(2, 8):
        for j in range(3, 9):
            hat = max(0.0, 1.0 - abs(x0[0] - i - 0.5))
            exp = -1.0 * eps * hat * O.S(x0[1] - j)
            assert J[0, 0, j, i] == pytest.approx(exp, abs=1e-11)


# --------------------------------------------------------------------------
# Yee solver
# --------------------------------------------------------------------------
def _eigenmode(g, m, e_dir, t0):
    """Discrete plane wave of the Yee scheme.  Returns (F with E at t0, B at
    t0 + dt/2, Bm at t0), omega)."""
    dims = g.dims
    L = [g.n[a] * g.d[a] for a in range(3)]
    k = np.array([2 * math.pi * m[a] / L[a] if a < dims else 0.0 for a in range(3)])
    K = np.array([math.sin(k[a] * g.d[a] / 2) / g.d[a] if a < dims else 0.0 for a in range(3)])
    Om = math.sqrt(K @ K)
    omega = 2.0 / g.dt * math.asin(Om * g.dt)
    e = np.array(e_dir, float)
    e = e - K * (K @ e) / (K @ K)          # transverse to the discrete K
    e = e / np.linalg.norm(e)
    b = np.cross(K, e) / Om
    F = g.zeros_fields()
    nz, ny, nx = g.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    stag = {0: (1, 0, 0), 1: (0, 1, 0), 2: (0, 0, 1), 3: (0, 1, 1), 4: (1, 0, 1), 5: (1, 1, 0)}

    def phase(comp, t):
        sx, sy, sz = stag[comp]
        ph = k[0] * (ii + 0.5 * sx) * g.d[0] + k[1] * (jj + 0.5 * sy) * g.d[1]
        if dims == 3:
            ph = ph + k[2] * (kk + 0.5 * sz) * g.d[2]
        return np.cos(ph - omega * t)

    for c in range(3):
        F[c] = e[c] * phase(c, t0)
        F[3 + c] = b[c] * phase(3 + c, t0 + 0.5 * g.dt)
        F[6 + c] = b[c] * phase(3 + c, t0)
    return F, omega, (e, b, phase)


@pytest.mark.parametrize("dims,m,e_dir", [
    (2, (3, 2, 0), (0, 0, 1)),          # TM: Ez, Bx, By
    (2, (1, 4, 0), (1, 0, 0)),          # TE: Ex, Ey, Bz
    (3, (2, 1, 3), (1, -1, 0.5)),
])
def test_yee_discrete_dispersion_eigenmode(dims, m, e_dir):
    n = (24, 20, 16) if dims == 3 else (32, 24)
    d = (0.3, 0.4, 0.5)[:dims]
    g = O.Grid(dims, n, d, WL.cfl_dt(d, 0.9))
    F, omega, (e, b, phase) = _eigenmode(g, m, e_dir, 0.0)
    steps = 300 if dims == 3 else 1000
    for _ in range(steps):
        O.yee(g, F)
    t = steps * g.dt
    for c in range(3):
        np.testing.assert_allclose(F[c], e[c] * phase(c, t), rtol=0, atol=2e-11)
        np.testing.assert_allclose(F[3 + c], b[c] * phase(3 + c, t + 0.5 * g.dt), rtol=0, atol=2e-11)


def test_yee_modified_energy_and_divergences_conserved():
    dims = 3
    g = O.Grid(dims, (10, 9, 8), (0.3, 0.4, 0.5), WL.cfl_dt((0.3, 0.4, 0.5), 0.9))
    rng = np.random.default_rng(7)
    F = g.zeros_fields()
    F[0:6] = rng.standard_normal((6,) + g.shape)

    def divB(F):
        return ((np.roll(F[3], -1, 2) - F[3]) / g.d[0] + (np.roll(F[4], -1, 1) - F[4]) / g.d[1]
                + (np.roll(F[5], -1, 0) - F[5]) / g.d[2])

    def menergy(F, Bprev):
        return 0.5 * ((F[0:3] ** 2).sum() + (Bprev * F[3:6]).sum())

    div0, dB0 = O.divE(g, F), divB(F)
    Bprev = F[3:6].copy()
    O.yee(g, F)
    U1 = menergy(F, Bprev)
    for _ in range(200):
        Bprev = F[3:6].copy()
        O.yee(g, F)
    U2 = menergy(F, Bprev)
    assert U2 == pytest.approx(U1, rel=1e-13)
    np.testing.assert_allclose(O.divE(g, F), div0, atol=1e-11)
    np.testing.assert_allclose(divB(F), dB0, atol=1e-11)


def test_yee_half_step_init_matches_faraday_half_step():
    g = O.Grid(2, (16, 16), (0.5, 0.5), 0.2)
    F, omega, (e, b, phase) = _eigenmode(g, (2, 1, 0), (0, 0, 1), 0.0)
    # put B at t=0 in the B slot and let init produce B(+dt/2), Bm = B(0)
    G = F.copy()
    for c in range(3):
        G[3 + c] = b[c] * phase(3 + c, 0.0)
    O.init_fields(g, G)
    for c in range(3):
        np.testing.assert_allclose(G[6 + c], b[c] * phase(3 + c, 0.0), atol=1e-15)
    # the centred half step is second order accurate: O((omega dt)^2) error
    err = np.abs(G[3:6] - F[3:6]).max()
    assert err < (omega * g.dt) ** 2


# --------------------------------------------------------------------------
# binning and wrap
# --------------------------------------------------------------------------
def test_wrap_and_cell_edges():
    L = 6.4
    assert O.wrap(L, L) == 0.0
    assert O.wrap(-1e-18, L) == 0.0          # x + L rounds to L -> 0
    assert O.wrap(L + 0.1, L) == pytest.approx(0.1)
    assert O.wrap(-0.1, L) == pytest.approx(L - 0.1)
    below = np.nextafter(L, 0)
    assert O.wrap(below, L) == below
    assert O.cell(below, 0.1, 64) == 63
    # x < L whose quotient rounds up to n: the cell is clamped to n - 1
    L68 = 68 * 0.1
    x68 = np.nextafter(L68, 0)
    assert x68 < L68 and math.floor(x68 / 0.1) == 68
    assert O.cell(x68, 0.1, 68) == 67
    assert O.cell(0.0, 0.1, 64) == 0
    assert O.cell(0.8, 0.1, 64) == math.floor(0.8 / 0.1)


def test_bin_brute_force_with_edge_inputs():
    g = O.Grid(2, (32, 16), (0.1, 0.2), 0.05, patch=(8, 4))
    rng = np.random.default_rng(11)
    Lx, Ly = 3.2, 3.2
    xs = list(rng.uniform(0, Lx, 300)) + [0.0, np.nextafter(Lx, 0), 0.8, 1.6, np.nextafter(0.8, 0), 2.4]
    ys = list(rng.uniform(0, Ly, 300)) + [np.nextafter(Ly, 0), 0.0, 0.8, np.nextafter(1.6, 2), 0.8, 3.0]
    P = O.Particles(x=xs, y=ys)
    pid = O.bin_patches(g, P)
    for x, y, p in zip(xs, ys, pid):
        ci = min(int(math.floor(x / 0.1)), 31)
        cj = min(int(math.floor(y / 0.2)), 15)
        assert p == ci // 8 + 4 * (cj // 4)
        assert 0 <= p < 16
    counts = np.bincount(pid, minlength=16)
    assert counts.sum() == len(xs)


def test_split_position_round_up_guard():
    dx = 0.1
    i, xi = O.split(0.35, dx, 64)
    assert i == 3 and 0.0 <= xi < 1.0 and abs(float(xi) - 0.5) < 1e-6
    # an offset that rounds to 1.0f moves to the next cell with xi = 0
    x = (5 + (1.0 - 1e-12)) * dx
    i, xi = O.split(x, dx, 64)
    assert (i, float(xi)) == (6, 0.0)
    i, xi = O.split(np.nextafter(6.4, 0), dx, 64)
    assert (i, float(xi)) == (0, 0.0)


# --------------------------------------------------------------------------
# SDMD == SDSD
# --------------------------------------------------------------------------
def _dyadic_moves(rng, n, L, dims, count):
    q = 2.0 ** -8
    x0 = [np.round(rng.uniform(0, L[a], count) / q) * q for a in range(dims)]
    dx = [np.round(rng.uniform(-0.9, 0.9, count) / q) * q for a in range(dims)]
    x0 = [np.mod(x0[a], L[a]) for a in range(dims)]
    x1 = [x0[a] + dx[a] for a in range(dims)]
    return x0, x1


@pytest.mark.parametrize("nreg", [(1, 1), (2, 1), (4, 1), (2, 2)])
def test_sdmd_deposit_equals_sdsd_bitwise_on_dyadic_inputs(nreg):
    rng = np.random.default_rng(21)
    g = O.Grid(2, (32, 32), (1.0, 1.0), 0.5, patch=(8, 8), nreg=nreg)
    x0, x1 = _dyadic_moves(rng, 32, (32.0, 32.0), 2, 600)
    w = np.full(600, 2.0 ** -4)
    Ja = O.deposit_moves(g, 0, x0[0], x0[1], None, x1[0], x1[1], None, w)
    Jb = O.deposit_moves(g, 1, x0[0], x0[1], None, x1[0], x1[1], None, w)
    assert np.array_equal(Ja, Jb)
    assert np.abs(Ja).max() > 0


def test_sdmd_deposit_equals_sdsd_bitwise_3d_planar_moves():
    rng = np.random.default_rng(22)
    g = O.Grid(3, (16, 16, 16), (1.0, 1.0, 1.0), 0.5, patch=(8, 8, 8), nreg=(2, 1, 1))
    x0, x1 = _dyadic_moves(rng, 16, (16.0, 16.0, 16.0), 3, 300)
    x1[2] = x0[2].copy()            # no z motion keeps every W product dyadic
    w = np.full(300, 2.0 ** -4)
    Ja = O.deposit_moves(g, 0, *x0, *x1, w)
    Jb = O.deposit_moves(g, 1, *x0, *x1, w)
    assert np.array_equal(Ja, Jb)


@pytest.mark.parametrize("dims,nreg", [(2, (4, 1)), (2, (2, 2)), (3, (2, 2, 1))])
def test_region_yee_equals_global_yee_bitwise(dims, nreg):
    n = (32, 16, 16)[:dims] if dims == 3 else (32, 16)
    d = (0.3, 0.4, 0.5)[:dims]
    g1 = O.Grid(dims, n, d, WL.cfl_dt(d), patch=(8,) * dims, nreg=(1,) * dims)
    g4 = O.Grid(dims, n, d, WL.cfl_dt(d), patch=(8,) * dims, nreg=nreg)
    rng = np.random.default_rng(5)
    F = g1.zeros_fields()
    F[:] = rng.standard_normal(F.shape)
    Fa, Fb, Fc = F.copy(), F.copy(), F.copy()
    for _ in range(5):
        O.step_sdmd(g1, Fa, None)
        O.step_sdmd(g4, Fb, None)
        O.yee(g1, Fc)
    assert np.array_equal(Fa, Fb)
    assert np.array_equal(Fa[:9], Fc[:9])


def _thermal_parts(wl):
    p = wl.parts
    return O.Particles(x=p["x"], y=p["y"], z=p["z"], ux=p["ux"], uy=p["uy"], uz=p["uz"], w=p["w"])


def test_sdmd_full_step_matches_sdsd():
    wl = WL.thermal_2d(n=(32, 32), ppc=4, vth=0.05, patch=(8, 8), nreg=(2, 2))
    gA = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch, nreg=(1, 1))
    gB = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch, nreg=wl.nreg)
    FA = gA.zeros_fields()
    rng = np.random.default_rng(9)
    FA[0:6] = 0.01 * rng.standard_normal((6,) + gA.shape)
    O.init_fields(gA, FA)
    FB = FA.copy()
    PA, PB = _thermal_parts(wl), _thermal_parts(wl)
    O.step_sdsd(gA, FA, PA)
    O.step_sdmd(gB, FB, PB)
    scale = np.abs(FA[9:12]).max()
    assert np.abs(FA - FB).max() <= 1e-13 * max(scale, np.abs(FA).max())
    np.testing.assert_array_equal(PA.x, PB.x)          # interpolation is identical
    np.testing.assert_array_equal(PA.ux, PB.ux)
    for _ in range(99):
        O.step_sdsd(gA, FA, PA)
        O.step_sdmd(gB, FB, PB)
    for fam in (slice(0, 3), slice(3, 6), slice(9, 12)):
        nrm = np.linalg.norm(FA[fam])
        assert np.linalg.norm(FA[fam] - FB[fam]) <= 1e-9 * nrm


# --------------------------------------------------------------------------
# full step: Gauss law and plasma oscillation
# --------------------------------------------------------------------------
def test_gauss_residual_constant_over_100_steps():
    wl = WL.thermal_2d(n=(24, 24), ppc=4, vth=0.05)
    g = O.Grid(2, wl.n, wl.d, wl.dt, patch=(8, 8))
    F = g.zeros_fields()
    P = _thermal_parts(wl)
    r0 = O.divE(g, F) - O.rho(g, P)
    scale = np.abs(O.rho(g, P)).max()
    for _ in range(100):
        O.step_sdsd(g, F, P)
    r1 = O.divE(g, F) - O.rho(g, P)
    assert np.abs(r1 - r0).max() <= 1e-12 * scale


def test_gauss_residual_constant_3d():
    wl = WL.cylinder_3d(n=(16, 16, 16), ppc_bg=2, ppc_cyl=8, radius=4.0, vth=0.05)
    g = O.Grid(3, wl.n, wl.d, wl.dt, patch=(8, 8, 8))
    F = g.zeros_fields()
    P = _thermal_parts(wl)
    r0 = O.divE(g, F) - O.rho(g, P)
    scale = np.abs(O.rho(g, P)).max()
    for _ in range(10):
        O.step_sdsd(g, F, P)
    r1 = O.divE(g, F) - O.rho(g, P)
    assert np.abs(r1 - r0).max() <= 1e-12 * scale


def test_cold_plasma_oscillation_frequency():
    """Uniform cold electrons (n = 1, so omega_p = 1) with a small sinusoidal
    velocity along x: E_x oscillates at the grid-corrected plasma frequency
    (2/dt) sin(omega dt / 2) = omega_p."""
    nx, ny = 32, 4
    d = (0.2, 0.2)
    dt = 0.1
    g = O.Grid(2, (nx, ny), d, dt)
    pa = 4
    sub = (np.arange(pa) + 0.5) / pa
    X, Y = np.meshgrid((np.arange(nx)[:, None] + sub[None, :]).ravel() * d[0],
                       (np.arange(ny)[:, None] + sub[None, :]).ravel() * d[1], indexing="ij")
    x, y = X.ravel(), Y.ravel()
    L = nx * d[0]
    k = 2 * math.pi / L
    ux = 1e-4 * np.sin(k * x)
    P = O.Particles(x=x, y=y, ux=ux, w=np.full(len(x), 1.0 / (pa * pa)))
    F = g.zeros_fields()
    trace = []
    for _ in range(400):
        O.step_sdsd(g, F, P)
        trace.append(F[0].mean(axis=(0, 1)) @ np.sin(k * (np.arange(nx) + 0.5) * d[0]))
    trace = np.array(trace)
    s = np.sign(trace)
    crossings = np.nonzero(s[1:] != s[:-1])[0]
    # linear interpolation of the zero crossings
    tc = [(c + trace[c] / (trace[c] - trace[c + 1])) * dt for c in crossings]
    period = 2 * (tc[-1] - tc[0]) / (len(tc) - 1)
    omega = 2 * math.pi / period
    omega_expected = 2.0 / dt * math.asin(dt / 2.0)
    assert omega == pytest.approx(omega_expected, rel=1e-2)


def test_esirkepov_2d_jz_is_time_average_of_shape_product():
    """In 2D3V, Jz / (q w vz) at a node is the average over the step of the
    product of the linearly time-interpolated shape factors,
    int_0^1 (S0x + t DSx)(S0y + t DSy) dt; 3-point Gauss-Legendre is exact."""
    g = O.Grid(2, (12, 12), (1.0, 1.0), 1.0)
    rng = np.random.default_rng(31)
    gl_t = 0.5 + 0.5 * np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    gl_w = np.array([5 / 18, 8 / 18, 5 / 18])
    for _ in range(20):
        x0 = rng.uniform(3, 9, 2)
        x1 = x0 + rng.uniform(-0.95, 0.95, 2)
        vz = 0.3
        J = np.zeros((3,) + g.shape)
        O.deposit_one(g, J, list(x0), list(x1), 1.0, vz)
        for i in range(1, 11):
            for j in range(1, 11):
                s0x, s1x = O.S(x0[0] - i), O.S(x1[0] - i)
                s0y, s1y = O.S(x0[1] - j), O.S(x1[1] - j)
                avg = sum(wt * (s0x + t * (s1x - s0x)) * (s0y + t * (s1y - s0y)) for t, wt in zip(gl_t, gl_w))
                assert J[2, 0, j, i] == pytest.approx(-1.0 * vz * avg, abs=1e-15)


def test_diagnostics_closed_forms():
    g = O.Grid(2, (8, 6), (0.5, 0.25), 0.1)
    F = g.zeros_fields()
    F[0] = 2.0
    F[8] = -3.0
    u = np.array([0.3, 0.4, 1.2])
    P = O.Particles(x=[1.1, 2.3], y=[0.2, 1.4], ux=[u[0], 0], uy=[u[1], 0], uz=[u[2], 0], w=[0.7, 0.2])
    ue, ub, k = O.energy(g, F, P)
    vol = 8 * 6 * 0.5 * 0.25
    assert ue == pytest.approx(0.5 * 4.0 * vol)
    assert ub == pytest.approx(0.5 * 9.0 * vol)
    assert k == pytest.approx(0.7 * (math.sqrt(1 + u @ u) - 1.0) * 0.5 * 0.25)
    r = O.rho(g, P)
    assert r.sum() == pytest.approx(-1.0 * (0.7 + 0.2), abs=1e-14)


# --------------------------------------------------------------------------
# binomial current filter
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [2, 3])
@pytest.mark.parametrize("passes", [1, 2, 3])
def test_binomial_filter_fourier_transfer_function(dims, passes):
    """The 1-2-1 kernel multiplies the periodic mode exp(i theta i) by
    (2 + 2 cos theta) / 4 = cos^2(theta / 2); a pass applies it along every
    axis, so a cosine mode comes back scaled by prod_a cos^2(pi m_a / n_a),
    raised to the number of passes."""
    n = (16, 12, 1) if dims == 2 else (8, 6, 10)
    g = O.Grid(dims, n[:dims], (0.1,) * dims, 0.01)
    rng = np.random.default_rng(40 + passes)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for _ in range(4):
        m = [int(rng.integers(0, n[a])) for a in range(3)]
        if dims == 2:
            m[2] = 0
        phi = rng.uniform(0, 2 * math.pi)
        a = np.cos(2 * math.pi * (m[0] * i / n[0] + m[1] * j / n[1] + m[2] * k / n[2]) + phi)
        factor = 1.0
        for ax in range(dims):
            factor *= math.cos(math.pi * m[ax] / n[ax]) ** 2
        out = O.filter_arrays(g, a, passes)
        np.testing.assert_allclose(out, factor ** passes * a, rtol=0, atol=1e-14)


def test_binomial_filter_special_cases():
    """Constants pass unchanged, the checkerboard (Nyquist) mode along an axis
    is removed by one pass, and the sum over the grid is preserved."""
    g = O.Grid(2, (10, 8), (0.1, 0.1), 0.01)
    const = np.full((1, 8, 10), 3.25)
    assert np.array_equal(O.filter_arrays(g, const, 2), const)
    nyq = np.tile((-1.0) ** np.arange(10), (1, 8, 1))
    assert np.array_equal(O.filter_arrays(g, nyq, 1), np.zeros_like(nyq))
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 1, 8, 10))
    f = O.filter_arrays(g, a, 2)
    np.testing.assert_allclose(f.sum(axis=(1, 2, 3)), a.sum(axis=(1, 2, 3)), atol=1e-13)
    # each component is filtered on its own
    np.testing.assert_array_equal(f[1], O.filter_arrays(g, a[1], 2))


@pytest.mark.parametrize("nreg", [(2, 2), (4, 4)])
def test_sdmd_filtered_step_matches_sdsd(nreg):
    """With the filter on, regions filter with a J ghost exchange before each
    pass; the result is the global filter's (regions = patches at (4, 4))."""
    wl = WL.thermal_2d(n=(32, 32), ppc=4, vth=0.05, patch=(8, 8))
    gA = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch, nreg=(1, 1), filter=2)
    gB = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch, nreg=nreg, filter=2)
    g0 = O.Grid(2, wl.n, wl.d, wl.dt, patch=wl.patch)
    FA = gA.zeros_fields()
    FB, F0 = FA.copy(), FA.copy()
    PA, PB, P0 = _thermal_parts(wl), _thermal_parts(wl), _thermal_parts(wl)
    O.step_sdsd(gA, FA, PA)
    O.step_sdmd(gB, FB, PB)
    O.step_sdsd(g0, F0, P0)
    scale = np.abs(FA[9:12]).max()
    assert np.abs(FA - FB).max() <= 1e-13 * scale
    # the filter did act: the unfiltered current differs at O(1)
    assert np.abs(FA[9:12] - F0[9:12]).max() > 0.1 * scale
    np.testing.assert_allclose(FA[9:12], O.filter_arrays(g0, F0[9:12], 2), rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("nreg", [(1, 1), (3, 3)])
def test_gauss_residual_with_filter(nreg):
    """The binomial filter commutes with the discrete divergence (both are
    shift invariant and periodic), so with a filtered current
    div E - F(rho) stays constant, where F is the same filter applied to
    rho."""
    wl = WL.thermal_2d(n=(24, 24), ppc=4, vth=0.05)
    g = O.Grid(2, wl.n, wl.d, wl.dt, patch=(8, 8), nreg=nreg, filter=2)
    F = g.zeros_fields()
    P = _thermal_parts(wl)

    def resid():
        return O.divE(g, F) - O.filter_arrays(g, O.rho(g, P), 2)[0]

    r0 = resid()
    scale = np.abs(O.rho(g, P)).max()
    for _ in range(60):
        if nreg == (1, 1):
            O.step_sdsd(g, F, P)
        else:
            O.step_sdmd(g, F, P)
    r1 = resid()
    assert np.abs(r1 - r0).max() <= 1e-12 * scale
    # without filtering rho the residual drifts: the filter is really there
    r_unf = O.divE(g, F) - O.rho(g, P) - (0.0 - O.rho(g, _thermal_parts(wl)))
    assert np.abs(r_unf).max() > 1e-6 * scale


# --------------------------------------------------------------------------
# spectral (PSATD) field update
# --------------------------------------------------------------------------
from oracle import psatd as PS


def _lattice_wave(g, m, e_dir, t):
    """Plane wave of the semi-discrete Yee-lattice equations: E = e cos(k.x_E
    - w t), B = (k~ x e / w) cos(k.x_B - w t) with w = |k~|, k~_a = 2 sin(k_a
    d_a / 2) / d_a, each component at its staggered position."""
    L = [g.n[a] * g.d[a] for a in range(3)]
    k = np.array([2 * math.pi * m[a] / L[a] if a < g.dims else 0.0 for a in range(3)])
    kt = np.array([2 * math.sin(k[a] * g.d[a] / 2) / g.d[a] if a < g.dims else 0.0 for a in range(3)])
    w = math.sqrt(kt @ kt)
    e = np.array(e_dir, float)
    e = e - kt * (kt @ e) / (kt @ kt)
    e /= np.linalg.norm(e)
    b = np.cross(kt, e) / w
    nz, ny, nx = g.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    F = g.zeros_fields()
    for c in range(6):
        s = PS.STAG[c]
        ph = k[0] * (ii + 0.5 * s[0]) * g.d[0] + k[1] * (jj + 0.5 * s[1]) * g.d[1]
        if g.dims == 3:
            ph = ph + k[2] * (kk + 0.5 * s[2]) * g.d[2]
        amp = e[c] if c < 3 else b[c - 3]
        F[c] = amp * np.cos(ph - w * t)
    F[6:9] = F[3:6]
    return F, w


@pytest.mark.parametrize("dims,m,e_dir,cfl", [
    (2, (3, 2, 0), (0, 0, 1), 0.5),
    (2, (1, 4, 0), (1, 0, 0), 3.0),      # three times the Yee Courant limit
    (3, (2, 1, 3), (1, -1, 0.5), 2.0),
])
def test_psatd_vacuum_wave_exact_for_any_dt(dims, m, e_dir, cfl):
    """The spectral step integrates the lattice equations exactly in time:
    a lattice plane wave after n steps is the closed form at t = n dt, for a
    time step beyond the Yee stability limit too."""
    n = (16, 12) if dims == 2 else (8, 6, 10)
    d = (0.1, 0.15) if dims == 2 else (0.2, 0.1, 0.15)
    g = O.Grid(dims, n, d, cfl * WL.cfl_dt(d, frac=1.0))
    F, w = _lattice_wave(g, m, e_dir, 0.0)
    for _ in range(40):
        PS.step_fields(g, F)
    ref, _ = _lattice_wave(g, m, e_dir, 40 * g.dt)
    assert np.abs(F[0:6] - ref[0:6]).max() < 1e-12


def _curl_h_of(g, A):
    """Discrete curl on the Yee lattice: A at E positions -> B positions
    (forward differences), a divergence-free B."""
    dx, dy, dz = g.d
    def fwd(a, ax):
        return (np.roll(a, -1, axis=ax) - a) / [dz, dy, dx][ax]
    zero = np.zeros_like(A[0])
    dAz_dy, dAy_dz = fwd(A[2], 1), (fwd(A[1], 0) if g.dims == 3 else zero)
    dAx_dz, dAz_dx = (fwd(A[0], 0) if g.dims == 3 else zero), fwd(A[2], 2)
    dAy_dx, dAx_dy = fwd(A[1], 2), fwd(A[0], 1)
    return np.stack([dAz_dy - dAy_dz, dAx_dz - dAz_dx, dAy_dx - dAx_dy])


def test_psatd_vacuum_energy_and_uniform_current():
    """In vacuum the step is a rotation of the transverse fields: the field
    energy is conserved exactly (for a divergence-free B); a uniform current
    (the k = 0 mode) only changes E, by -dt J."""
    g = O.Grid(2, (16, 16), (0.1, 0.1), 0.2)
    rng = np.random.default_rng(11)
    F = g.zeros_fields()
    F[0:3] = rng.standard_normal((3,) + g.shape)
    F[3:6] = _curl_h_of(g, rng.standard_normal((3,) + g.shape))
    U0 = (F[0:6] ** 2).sum()
    for _ in range(30):
        PS.step_fields(g, F)
    assert (F[0:6] ** 2).sum() == pytest.approx(U0, rel=1e-12)
    G = g.zeros_fields()
    G[9:12] = np.array([0.3, -0.2, 0.7])[:, None, None, None]
    PS.step_fields(g, G)
    np.testing.assert_allclose(G[0:3], -g.dt * G[9:12], atol=1e-15)
    assert np.abs(G[3:6]).max() < 1e-15


def test_psatd_gauss_law_with_particles():
    """Esirkepov's current satisfies the lattice continuity equation and the
    spectral step keeps k~.E^{n+1} = k~.E^n - dt k~.J: div E - rho stays
    constant."""
    wl = WL.thermal_2d(n=(16, 16), ppc=4, vth=0.1)
    g = O.Grid(2, wl.n, wl.d, wl.dt)
    F = g.zeros_fields()
    P = _thermal_parts(wl)
    r0 = O.divE(g, F) - O.rho(g, P)
    scale = np.abs(O.rho(g, P)).max()
    for _ in range(60):
        PS.step(g, F, P)
    r1 = O.divE(g, F) - O.rho(g, P)
    assert np.abs(r1 - r0).max() <= 1e-12 * scale
    assert np.abs(F[0:3]).max() > 1e-4 * scale       # the plasma did drive fields


def test_psatd_matches_yee_as_dt_goes_to_zero():
    """Both integrate the same lattice equations; Yee's leapfrog is second
    order in dt, so the difference at a fixed time falls 4x when dt halves."""
    g0 = O.Grid(2, (16, 16), (0.1, 0.1), 0.02)
    rng = np.random.default_rng(5)
    E0 = 0.1 * rng.standard_normal((3,) + g0.shape)
    A = rng.standard_normal((3,) + g0.shape)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        g = O.Grid(2, (16, 16), (0.1, 0.1), dt)
        Fp = g.zeros_fields()
        Fp[0:3] = E0
        Fp[3:6] = _curl_h_of(g, A) * 0.01
        Fy = Fp.copy()
        PS.init_fields(Fp)
        O.init_fields(g, Fy)
        nsteps = int(round(0.4 / dt))
        for _ in range(nsteps):
            PS.step_fields(g, Fp)
            O.yee(g, Fy)
        errs.append(np.abs(Fp[0:3] - Fy[0:3]).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


@pytest.mark.parametrize("longitudinal", [False, True])
def test_psatd_response_to_a_current_mode(longitudinal):
    """From zero fields, a current mode held over one step gives, in closed
    form: transverse J -> E = -(sin(w dt)/w) J and B = ((1 - cos(w dt))/w^2)
    curl_h J; longitudinal J -> E = -dt J and B = 0."""
    g = O.Grid(2, (16, 12), (0.1, 0.15), 0.07)
    m = (3, 2)
    L = [g.n[a] * g.d[a] for a in range(2)]
    k = np.array([2 * math.pi * m[0] / L[0], 2 * math.pi * m[1] / L[1], 0.0])
    kt = np.array([2 * math.sin(k[0] * g.d[0] / 2) / g.d[0], 2 * math.sin(k[1] * g.d[1] / 2) / g.d[1], 0.0])
    w = math.sqrt(kt @ kt)
    e = kt / w if longitudinal else np.array([-kt[1], kt[0], 0.0]) / w
    nz, ny, nx = g.shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    F = g.zeros_fields()
    for c in range(3):
        s = PS.STAG[c]
        F[9 + c, 0] = e[c] * np.cos(k[0] * (ii + 0.5 * s[0]) * g.d[0] + k[1] * (jj + 0.5 * s[1]) * g.d[1])
    J = F[9:12].copy()
    PS.step_fields(g, F)
    if longitudinal:
        np.testing.assert_allclose(F[0:3], -g.dt * J, atol=1e-14)
        assert np.abs(F[3:6]).max() < 1e-14
    else:
        np.testing.assert_allclose(F[0:3], -math.sin(w * g.dt) / w * J, atol=1e-14)
        np.testing.assert_allclose(F[3:6], (1 - math.cos(w * g.dt)) / w ** 2 * _curl_h_of(g, J), atol=1e-14)


@pytest.mark.parametrize("dims,n", [(2, (16, 8)), (3, (8, 4, 8))])
def test_psatd_step_keeps_real_fields_real(monkeypatch, dims, n):
    """The spectral step maps the spectra of real fields to spectra of real
    fields: each lattice wavenumber k~_a multiplies a half-cell shift along
    the same axis, so the step at -k of conj A(k) is the conjugate of the
    step at k for every wavevector, the Nyquist planes (where the sampled
    -pi/d stands for +pi/d) included.  The inverse transforms of random
    fields, which carry every wavevector, then have no imaginary part.  (The
    GPU path steps k and obtains -k by conjugation, so it relies on this.)"""
    worst = []
    orig = PS.from_spectrum

    def recording(g, X, comp, ks):
        z = np.fft.ifftn(X * PS._phase(ks, g, comp, +1.0), axes=(0, 1, 2))
        worst.append(np.abs(z.imag).max() / np.abs(z.real).max())
        return orig(g, X, comp, ks)

    monkeypatch.setattr(PS, "from_spectrum", recording)
    d = (0.1, 0.15, 0.12)[:dims]
    g = O.Grid(dims, n, d, 0.9 * min(d))
    rng = np.random.default_rng(5 + dims)
    F = g.zeros_fields()
    F[0:6] = rng.standard_normal(F[0:6].shape)
    F[9:12] = rng.standard_normal(F[9:12].shape)
    PS.init_fields(F)
    PS.step_fields(g, F)
    assert len(worst) == 6
    assert max(worst) < 1e-13
