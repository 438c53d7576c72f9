"""Spectral (PSATD) Maxwell update for the oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this module; the HIP library shares no code with it.

The paper names a spectral Maxwell solver on large regions as the motivation
of SDMD (sections 1 and 2.2: FFTs need large, contiguous subdomains).  This
module integrates, exactly in time, the semi-discrete Maxwell equations of
the Yee lattice on one periodic grid:

    dE/dt = curl_h B - J,      dB/dt = -curl_h E,

where curl_h is the staggered centred difference of the Yee scheme.  With
every component transformed at its own (staggered) position, curl_h becomes
i k~ x in Fourier space with the lattice wavenumber k~_a = 2 sin(k_a d_a / 2)
/ d_a.  Over one step with J held at J^{n+1/2}, and omega = |k~|,
kappa = k~ / omega, C = cos(omega dt), S = sin(omega dt):

    E^{n+1} = C E + (1 - C) kappa (kappa.E) + i S kappa x B
              - (S / omega) J + kappa (kappa.J) (S / omega - dt)
    B^{n+1} = C B - i S kappa x E + i ((1 - C) / omega) kappa x J

(the k~ = 0 mode: E -= dt J, B unchanged).  This follows from splitting E
into its part along kappa, which only integrates -J, and the transverse
part, which rotates with B at angular frequency omega.  Because
k~ . E^{n+1} = k~ . E^n - dt k~ . J, the discrete Gauss law kept by
Esirkepov's deposition holds exactly, as with the Yee update.

State for this solver: E^n and B^n at the same time (no half-step
staggering in time); Bm^n = B^n.  Field arrays follow the oracle's layout
(12, nz, ny, nx): E, B, Bm, J.  The FFT is numpy's.
"""
from __future__ import annotations

import numpy as np

# staggering of E (0..2) and B (3..5) components: 1 = half-integer position
STAG = {0: (1, 0, 0), 1: (0, 1, 0), 2: (0, 0, 1), 3: (0, 1, 1), 4: (1, 0, 1), 5: (1, 1, 0)}
STAG.update({9 + c: STAG[c] for c in range(3)})   # J like E


def wavenumbers(g):
    """Per-axis FFT wavenumbers k (physical) and lattice wavenumbers k~,
    shaped to broadcast over (nz, ny, nx)."""
    ks, kts = [], []
    for a in range(3):
        n = g.n[a]
        if a >= g.dims:
            k = np.zeros(n)
            kt = np.zeros(n)
        else:
            k = 2.0 * np.pi * np.fft.fftfreq(n, d=g.d[a])
            kt = 2.0 * np.sin(0.5 * k * g.d[a]) / g.d[a]
        shape = [1, 1, 1]
        shape[2 - a] = n
        ks.append(k.reshape(shape))
        kts.append(kt.reshape(shape))
    return ks, kts


def _phase(ks, g, comp, sign):
    s = STAG[comp]
    ph = 0.0
    for a in range(g.dims):
        ph = ph + ks[a] * 0.5 * s[a] * g.d[a]
    return np.exp(sign * 1j * ph)


def to_spectrum(g, F, comp, ks):
    """Transform of one component at its physical (staggered) positions."""
    return np.fft.fftn(F[comp], axes=(0, 1, 2)) * _phase(ks, g, comp, -1.0)


def from_spectrum(g, X, comp, ks):
    return np.real(np.fft.ifftn(X * _phase(ks, g, comp, +1.0), axes=(0, 1, 2)))


def step_fields(g, F):
    """One exact step of E^n, B^n with J = F[9:12] (J^{n+1/2}); writes E^{n+1},
    B^{n+1} and Bm = B^{n+1} into F."""
    ks, kts = wavenumbers(g)
    dt = g.dt
    E = [to_spectrum(g, F, c, ks) for c in range(3)]
    B = [to_spectrum(g, F, 3 + c, ks) for c in range(3)]
    J = [to_spectrum(g, F, 9 + c, ks) for c in range(3)]
    kt = np.broadcast_arrays(*kts)
    w = np.sqrt(kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2)
    zero = w == 0.0
    ws = np.where(zero, 1.0, w)
    kap = [np.where(zero, 0.0, kt[a] / ws) for a in range(3)]
    C = np.cos(w * dt)
    S = np.sin(w * dt)
    S_w = np.where(zero, dt, S / ws)
    C1_w = np.where(zero, 0.0, (1.0 - C) / ws)

    def cross(a, b):
        return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]

    kE = kap[0] * E[0] + kap[1] * E[1] + kap[2] * E[2]
    kJ = kap[0] * J[0] + kap[1] * J[1] + kap[2] * J[2]
    kxB, kxE, kxJ = cross(kap, B), cross(kap, E), cross(kap, J)
    En = [C * E[c] + (1.0 - C) * kap[c] * kE + 1j * S * kxB[c] - S_w * J[c] + kap[c] * kJ * (S_w - dt)
          for c in range(3)]
    Bn = [C * B[c] - 1j * S * kxE[c] + 1j * C1_w * kxJ[c] for c in range(3)]
    for c in range(3):
        F[c] = from_spectrum(g, En[c], c, ks)
        F[3 + c] = from_spectrum(g, Bn[c], 3 + c, ks)
        F[6 + c] = F[3 + c]


def init_fields(F):
    """State at t = 0 from E^0, B^0 in F[0:6]: Bm^0 = B^0, no half step."""
    F[6:9] = F[3:6]


def step(g, F, P):
    """One PIC step with the spectral field update: particles and deposition
    as in the oracle's undecomposed mode (B for the push is Bm^n = B^n), the
    binomial filter of the grid if it has one, then step_fields."""
    import oracle as O
    maxd = O.particles_sdsd(g, F, P)
    if g.filter > 0:
        F[9:12] = O.filter_arrays(g, F[9:12], g.filter)
    step_fields(g, F)
    return maxd
