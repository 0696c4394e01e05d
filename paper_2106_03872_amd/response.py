"""Optical absorption from a kicked propagation (host side).

After a field kick ``exp(i k.r)`` at t = 0 (``State.kick``; the electrons
gain momentum k) the dipole moment ``d(t)`` (``System.dipole`` of each step's
density, the first moment of the electron number density) responds linearly
for a small kick; the absorption (dipole strength) along the kick direction is
``S(w) = (2 w / pi) Im[alpha(w)]`` with
``alpha(w) = (1/|k|) int_0^T (d(t) - d(0)) . k_hat e^{i w t} e^{-eta t} dt``,
normalised so that the integral of S over w is the number of electrons
(f-sum rule)
(Section "Results": the spectrum is the Fourier transform of the dipole
moments recorded after the kick).  The time integral is the trapezoidal rule
over the recorded steps.
"""
from __future__ import annotations

import numpy as np


def absorption_spectrum(dipoles, dt, k, omegas, damping=0.005):
    """dipoles: [nsteps + 1, 3] with d(0) first (the density right after the
    kick); dt: time step; k: kick vector; omegas: frequencies (Ha).  Returns
    (alpha(w) complex, S(w))."""
    d = np.asarray(dipoles, np.float64)
    k = np.asarray(k, np.float64)
    kn = float(np.linalg.norm(k))
    if kn == 0.0:
        raise ValueError("the kick must be non-zero")
    x = (d - d[0]) @ (k / kn)
    t = dt * np.arange(len(x))
    w = np.asarray(omegas, np.float64)[:, None]
    f = x[None, :] * np.exp(1j * w * t[None, :] - damping * t[None, :])
    integral = dt * (f.sum(axis=1) - 0.5 * (f[:, 0] + f[:, -1]))
    alpha = integral / kn
    return alpha, 2.0 * w[:, 0] / np.pi * alpha.imag
