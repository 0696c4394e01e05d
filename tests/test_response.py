"""Host-side absorption spectrum from a dipole time series."""
import numpy as np

from paper_2106_03872_amd import response


def test_single_oscillator_peak_and_sum_rule():
    # one oscillator of strength f kicked with momentum k: d(t) - d(0) =
    # k f / w0 sin(w0 t) (f electrons start moving with velocity k); the
    # spectrum peaks at w0 and integrates to f
    w0, f, kk, dt = 0.6, 0.8, 1e-3, 0.05
    t = dt * np.arange(8000)
    dz = kk * f / w0 * np.sin(w0 * t)
    dip = np.stack([np.zeros_like(t), np.zeros_like(t), dz], axis=1)
    w = np.linspace(0.05, 1.5, 2901)
    alpha, S = response.absorption_spectrum(dip, dt, (0.0, 0.0, kk), w, damping=0.01)
    assert abs(w[np.argmax(S)] - w0) < 0.01
    integral = np.trapezoid(S, w) if hasattr(np, "trapezoid") else np.trapz(S, w)
    assert abs(integral - f) < 0.05 * f


def test_rejects_zero_kick():
    import pytest
    with pytest.raises(ValueError):
        response.absorption_spectrum(np.zeros((3, 3)), 0.1, (0, 0, 0), [0.1])
