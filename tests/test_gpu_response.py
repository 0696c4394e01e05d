"""Absorption spectrum on the device (ks_spectrum) against the oracle's, on
seeded synthetic dipole series (damped oscillators along several directions
plus noise).  Tolerance: the sums run in a different order, so the bound is
1e-12 of dt sum |x| / |k| (the sum of the magnitudes of the terms)."""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def resp():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import response
    return response


def _series(seed, nt, dt):
    rng = np.random.default_rng(seed)
    t = dt * np.arange(nt)
    d = rng.standard_normal(3)[None, :] + np.zeros((nt, 3))
    for _ in range(4):
        w0, g = rng.uniform(0.2, 1.5), rng.uniform(0.0, 0.02)
        d += 1e-3 * rng.standard_normal(3)[None, :] * (np.sin(w0 * t) * np.exp(-g * t))[:, None]
    d += 1e-7 * rng.standard_normal((nt, 3))
    return d


@pytest.mark.parametrize("nt,seed", [(1, 1), (2, 2), (257, 3), (6000, 4)])
def test_spectrum_matches_oracle(resp, nt, seed):
    print(f"[case] spectrum nt={nt}", file=sys.stderr, flush=True)
    dt, k, eta = 0.05, np.array([1e-3, -2e-3, 5e-4]), 0.007
    d = _series(seed, nt, dt)
    w = np.linspace(0.0, 2.0, 513)
    alpha, S = resp.absorption_spectrum(d, dt, k, w, eta)
    ra, rS = ko.spectrum(d, dt, k, w, eta)
    x = (d - d[0]) @ (k / np.linalg.norm(k))
    bound = 1e-12 * dt * np.abs(x).sum() / np.linalg.norm(k) + 1e-300
    assert np.abs(alpha.cpu().numpy() - ra).max() <= bound
    assert np.abs(S.cpu().numpy() - rS).max() <= bound * 2 * w.max() / np.pi


def test_spectrum_errors(resp):
    from paper_2106_03872_amd import ks
    with pytest.raises(ks.KSError):
        resp.absorption_spectrum(np.zeros((3, 3)), 0.1, (0, 0, 0), [0.1])
    with pytest.raises(ks.KSError):
        resp.absorption_spectrum(np.zeros((3, 3)), -0.1, (1, 0, 0), [0.1])
