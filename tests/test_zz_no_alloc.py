"""The allocation-free dipole entry point (ks_dipole_noalloc) against the
system's ks_dipole: same kernels and summation order, so the results must be
bit-identical; also against the oracle's dipole at 1e-12.  Two calls in a row
share the device's static scratch, the second on a smaller grid."""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _density(spec, seed):
    # a positive, seeded field with the grid's shape (any density will do)
    rng = np.random.default_rng(seed)
    return rng.random(spec.n) + 0.1


def test_dipole_noalloc_equals_system_dipole(ks):
    for name, seed in (("t48", 5), ("t24", 6)):          # second call: smaller grid
        print(f"[case] dipole_noalloc {name}", file=sys.stderr, flush=True)
        spec = synth.CONFIGS[name]
        rho_np = _density(spec, seed)
        rho = torch.from_numpy(rho_np).cuda()
        gs = ks.System(spec.n, spec.L, spec.ecut, 1)
        ref = gs.dipole(rho)
        d = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        ks.dipole_noalloc(spec.n, spec.L, rho, d)
        torch.cuda.synchronize()
        assert torch.equal(d, ref), (d, ref)
        g = ko.Grid(spec.n, spec.L, spec.ecut)
        want = ko.dipole(g, rho_np)
        np.testing.assert_allclose(d.cpu().numpy(), want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
        gs.close()


def test_dipole_noalloc_rejects_bad_sizes(ks):
    rho = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    d = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(ks.KSError) as e:
        ks.dipole_noalloc((4, 4, 4), (1.0, 0.0, 1.0), rho, d)
    assert e.value.status == ks.KS_EINVAL
    lib = ks.library()
    import ctypes
    n = (ctypes.c_int * 3)(2048, 2048, 1024)            # 2^32 points: beyond the limit
    L = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    st = lib.ks_dipole_noalloc(n, L, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(d.data_ptr()), None)
    assert st == ks.KS_EINVAL
    assert b"limit" in lib.ks_last_error(None)
