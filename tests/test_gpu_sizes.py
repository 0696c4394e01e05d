"""Every grid size the library accepts, as the x-pencil length n0 and as the
plane size n1 = n2, against the FP64 oracle (H psi at 1e-12 in FP64 and 1e-5
in mixed precision, with either projection mode; a two-step resident propagation with its densities at
1e-12).  The 16, 24, 32, 40, 48, 60, 64, 96 and 120-point kernels are covered
by the other parity tests; these anisotropic grids cover the rest with a
grid spacing of 0.33-0.6 bohr, so the E_cut = 10 Ha sphere stays inside the
box and each cell holds a whole projector sphere (R_c = 2 bohr).
"""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth

from gpu_common import oracle_ham, orbitals_device, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12
TOL_MIXED = 1e-5

# (n, L, natoms): n0 covers 8 12 20 72 80 128, n1 = n2 covers 12 8 72 80 128 20
GRIDS = [
    ((8, 12, 12), (4.8, 7.2, 7.2), 1),
    ((12, 8, 8), (7.2, 4.8, 4.8), 1),
    ((20, 72, 72), (6.6, 23.8, 23.8), 4),
    ((72, 80, 80), (23.8, 26.4, 26.4), 6),
    ((80, 128, 128), (26.4, 40.0, 40.0), 6),
    ((128, 20, 20), (42.0, 6.6, 6.6), 3),
]


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


@pytest.mark.parametrize("n,L,natoms", GRIDS, ids=["x".join(map(str, g[0])) for g in GRIDS])
def test_grid_size_parity(ks, n, L, natoms):
    name = "g" + "x".join(map(str, n))
    print(f"[case] sizes {name}", file=sys.stderr, flush=True)
    spec = synth.Spec(name=name, n=n, L=L, ecut=10.0, norb=3, natoms=natoms, seed=8100 + n[0] + n[1])
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    ref = ko.ham_apply(ham, c0)
    gs = ks.system_from_synth(sysm)
    got = gs.ham_apply(c).cpu().numpy()
    assert rel_err(got, ref) < TOL
    assert np.all(got[:, ~ham.grid.chi] == 0)
    gm = ks.system_from_synth(sysm, precision=ks.KS_MIXED)
    assert rel_err(gm.ham_apply(c).cpu().numpy(), ref) < TOL_MIXED
    gm.set_tuning(gm.info()["x_group"], gm.info()["plane_group"], projection=1)   # split-BF16 projections
    assert rel_err(gm.ham_apply(c).cpu().numpy(), ref) < TOL_MIXED
    gm.close()
    occ_np = np.array([2.0, 1.0, 0.5])
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    rho = torch.empty((2,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate(spec.dt, 2, occ, rho)
    r = c0
    for s in range(2):
        r = ko.taylor4_step(ham, r, spec.dt, 1)
        rr = ko.density(ham, r, occ_np)
        assert np.linalg.norm(rho[s].cpu().numpy() - rr) / np.linalg.norm(rr) < TOL
    assert rel_err(st.download().cpu().numpy(), r) < TOL
    st.close()
    gs.close()
