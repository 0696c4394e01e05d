"""Steepest-descent eigensolver (Section "Ground-state solution") on the
device against the FP64 oracle: orbitals, Ritz values and residual norms
after every iteration, from orthonormalised random orbitals; ragged orbital
counts (one orbital, an odd count, several passes; 33 and 128 orbitals,
whose subspace problems span several padded Jacobi blocks), a longer run
that converges, and the error paths.

Tolerance: the iteration is FP64 throughout; its operations (H psi at 1e-12,
reductions, dense products, Jacobi rotations) each round at 1e-15 -- 1e-12,
and a few iterations contract rather than amplify differences, so 1e-9
relative on the orbitals and 1e-10 on the Ritz values is a wide margin.
"""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth

from gpu_common import oracle_ham, orbitals_device, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_C = 1e-9
TOL_E = 1e-10


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _start(ks, name, norb=None, chunk=None):
    print(f"[case] ground {name} norb={norb} chunk={chunk}", file=sys.stderr, flush=True)
    spec = synth.CONFIGS[name]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    if chunk:
        gs.set_chunk(chunk)
    c = orbitals_device(spec, norb)
    gs.orthonormalize(c)
    st = ks.State(gs, c.shape[0])
    st.upload(c)
    return spec, ham, gs, st, c.cpu().numpy()


def _oracle_run(ham, c0, K):
    c, E, RN = c0, [], []
    for _ in range(K):
        c, e, rn = ko.sd_iteration(ham, c)
        E.append(e)
        RN.append(rn)
    return c, np.array(E), np.array(RN)


@pytest.mark.parametrize("name,norb,chunk", [("t24", None, None), ("cfg1_16", None, None), ("t32x", 5, None),
                                             ("t24", 1, None), ("t24", None, 4), ("t48", 12, None),
                                             ("t48", None, None), ("cfg2_64", None, None)])
def test_sd_iterations_vs_oracle(ks, name, norb, chunk):
    spec, ham, gs, st, c0 = _start(ks, name, norb, chunk)
    K = 3
    eig, resid = st.eigensolve(K)
    got = st.download().cpu().numpy()
    ref, E, RN = _oracle_run(ham, c0, K)
    e_err = np.abs(eig.cpu().numpy() - E).max() / np.abs(E).max()
    print(f"[ground] {name}: orbital rel err {rel_err(got, ref):.2e}, Ritz value err {e_err:.2e}", file=sys.stderr)
    assert rel_err(got, ref) < TOL_C
    assert e_err < TOL_E
    np.testing.assert_allclose(resid.cpu().numpy(), RN, rtol=1e-8)
    assert np.all(got[:, ~ham.grid.chi] == 0)
    st.close()


def test_sd_converges(ks):
    """40 iterations: the Ritz values settle and match the oracle's run, the
    residuals fall by orders of magnitude, the orbitals stay orthonormal."""
    spec, ham, gs, st, c0 = _start(ks, "t24")
    K = 40
    eig, resid = st.eigensolve(K)
    e, r = eig.cpu().numpy(), resid.cpu().numpy()
    _, E, RN = _oracle_run(ham, c0, K)
    print(f"[ground] 40 iterations: max residual {r[0].max():.2e} -> {r[-1].max():.2e}; "
          f"Ritz err vs oracle {np.abs(e[-1] - E[-1]).max():.2e}", file=sys.stderr)
    assert np.abs(e[-1] - E[-1]).max() < 1e-9 * np.abs(E[-1]).max()
    assert r[-1].max() < 1e-2 * r[0].max()
    assert np.all(np.diff(e[-1]) > 0)
    assert np.all(np.diff(e.sum(axis=1))[5:] < 1e-9)
    C = st.download().cpu().numpy().reshape(spec.norb, -1)
    np.testing.assert_allclose(C.conj() @ C.T, np.eye(spec.norb), atol=1e-12)
    st.close()


def test_sd_errors(ks):
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    gm = ks.system_from_synth(sysm, precision=ks.KS_MIXED)
    st = ks.State(gm, 2)
    with pytest.raises(ks.KSError) as ei:
        st.eigensolve(1)
    assert ei.value.status == ks.KS_EUNSUPPORTED
    st.close()
    g = ks.system_from_synth(sysm)
    st = ks.State(g, 2)
    with pytest.raises(ks.KSError) as ei:
        st.eigensolve(-1)
    assert ei.value.status == ks.KS_EINVAL
    st.close()


def test_sd_full_size_cfg3(ks):
    """96^3, 512 orbitals, 128 atoms (the benchmark's system): the first
    iteration's Ritz values equal the eigenvalues (LAPACK) of C^H H C with
    H C from the oracle (the products over the sphere's coefficients, where
    C and H C live), and the orbitals come back orthonormal."""
    print("[case] ground cfg3_96 full size", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["cfg3_96"]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    gs.orthonormalize(c)
    c0 = c.cpu().numpy()
    chi = ham.grid.chi.reshape(-1)
    C = c0.reshape(spec.norb, -1)[:, chi]
    Hs = np.empty((spec.norb, spec.norb), complex)
    for o in range(0, spec.norb, 64):
        hc = ko.ham_apply(ham, c0[o:o + 64]).reshape(-1, chi.size)[:, chi]
        Hs[:, o:o + 64] = C.conj() @ hc.T
    del c0
    lam = np.linalg.eigvalsh(0.5 * (Hs + Hs.conj().T))
    st = ks.State(gs, spec.norb)
    st.upload(c)
    del c, C
    eig, resid = st.eigensolve(2)
    e = eig.cpu().numpy()
    err = np.abs(e[0] - lam).max() / np.abs(lam).max()
    print(f"[ground] cfg3_96: Ritz values vs oracle H {err:.2e}; residual max {resid[0].max().item():.3e} -> "
          f"{resid[1].max().item():.3e}", file=sys.stderr)
    assert err < 1e-11
    assert np.all(np.diff(e[1]) >= 0)
    out = st.download().reshape(spec.norb, -1)
    S = (out.conj() @ out.T).cpu().numpy()
    assert np.abs(S - np.eye(spec.norb)).max() < 1e-11
    st.close()


def test_sd_is_deterministic(ks):
    """Fixed-order reductions everywhere: two runs from the same start give
    bit-identical orbitals, Ritz values and residual norms."""
    spec, ham, gs, st, c0 = _start(ks, "t48")
    st2 = ks.State(gs, spec.norb)
    st2.upload(torch.from_numpy(c0).cuda())
    e1, r1 = st.eigensolve(3)
    e2, r2 = st2.eigensolve(3)
    assert torch.equal(e1, e2) and torch.equal(r1, r2)
    assert torch.equal(st.download(), st2.download())
    st.close()
    st2.close()


def test_sd_local_only_system(ks):
    """No projectors (the x-projection pass is skipped): 3 iterations against
    the oracle on the t24 grid with its local potential only."""
    print("[case] ground t24 local only", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    ham = ko.Hamiltonian(g, sysm.vloc)
    gs = ks.System(spec.n, spec.L, spec.ecut, spec.norb)
    gs.set_vloc(torch.from_numpy(sysm.vloc).cuda())
    c = orbitals_device(spec)
    gs.orthonormalize(c)
    c0 = c.cpu().numpy()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    eig, resid = st.eigensolve(3)
    ref, E, RN = _oracle_run(ham, c0, 3)
    got = st.download().cpu().numpy()
    print(f"[ground] t24 local only: orbital rel err {rel_err(got, ref):.2e}", file=sys.stderr)
    assert rel_err(got, ref) < TOL_C
    assert np.abs(eig.cpu().numpy() - E).max() < TOL_E * np.abs(E).max()
    np.testing.assert_allclose(resid.cpu().numpy(), RN, rtol=1e-8)
    st.close()
