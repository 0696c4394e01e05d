"""FP64 parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: 1e-12 relative per orbital on H psi (the FP64 target), and the
same bound on every quantity derived from it (Taylor-4 steps, density,
norms, band energy).  Integer/structural facts (zeros outside the sphere,
determinism, chunk independence) are checked bit-exactly.
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
SMALL = ["cfg1_16", "t24", "t40", "t32x", "t60", "t48"]


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _case(name):
    print(f"[case] {name}", file=sys.stderr, flush=True)
    spec = synth.CONFIGS[name]
    return spec, synth.system(spec)


@pytest.mark.parametrize("name", SMALL)
def test_ham_apply_parity(ks, name):
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    hc = gs.ham_apply(c)
    torch.cuda.synchronize()
    ref = ko.ham_apply(ham, c.cpu().numpy())
    got = hc.cpu().numpy()
    assert rel_err(got, ref) < TOL
    assert np.all(got[:, ~ham.grid.chi] == 0)


def test_ham_apply_chunking_is_exact(ks):
    spec, sysm = _case("t48")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    a = gs.ham_apply(c).clone()
    gs.set_chunk(7)                      # 33 orbitals -> 4 full chunks + a ragged one
    assert gs.chunk == 7
    b = gs.ham_apply(c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_autotune_keeps_results_and_caches(ks):
    spec, sysm = _case("t48")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    a = gs.ham_apply(c).clone()
    t = gs.autotune(spec.norb)
    assert t["x_group"] in (2, 4, 8, 16, 32, 64) and t["plane_group"] in (1, 2, 4, 8, 16)
    info = gs.info()
    assert (info["x_group"], info["plane_group"]) == (t["x_group"], t["plane_group"])
    assert torch.equal(a, gs.ham_apply(c))
    # every launch schedule gives bit-identical results
    for xg, pg in ((1, 1), (3, 5), (16, 8), (64, 64)):
        gs.set_tuning(xg, pg)
        assert torch.equal(a, gs.ham_apply(c))
    with pytest.raises(ks.KSError):
        gs.set_tuning(0, 1)
    gs2 = ks.system_from_synth(sysm)
    t2 = gs2.autotune(spec.norb)
    assert t2["from_cache"] and (t2["x_group"], t2["plane_group"]) == (t["x_group"], t["plane_group"])
    with pytest.raises(ks.KSError):
        gs2.autotune(0)


def test_ham_apply_deterministic(ks):
    spec, sysm = _case("t40")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    a = gs.ham_apply(c).clone()
    b = gs.ham_apply(c)
    assert torch.equal(a, b)


def test_full_box_no_cutoff(ks):
    spec = synth.Spec(name="box16", n=(16, 16, 16), L=(8.0, 8.0, 8.0), ecut=0.0, norb=3, natoms=2, seed=77)
    print("[case] box16", file=sys.stderr, flush=True)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    assert gs.npw == 16 ** 3
    c = orbitals_device(spec)
    ref = ko.ham_apply(ham, c.cpu().numpy())
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ref) < TOL


def test_local_only_and_kinetic_only(ks):
    spec, sysm = _case("t24")
    c = orbitals_device(spec)
    # no projectors
    ham = oracle_ham(sysm)
    ham.atoms = []
    gs = ks.System(spec.n, spec.L, spec.ecut, spec.norb)
    gs.set_vloc(torch.from_numpy(sysm.vloc).cuda())
    gs.set_projectors(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros((0, 4)))
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ko.ham_apply(ham, c.cpu().numpy())) < TOL
    # plane waves: V = 0, no atoms -> eigenvalue |G|^2/2 on the sphere
    gk = ks.System(spec.n, spec.L, spec.ecut, spec.norb)
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    hc = gk.ham_apply(c).cpu().numpy()
    expect = np.where(g.chi, g.K * c.cpu().numpy(), 0)
    assert rel_err(hc, expect) < TOL


def test_propagate_and_density_parity(ks):
    spec, sysm = _case("t24")       # 2 steps, dt = 0.05
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    occ = torch.from_numpy(synth.occupations(spec)).cuda()
    rho = torch.empty((spec.nsteps,) + spec.n, dtype=torch.float64, device="cuda")
    gs.propagate_step(c, spec.dt, spec.nsteps, occ, rho)
    torch.cuda.synchronize()
    ref = ko.taylor4_step(ham, c0, spec.dt, spec.nsteps)
    assert rel_err(c.cpu().numpy(), ref) < TOL
    for s in range(spec.nsteps):
        rs = ko.density(ham, ko.taylor4_step(ham, c0, spec.dt, s + 1), synth.occupations(spec))
        r = rho[s].cpu().numpy()
        assert np.linalg.norm(r - rs) / np.linalg.norm(rs) < TOL


@pytest.mark.parametrize("name", ["t48", "t24"])
def test_state_multistep_density_and_norms(ks, name):
    # one call of K steps: the densities of steps 0..K-2 come from the next
    # step's first H psi, the last from a density pass; norms after each step
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    occ_np = np.linspace(0.5, 2.0, spec.norb)
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    K = 3
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    nrm = torch.empty((K, spec.norb), dtype=torch.float64, device="cuda")
    st.propagate(spec.dt, K, occ, rho, nrm)
    torch.cuda.synchronize()
    for s in range(K):
        cs = ko.taylor4_step(ham, c0, spec.dt, s + 1)
        rs = ko.density(ham, cs, occ_np)
        r = rho[s].cpu().numpy()
        assert np.linalg.norm(r - rs) / np.linalg.norm(rs) < TOL
        np.testing.assert_allclose(nrm[s].cpu().numpy(), ko.norms(ham, cs), rtol=TOL)
    assert rel_err(st.download().cpu().numpy(), ko.taylor4_step(ham, c0, spec.dt, K)) < TOL
    st.close()


@pytest.mark.parametrize("name", ["cfg1_16", "t40", "t48"])
def test_density_and_reduce_parity(ks, name):
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    occ_np = np.linspace(0.5, 2.0, spec.norb)
    occ = torch.from_numpy(occ_np).cuda()
    rho = gs.density(c, occ).cpu().numpy()
    cn = c.cpu().numpy()
    rr = ko.density(ham, cn, occ_np)
    assert np.linalg.norm(rho - rr) / np.linalg.norm(rr) < TOL
    norms, energy = gs.reduce(c, occ)
    np.testing.assert_allclose(norms.cpu().numpy(), ko.norms(ham, cn), rtol=TOL)
    E, _ = ko.band_energy(ham, cn, occ_np)
    assert abs(energy.item() - E) < TOL * abs(E)


def test_propagate_zero_steps_and_empty(ks):
    spec, sysm = _case("cfg1_16")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c_before = c.clone()
    gs.propagate_step(c, 0.05, 0)
    assert torch.equal(c, c_before)
    empty = torch.zeros((0,) + spec.n, dtype=torch.complex128, device="cuda")
    gs.ham_apply(empty)


def test_errors_are_reported(ks):
    spec, sysm = _case("cfg1_16")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    with pytest.raises(ks.KSError) as e:
        gs.ham_apply(c, c)
    assert e.value.status == ks.KS_EINVAL
    big = torch.zeros((spec.norb + 1,) + spec.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(ks.KSError):
        gs.ham_apply(big)


# ---------------------------------------------------- full size, sampled outputs

def test_full_size_cfg3_sampled(ks):
    """96^3 grid, 512 orbitals, 128 atoms in the benchmark's launch
    configuration; the oracle recomputes sampled orbitals one by one (orbitals
    are independent), and the density is sampled with one-hot occupations."""
    spec, sysm = _case("cfg3_96")
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    hc = gs.ham_apply(c)
    sample = [0, 137, spec.norb - 1]
    cs = c[sample].cpu().numpy()
    assert rel_err(hc[sample].cpu().numpy(), ko.ham_apply(ham, cs)) < TOL
    occ = torch.zeros(spec.norb, dtype=torch.float64, device="cuda")
    occ[137] = 2.0
    rho = torch.empty((1,) + spec.n, dtype=torch.float64, device="cuda")
    gs.propagate_step(c, spec.dt, 1, occ, rho)
    ref = ko.taylor4_step(ham, cs, spec.dt, 1)
    assert rel_err(c[sample].cpu().numpy(), ref) < TOL
    rr = ko.density(ham, ref[1:2], [2.0])
    assert np.linalg.norm(rho[0].cpu().numpy() - rr) / np.linalg.norm(rr) < TOL


# ------------------------------------------------------- orthonormalisation (a10)

@pytest.mark.parametrize("name", ["t24", "t48", "cfg2_64"])
def test_orthonormalize_parity(ks, name):
    """Cholesky orthonormalisation vs the oracle.  The Cholesky factor is
    unique (positive diagonal), so the result is compared element by element;
    the tolerance scales with the conditioning of the overlap matrix
    (first-order perturbation of a Cholesky factor is bounded by
    cond(S) times the rounding of S)."""
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    cn = c.cpu().numpy()
    ref = ko.orthonormalize(ham, cn)
    A = np.where(ham.grid.chi, cn, 0).reshape(spec.norb, -1)
    sv = np.linalg.svd(A, compute_uv=False)
    cond = (sv[0] / sv[-1]) ** 2
    gs.orthonormalize(c)
    got = c.cpu().numpy()
    tol = max(1e-12, 1e-14 * cond * np.sqrt(spec.norb))
    assert rel_err(got, ref) < tol, (rel_err(got, ref), cond)
    M = got.reshape(spec.norb, -1)
    assert np.abs(M.conj() @ M.T - np.eye(spec.norb)).max() < 1e-12
    assert np.all(got[:, ~ham.grid.chi] == 0)


def test_orthonormalize_rejects_dependent(ks):
    spec, sysm = _case("t24")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c[3] = c[1]                                    # linearly dependent set
    with pytest.raises(ks.KSError) as e:
        gs.orthonormalize(c)
    assert e.value.status == ks.KS_EINVAL


# ------------------------------------------------------------------ edge cases

def test_anisotropic_grid_and_ragged_tile(ks):
    """n0 != n1 = n2 (different x-pencil length), non-cubic cell; 40*40 = 1600
    pencils is not a multiple of the 32-pencil x-tile width... (50 tiles), and
    the 60-point case in SMALL covers a ragged last tile."""
    spec = synth.Spec(name="aniso", n=(24, 40, 40), L=(7.5, 12.5, 13.0), ecut=10.0, norb=5, natoms=3, seed=91)
    print("[case] aniso", file=sys.stderr, flush=True)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ko.ham_apply(ham, c.cpu().numpy())) < TOL
    occ = torch.full((spec.norb,), 1.5, dtype=torch.float64, device="cuda")
    rho = gs.density(c, occ).cpu().numpy()
    rr = ko.density(ham, c.cpu().numpy(), np.full(spec.norb, 1.5))
    assert np.linalg.norm(rho - rr) / np.linalg.norm(rr) < TOL


def test_duplicate_and_overlapping_projector_points(ks):
    """Projector lists with a repeated point inside one atom and two atoms
    sharing points: every entry counts (the sums of Eq. vnl run over list
    entries)."""
    spec = synth.CONFIGS["t24"]
    print("[case] duplicates", file=sys.stderr, flush=True)
    sysm = synth.system(spec)
    rng = np.random.default_rng(12)
    npts = sysm.proj.npts.copy()
    idx = sysm.proj.idx.copy()
    beta = sysm.proj.beta.copy()
    idx[5] = idx[6]                                   # duplicate within atom 0
    o1 = int(npts[0])
    idx[o1:o1 + 20] = idx[0:20]                       # atom 1 shares 20 points with atom 0
    beta[o1:o1 + 20] = rng.standard_normal((20, 4))
    atoms = []
    off = 0
    for n_ in npts:
        atoms.append((idx[off:off + n_], beta[off:off + n_]))
        off += n_
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    ham = ko.Hamiltonian(g, sysm.vloc, atoms, sysm.proj.d)
    gs = ks.System(spec.n, spec.L, spec.ecut, spec.norb)
    gs.set_vloc(torch.from_numpy(sysm.vloc).cuda())
    gs.set_projectors(npts, idx, beta, sysm.proj.d)
    c = orbitals_device(spec)
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ko.ham_apply(ham, c.cpu().numpy())) < TOL


def test_single_orbital_and_max_chunk(ks):
    spec, sysm = _case("t40")
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    gs.set_chunk(spec.norb)
    one = c[2:3].contiguous()
    assert rel_err(gs.ham_apply(one).cpu().numpy(), ko.ham_apply(ham, one.cpu().numpy())) < TOL
    gs.set_chunk(1)
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ko.ham_apply(ham, c.cpu().numpy())) < TOL


# ------------------------------------------ Hartree potential and ETRS (NEXT rows)

@pytest.mark.parametrize("name", ["t24", "t32x", "t48"])
def test_hartree_parity(ks, name):
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    rng = np.random.default_rng(5)
    rho_np = rng.random(spec.n) + 0.5
    rho = torch.from_numpy(rho_np).cuda()
    v = gs.hartree(rho).cpu().numpy()
    ref = ko.hartree(ham.grid, rho_np)
    assert np.linalg.norm(v - ref) / np.linalg.norm(ref) < TOL
    vt = gs.hartree(rho, add_vloc=True).cpu().numpy()
    reft = ref + sysm.vloc.reshape(spec.n)
    assert np.linalg.norm(vt - reft) / np.linalg.norm(reft) < TOL
    # in place (rho and v the same array)
    gs.hartree(rho, out=rho)
    assert np.linalg.norm(rho.cpu().numpy() - ref) / np.linalg.norm(ref) < TOL


@pytest.mark.parametrize("name", ["t24", "t48"])
def test_etrs_parity(ks, name):
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    # unit-norm orbitals, two electrons each: a physical density and Hartree potential
    c = c / torch.sqrt(torch.from_numpy(ko.norms(ham, c.cpu().numpy())).cuda()).reshape(-1, 1, 1, 1)
    c0 = c.cpu().numpy()
    occ_np = np.full(spec.norb, 2.0)
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    K = 2
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    nrm = torch.empty((K, spec.norb), dtype=torch.float64, device="cuda")
    st.propagate_etrs(spec.dt, K, occ, rho, nrm)
    torch.cuda.synchronize()
    ref, dens = ko.etrs_step(ham, c0, spec.dt, occ_np, nsteps=K)
    assert rel_err(st.download().cpu().numpy(), ref) < TOL
    for s in range(K):
        r = rho[s].cpu().numpy()
        assert np.linalg.norm(r - dens[s]) / np.linalg.norm(dens[s]) < TOL
    np.testing.assert_allclose(nrm[-1].cpu().numpy(), ko.norms(ham, ref), rtol=TOL)
    # the density-dependent term is active: ETRS differs from two static half steps
    assert rel_err(ref, ko.taylor4_step(ham, c0, spec.dt / 2, 2 * K)) > 1e-6
    # the system's Hamiltonian is static again after the call
    a = gs.ham_apply(c)
    assert rel_err(a.cpu().numpy(), ko.ham_apply(ham, c0)) < TOL
    st.close()


def test_lda_xc_parity(ks):
    """The local-density exchange-correlation potential pointwise against the
    oracle, on densities over eleven decades (both branches of the
    correlation fit, rs from 0.06 to 300) with zeros, and added to a field."""
    spec, sysm = _case("t24")
    gs = ks.system_from_synth(sysm)
    rng = np.random.default_rng(7100)
    n = 10.0 ** rng.uniform(-8.0, 3.0, size=spec.n)
    n.flat[::7] = 0.0
    rho = torch.from_numpy(n).cuda()
    ref = ko.lda_xc(n)[0]
    np.testing.assert_allclose(gs.lda_xc(rho).cpu().numpy(), ref, rtol=1e-13, atol=0.0)
    base = torch.from_numpy(rng.normal(size=spec.n)).cuda()
    acc = base.clone()
    gs.lda_xc(rho, out=acc, accumulate=True)
    np.testing.assert_allclose(acc.cpu().numpy(), base.cpu().numpy() + ref, rtol=1e-13, atol=1e-15)
    with pytest.raises(ks.KSError) as e:
        gs.set_xc(7)
    assert e.value.status == ks.KS_EINVAL


@pytest.mark.parametrize("name", ["t24", "t48"])
def test_etrs_lda_parity(ks, name):
    """ETRS under V_loc + V_H[n] + v_xc[n] (local-density form) against the
    oracle: orbitals, per-step densities and norms at 1e-12."""
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    gs.set_xc(ks.KS_XC_LDA)
    c = orbitals_device(spec)
    c = c / torch.sqrt(torch.from_numpy(ko.norms(ham, c.cpu().numpy())).cuda()).reshape(-1, 1, 1, 1)
    c0 = c.cpu().numpy()
    occ_np = np.full(spec.norb, 2.0)
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    K = 2
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    nrm = torch.empty((K, spec.norb), dtype=torch.float64, device="cuda")
    st.propagate_etrs(spec.dt, K, occ, rho, nrm)
    torch.cuda.synchronize()
    ref, dens = ko.etrs_step(ham, c0, spec.dt, occ_np, nsteps=K, xc=True)
    assert rel_err(st.download().cpu().numpy(), ref) < TOL
    for s in range(K):
        r = rho[s].cpu().numpy()
        assert np.linalg.norm(r - dens[s]) / np.linalg.norm(dens[s]) < TOL
    np.testing.assert_allclose(nrm[-1].cpu().numpy(), ko.norms(ham, ref), rtol=TOL)
    # the xc term acts: the result differs from ETRS with the Hartree term alone
    assert rel_err(ref, ko.etrs_step(ham, c0, spec.dt, occ_np, nsteps=K)[0]) > 1e-8
    st.close()


# --------------------------------------------------- kick and dipole (NEXT-3)

@pytest.mark.parametrize("name", ["t24", "t32x", "t48"])
def test_kick_and_dipole_parity(ks, name):
    spec, sysm = _case(name)
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    k = (0.05, -0.02, 0.11)
    st.kick(k)
    ref = ko.kick(ham.grid, c0, k)
    got = st.download().cpu().numpy()
    assert rel_err(got, ref) < TOL
    occ_np = np.linspace(0.5, 2.0, spec.norb)
    rho = gs.density(torch.from_numpy(got).cuda(), torch.from_numpy(occ_np).cuda())
    d = gs.dipole(rho).cpu().numpy()
    dr = ko.dipole(ham.grid, ko.density(ham, ref, occ_np))
    assert np.max(np.abs(d - dr)) < TOL * np.max(np.abs(dr))
    st.close()


def test_kicked_etrs_dipole_series(ks):
    # the optical-response workload: kick at t = 0, ETRS steps, dipole per step
    spec, sysm = _case("t24")
    ham = oracle_ham(sysm)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    c = c / torch.sqrt(torch.from_numpy(ko.norms(ham, c.cpu().numpy())).cuda()).reshape(-1, 1, 1, 1)
    c0 = c.cpu().numpy()
    occ_np = np.full(spec.norb, 2.0)
    st = ks.State(gs, spec.norb)
    st.upload(c)
    k = (0.0, 0.0, 0.01)
    st.kick(k)
    K = 3
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate_etrs(spec.dt, K, torch.from_numpy(occ_np).cuda(), rho)
    d = torch.stack([gs.dipole(rho[s]) for s in range(K)]).cpu().numpy()
    _, dens = ko.etrs_step(ham, ko.kick(ham.grid, c0, k), spec.dt, occ_np, nsteps=K)
    dr = np.array([ko.dipole(ham.grid, x) for x in dens])
    assert np.max(np.abs(d - dr)) < TOL * np.max(np.abs(dr))
    st.close()


def test_etrs_local_only_system(ks):
    """ETRS under V_loc + V_H[n] on a system without projectors (density
    passes only, no x-projection pass) against the oracle."""
    print("[case] etrs t24 local only", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    ham = ko.Hamiltonian(g, sysm.vloc)
    gs = ks.System(spec.n, spec.L, spec.ecut, spec.norb)
    gs.set_vloc(torch.from_numpy(sysm.vloc).cuda())
    c = orbitals_device(spec)
    c = c / torch.sqrt(torch.from_numpy(ko.norms(ham, c.cpu().numpy())).cuda()).reshape(-1, 1, 1, 1)
    c0 = c.cpu().numpy()
    occ_np = np.full(spec.norb, 2.0)
    st = ks.State(gs, spec.norb)
    st.upload(c)
    K = 2
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate_etrs(spec.dt, K, torch.from_numpy(occ_np).cuda(), rho)
    ref, dens = ko.etrs_step(ham, c0, spec.dt, occ_np, nsteps=K)
    assert rel_err(st.download().cpu().numpy(), ref) < TOL
    assert np.linalg.norm(rho[-1].cpu().numpy() - dens[-1]) / np.linalg.norm(dens[-1]) < TOL
    st.close()


def test_hartree_and_dipole_full_size(ks):
    """96^3 box (the benchmark's grid): the periodic Hartree potential and the
    dipole of a seeded positive density against the oracle."""
    print("[case] hartree/dipole cfg3_96", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["cfg3_96"]
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    rng = np.random.default_rng(4242)
    n = rng.uniform(0.0, 1.0, spec.n) ** 2
    gs = ks.System(spec.n, spec.L, spec.ecut, 1)
    rho = torch.from_numpy(n).cuda()
    v = gs.hartree(rho).cpu().numpy()
    ref = ko.hartree(g, n)
    assert np.abs(v - ref).max() < TOL * np.abs(ref).max()
    d = gs.dipole(rho).cpu().numpy()
    dr = ko.dipole(g, n)
    assert np.abs(d - dr).max() < TOL * np.abs(dr).max()


def test_kick_full_size_sampled(ks):
    """96^3 grid, 512 resident orbitals: the field kick on every orbital, with
    sampled orbitals recomputed by the oracle one by one."""
    print("[case] kick cfg3_96 sampled", file=sys.stderr, flush=True)
    spec, sysm = _case("cfg3_96")
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    st = ks.State(gs, spec.norb)
    st.upload(c)
    k = (0.0, 0.01, -0.02)
    st.kick(k)
    sample = [0, 301, spec.norb - 1]
    got = st.download()[sample].cpu().numpy()
    ref = ko.kick(ko.Grid(spec.n, spec.L, spec.ecut), c[sample].cpu().numpy(), k)
    assert rel_err(got, ref) < TOL
    st.close()
