"""Reciprocal-space split-BF16 projections (projection mode 1, mixed
precision): the KB projections of Eq. vnl as one product of the packed
orbitals with the table W_Ip(G) = d_Ip (Omega^1/2 / N) sum_j beta_Ip(r_j)
e^{iG.r_j} on the matrix cores.

H psi against the FP64 oracle at the mixed-precision target (1e-5) on small
systems that leave ragged orbital, column and k tails, with 1, 3, 4 and 8
projectors per atom, over several passes, at the 96^3 / 512-orbital /
128-atom and 120^3 / 1024-orbital / 256-atom sizes on sampled orbitals;
propagation (with and without the per-step densities, resident over several
passes) and ETRS with the Hartree and local-density xc potentials against the
oracle;
the band energy after 50 steps against the FP64 path; mode switches, graph
replays, refused cases and a table that does not fit.
"""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth

from gpu_common import oracle_ham, orbitals_device, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_H = 1e-5


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _mode1(ks, sysm, **kw):
    gs = ks.system_from_synth(sysm, precision=ks.KS_MIXED, **kw)
    info = gs.info()
    gs.set_tuning(info["x_group"], info["plane_group"], projection=1)
    assert gs.info()["projection"] == 1
    return gs


@pytest.mark.parametrize("name", ["cfg1_16", "t24", "t40", "t32x", "t60", "t48"])
def test_gproj_ham_apply_vs_oracle(ks, name):
    print(f"[case] gproj H psi {name}", file=sys.stderr, flush=True)
    spec = synth.CONFIGS[name]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    ref = ko.ham_apply(ham, c.cpu().numpy())
    g0 = ks.system_from_synth(sysm, precision=ks.KS_MIXED)
    g1 = _mode1(ks, sysm)
    h0 = g0.ham_apply(c).cpu().numpy()
    h1 = g1.ham_apply(c).cpu().numpy()
    err, d01 = rel_err(h1, ref), rel_err(h1, h0)
    print(f"[gproj] {name}: vs oracle {err:.2e} (real-space mode {rel_err(h0, ref):.2e}), modes differ {d01:.2e}",
          file=sys.stderr)
    assert err < TOL_H
    assert np.all(h1[:, ~ham.grid.chi] == 0)
    g0.close()
    g1.close()


def test_gproj_ragged_orbitals_and_columns(ks):
    """300 orbitals (three row tiles, the last ragged), 21 atoms x 4
    projectors (two column tiles, the second mostly padding), over passes of
    128 and of 300 orbitals."""
    print("[case] gproj ragged tiles", file=sys.stderr, flush=True)
    spec = synth.cubic_spec("gp24", 24, 10.0, 300, 21, 9401)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    ref = ko.ham_apply(ham, c.cpu().numpy())
    for chunk in (0, 128):
        gs = _mode1(ks, sysm, chunk=chunk)
        assert rel_err(gs.ham_apply(c).cpu().numpy(), ref) < TOL_H, chunk
        gs.close()


@pytest.mark.parametrize("np_", [1, 3, 8])
def test_gproj_projector_counts(ks, np_):
    """1, 3 and 8 projectors per atom (8: the four of the generator and the
    same four at half weight)."""
    print(f"[case] gproj {np_} projectors", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t40"]
    sysm = synth.system(spec)
    p = sysm.proj
    beta = p.beta if np_ <= 4 else np.concatenate([p.beta, 0.5 * p.beta], axis=1)
    d = p.d if np_ <= 4 else np.concatenate([p.d, 0.7 * p.d], axis=1)
    beta = np.ascontiguousarray(beta[:, :np_])
    d = np.ascontiguousarray(d[:, :np_])
    off = np.concatenate([[0], np.cumsum(p.npts)])
    atoms = [(p.idx[off[i]:off[i + 1]], beta[off[i]:off[i + 1]]) for i in range(len(p.npts))]
    ham = ko.Hamiltonian(ko.Grid(spec.n, spec.L, spec.ecut), sysm.vloc, atoms, d)
    c = orbitals_device(spec)
    ref = ko.ham_apply(ham, c.cpu().numpy())
    gs = _mode1(ks, sysm)
    gs.set_projectors(p.npts, p.idx, beta, d)          # rebuilt in mode 1
    assert gs.info()["projection"] == 1 and gs.info()["nproj"] == np_
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ref) < TOL_H
    gs.close()


def test_gproj_propagation_vs_oracle(ks):
    """Taylor-4 steps with the per-step densities (the density-fused first
    sub-step keeps the real-space sums, the other three use the product) and
    without (all four, the first on the FP64 state)."""
    print("[case] gproj propagation", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    occ_np = synth.occupations(spec)
    occ = torch.from_numpy(occ_np).cuda()
    gs = _mode1(ks, sysm)
    ref = ko.taylor4_step(ham, c0, spec.dt, spec.nsteps)
    a = c.clone()
    rho = torch.empty((spec.nsteps,) + spec.n, dtype=torch.float64, device="cuda")
    gs.propagate_step(a, spec.dt, spec.nsteps, occ, rho)
    assert rel_err(a.cpu().numpy(), ref) < TOL_H
    rr = ko.density(ham, ref, occ_np)
    assert np.linalg.norm(rho[-1].cpu().numpy() - rr) / np.linalg.norm(rr) < TOL_H
    b = c.clone()
    gs.propagate_step(b, spec.dt, spec.nsteps)
    assert rel_err(b.cpu().numpy(), ref) < TOL_H
    gs.close()


def test_gproj_resident_passes_and_etrs_vs_oracle(ks):
    """Resident states in mode 1: Taylor-4 steps with per-step densities over
    passes of 4 orbitals (10 orbitals: passes of 4, 3, 3), and ETRS under the
    density-dependent Hamiltonian with the local-density xc term, both
    against the oracle."""
    print("[case] gproj resident passes and ETRS", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    occ_np = synth.occupations(spec)
    occ = torch.from_numpy(occ_np).cuda()
    gs = _mode1(ks, sysm, chunk=4)
    st = ks.State(gs, spec.norb)
    st.upload(c)
    K = 3
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate(spec.dt, K, occ, rho)
    ref = c0
    for k in range(K):
        ref = ko.taylor4_step(ham, ref, spec.dt, 1)
        rr = ko.density(ham, ref, occ_np)
        assert np.linalg.norm(rho[k].cpu().numpy() - rr) / np.linalg.norm(rr) < TOL_H, k
    assert rel_err(st.download().cpu().numpy(), ref) < TOL_H
    st.close()
    gs.close()
    # ETRS with V_H and v_xc (t48: 33 orbitals, 6 atoms), orthonormalised start
    spec = synth.CONFIGS["t48"]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    gs = _mode1(ks, sysm)
    gs.set_xc(ks.KS_XC_LDA)
    c = orbitals_device(spec)
    gs.orthonormalize(c)
    c0 = c.cpu().numpy()
    occ_np = np.full(spec.norb, 2.0)
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    rho = torch.empty((K,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate_etrs(spec.dt, K, occ, rho)
    ref, dens = ko.etrs_step(ham, c0, spec.dt, occ_np, nsteps=K, xc=True)
    err = rel_err(st.download().cpu().numpy(), ref)
    print(f"[gproj] ETRS with xc, 3 steps: orbitals {err:.2e}", file=sys.stderr)
    assert err < TOL_H
    assert np.linalg.norm(rho[-1].cpu().numpy() - dens[-1]) / np.linalg.norm(dens[-1]) < TOL_H
    st.close()
    gs.close()


def test_gproj_energy_after_50_steps(ks):
    """Band energy after 50 Taylor-4 steps (dt = 0.05) with the split-BF16
    projections against the FP64 path, on orthonormalised orbitals."""
    print("[case] gproj 50 steps", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    g64 = ks.system_from_synth(sysm)
    gmx = _mode1(ks, sysm)
    c = orbitals_device(spec)
    g64.orthonormalize(c)
    occ = torch.full((spec.norb,), 2.0, dtype=torch.float64, device="cuda")
    a, b = c.clone(), c.clone()
    g64.propagate_step(a, 0.05, 50)
    gmx.propagate_step(b, 0.05, 50)
    _, e64 = g64.reduce(a, occ)
    _, e64m = g64.reduce(b, occ)
    d_e = abs(e64m.item() - e64.item()) / float(occ.sum())
    print(f"[gproj] 50 steps: |dE|/electron {d_e:.2e}, orbitals {rel_err(b.cpu().numpy(), a.cpu().numpy()):.2e}",
          file=sys.stderr)
    assert d_e < 1e-6
    assert rel_err(b.cpu().numpy(), a.cpu().numpy()) < 1e-5
    g64.close()
    gmx.close()


@pytest.mark.parametrize("name,sample", [("cfg3_96", [0, 255, 511]), ("cfg4_120", [0, 1023])])
def test_gproj_full_size_sampled(ks, name, sample):
    """The benchmark sizes: H psi of every orbital in one call in mode 1 (the
    launch the benchmark times), sampled orbitals against the oracle; all
    orbitals against the real-space mode."""
    print(f"[case] gproj full size {name}", file=sys.stderr, flush=True)
    spec = synth.CONFIGS[name]
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    gs = ks.system_from_synth(sysm, precision=ks.KS_MIXED)
    h0 = gs.ham_apply(c)
    gs.set_tuning(gs.info()["x_group"], gs.info()["plane_group"], projection=1)
    h1 = gs.ham_apply(c)
    d = 0.0
    for o in range(0, spec.norb, 128):            # 128 orbitals at a time: no full-size temporary
        a, b = h1[o:o + 128].reshape(-1, spec.npoints), h0[o:o + 128].reshape(-1, spec.npoints)
        d = max(d, (torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)).max().item())
    del h0
    err = rel_err(h1[sample].cpu().numpy(), ko.ham_apply(ham, c[sample].cpu().numpy()))
    print(f"[gproj] {name}: sampled vs oracle {err:.2e}, modes differ {d:.2e}", file=sys.stderr)
    assert err < TOL_H
    assert d < TOL_H
    gs.close()


def test_gproj_modes_graphs_and_refusals(ks):
    print("[case] gproj modes", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t40"]
    sysm = synth.system(spec)
    c = orbitals_device(spec)
    gs = _mode1(ks, sysm)
    h1 = gs.ham_apply(c).clone()
    gs.set_tuning(8, 4, projection=0)
    assert gs.info()["projection"] == 0
    h0 = gs.ham_apply(c).clone()
    assert not torch.equal(h0, h1)
    gs.set_tuning(8, 4, projection=1)
    gs.set_tuning(gs.info()["x_group"], gs.info()["plane_group"])     # projection kept
    assert gs.info()["projection"] == 1
    assert torch.equal(gs.ham_apply(c), h1)                            # table rebuilt: same bits
    t = gs.autotune(spec.norb)
    assert t["projection"] == 1 and gs.info()["projection"] == 1
    # kernel classes
    gs.set_kernel_timing(True)
    gs.ham_apply(c)
    kt = gs.kernel_times()
    assert kt["gproj"][1] == 1 and kt["xproj"][1] == 0
    gs.set_kernel_timing(False)
    # a captured step replays the product (no memset nodes): every replay
    # equals the eager step
    st = ks.State(gs, spec.norb)
    st.upload(c)
    st.propagate(spec.dt, 1)
    want = st.download().clone()
    s = torch.cuda.Stream()
    for _ in range(3):
        st.upload(c)
        torch.cuda.synchronize()
        st.capture(spec.dt, stream=s)
        st.replay(s)
        s.synchronize()
        assert torch.equal(st.download(), want)
        gs.ham_apply(c)                                  # eager work between replays
    st.close()
    # batches form the projections in real space
    st2 = ks.State(gs, spec.norb)
    with pytest.raises(ks.KSError) as e:
        ks.Batch([st2])
    assert e.value.status == ks.KS_EINVAL
    st2.close()
    # FP64 systems and unknown modes are refused
    g64 = ks.system_from_synth(sysm)
    for mode in (1, 2, -2):
        with pytest.raises(ks.KSError) as e:
            g64.set_tuning(8, 4, projection=mode)
        assert e.value.status == ks.KS_EINVAL
    assert g64.info()["projection"] == 0
    with pytest.raises(ks.KSError) as e:
        gs.set_tuning(8, 4, projection=2)
    assert e.value.status == ks.KS_EINVAL
    assert gs.info()["projection"] == 1
    g64.close()
    gs.close()


def test_gproj_table_without_memory_keeps_mode(ks):
    """Switching to mode 1 in a pool without room for the table fails with
    KS_ENOMEM and leaves the system in mode 0 with its results."""
    print("[case] gproj out of memory", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t40"]
    sysm = synth.system(spec)
    c = orbitals_device(spec)
    big = ks.Pool(512 << 20)
    a = ks.system_from_synth(sysm, precision=ks.KS_MIXED, pool=big)
    used = big.usage()[0]
    ref = a.ham_apply(c).clone()
    a.close()
    big.close()
    tight = ks.Pool(used + 4096)
    b = ks.system_from_synth(sysm, precision=ks.KS_MIXED, pool=tight)
    with pytest.raises(ks.KSError) as e:
        b.set_tuning(8, 4, projection=1)
    assert e.value.status == ks.KS_ENOMEM
    assert b.info()["projection"] == 0
    assert torch.equal(b.ham_apply(c), ref)
    b.close()
    tight.close()
