"""x-pass launch shapes of the 96- and 120-point x-pencil passes (16 pencils
x 192 threads next to the default 32 x 256; at 96 both tiles also with the
x-transform factorised 8 x 12 instead of 12 x 8): H psi in every shape
against the FP64 oracle at 1e-12 (1e-5 mixed), a resident propagation with
the fused density at 1e-12, switching shapes back and forth (the per-tile
projector tables are rebuilt from the stored inputs), the autotuner's choice,
batches, and the errors.  The grids cover the band-limited (HB) and full x-synthesis inputs.
With n1 = n2 every accepted plane holds a multiple of 16 pencils, so the
16-pencil tiles are never ragged.
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

# (n, L, natoms): x_half (|m0| < n0/4 on the sphere) holds for the first and
# third, not for the second and fourth (E_cut = 10 Ha, |G| < 4.47)
GRIDS = [
    ((96, 40, 40), (30.0, 13.2, 13.2), 6),
    ((96, 40, 40), (40.0, 13.2, 13.2), 6),
    ((120, 48, 48), (36.0, 16.0, 16.0), 8),
    ((120, 24, 24), (48.0, 8.0, 8.0), 4),
]
IDS = [f"{g[0][0]}x{g[0][1]}-L{g[1][0]:g}" for g in GRIDS]


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _spec(n, L, natoms, norb=4):
    name = "s" + "x".join(map(str, n)) + f"L{L[0]:g}"
    return synth.Spec(name=name, n=n, L=L, ecut=10.0, norb=norb, natoms=natoms, seed=9100 + n[0] + n[1] + int(L[0]))


@pytest.mark.parametrize("n,L,natoms", GRIDS, ids=IDS)
def test_shapes_vs_oracle(ks, n, L, natoms):
    print(f"[case] shapes {n} L {L}", file=sys.stderr, flush=True)
    spec = _spec(n, L, natoms)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    ref = ko.ham_apply(ham, c0)
    gs = ks.system_from_synth(sysm)
    assert gs.info()["x_half"] == int(L[0] * np.sqrt(20.0) / (2 * np.pi) < n[0] / 4 - 1)
    out = {}
    shapes = (0, 1, 2, 3, 0, 2, 1, 3) if n[0] == 96 else (0, 1, 0, 1)   # tables rebuilt on every switch
    for shape in shapes:
        gs.set_tuning(8, 4, x_shape=shape)
        info = gs.info()
        assert (info["x_shape"], info["x_tile"], info["x_threads"]) == \
            ((0, 32, 256), (1, 16, 192), (2, 32, 256), (3, 16, 192))[shape]
        got = gs.ham_apply(c).clone()
        assert rel_err(got.cpu().numpy(), ref) < TOL, shape
        assert np.all(got.cpu().numpy()[:, ~ham.grid.chi] == 0)
        if shape in out:
            assert torch.equal(out[shape], got)      # same shape, same tables: bit-identical
        out[shape] = got
    gm = ks.system_from_synth(sysm, precision=ks.KS_MIXED)
    for shape in shapes[:len(set(shapes))]:
        gm.set_tuning(8, 4, x_shape=shape)
        assert rel_err(gm.ham_apply(c).cpu().numpy(), ref) < TOL_MIXED, shape
    gm.close()
    gs.close()


@pytest.mark.parametrize("shape", [1, 2])
@pytest.mark.parametrize("n,L,natoms", GRIDS[::3], ids=IDS[::3])
def test_shape1_propagation_with_fused_density(ks, n, L, natoms, shape):
    if shape == 2 and n[0] != 96:
        pytest.skip("the second radix plan is built for n0 = 96 only")
    print(f"[case] shape-{shape} propagation {n} L {L}", file=sys.stderr, flush=True)
    spec = _spec(n, L, natoms, norb=3)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    c0 = c.cpu().numpy()
    gs = ks.system_from_synth(sysm)
    gs.set_tuning(8, 4, x_shape=shape)
    occ_np = np.array([2.0, 1.0, 0.5])
    occ = torch.from_numpy(occ_np).cuda()
    st = ks.State(gs, spec.norb)
    st.upload(c)
    rho = torch.empty((3,) + spec.n, dtype=torch.float64, device="cuda")
    st.propagate(spec.dt, 3, occ, rho)
    r = c0
    for s in range(3):
        r = ko.taylor4_step(ham, r, spec.dt, 1)
        rr = ko.density(ham, r, occ_np)
        assert np.linalg.norm(rho[s].cpu().numpy() - rr) / np.linalg.norm(rr) < TOL, s
    assert rel_err(st.download().cpu().numpy(), r) < TOL
    st.close()
    gs.close()


def test_projectors_set_after_shape_change(ks):
    """New projectors on a system already in shape 1 are tiled for shape 1."""
    print("[case] projectors after shape change", file=sys.stderr, flush=True)
    n, L, natoms = GRIDS[0]
    spec = _spec(n, L, natoms)
    sysm = synth.system(spec)
    ham = oracle_ham(sysm)
    c = orbitals_device(spec)
    gs = ks.system_from_synth(synth.system(_spec(n, L, 2)))   # other projectors and potential first
    gs.set_tuning(8, 4, x_shape=1)
    p = sysm.proj
    gs.set_vloc(torch.from_numpy(sysm.vloc).cuda())
    gs.set_projectors(p.npts, p.idx, p.beta, p.d)
    assert gs.info()["x_shape"] == 1
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ko.ham_apply(ham, c.cpu().numpy())) < TOL
    gs.close()


def test_autotune_chooses_a_shape(ks):
    print("[case] autotune shapes", file=sys.stderr, flush=True)
    n, L, natoms = GRIDS[2]
    spec = _spec(n, L, natoms, norb=16)
    sysm = synth.system(spec)
    gs = ks.system_from_synth(sysm)
    c = orbitals_device(spec)
    t = gs.autotune(spec.norb)
    assert t["x_shape"] in (0, 1) and not t["from_cache"]
    assert gs.info()["x_shape"] == t["x_shape"]
    ref = ko.ham_apply(oracle_ham(sysm), c.cpu().numpy())
    assert rel_err(gs.ham_apply(c).cpu().numpy(), ref) < TOL
    g2 = ks.system_from_synth(sysm)
    t2 = g2.autotune(spec.norb)
    assert t2["from_cache"] and t2["x_shape"] == t["x_shape"] and g2.info()["x_shape"] == t["x_shape"]
    # grids without a second shape keep shape 0
    s48 = synth.cubic_spec("a48", 48, 15.84, 4, 2, 9300)
    g3 = ks.system_from_synth(synth.system(s48))
    assert g3.autotune(4)["x_shape"] == 0
    for g in (gs, g2, g3):
        g.close()


def test_shape_errors_and_batches(ks):
    print("[case] shape errors and batches", file=sys.stderr, flush=True)
    s48 = synth.cubic_spec("e48", 48, 15.84, 4, 2, 9310)
    g48 = ks.system_from_synth(synth.system(s48))
    with pytest.raises(ks.KSError) as e:
        g48.set_tuning(8, 4, x_shape=1)               # no second shape at 48
    assert e.value.status == ks.KS_EINVAL
    with pytest.raises(ks.KSError) as e:
        g48.set_tuning(8, 4, x_shape=2)
    assert e.value.status == ks.KS_EINVAL
    assert g48.info()["x_shape"] == 0
    g48.close()
    g120 = ks.system_from_synth(synth.system(_spec(*GRIDS[2])))      # no second radix plan at 120
    for shape in (2, 3):
        with pytest.raises(ks.KSError) as e:
            g120.set_tuning(8, 4, x_shape=shape)
        assert e.value.status == ks.KS_EINVAL
    g120.close()
    # batches: one launch per kernel needs one shape; results equal the states stepped alone
    n, L, _ = GRIDS[0]
    specs = [_spec(n, L, na, norb=nb) for na, nb in ((3, 5), (5, 2), (1, 7))]
    def states(shape):
        out = []
        for sp in specs:
            gs = ks.system_from_synth(synth.system(sp))
            gs.set_tuning(8, 4, x_shape=shape)
            st = ks.State(gs, sp.norb)
            st.upload(orbitals_device(sp))
            out.append((gs, st))
        return out
    alone, batched = states(1), states(1)
    for _, st in alone:
        st.propagate(0.05, 2)
    b = ks.Batch([st for _, st in batched])
    b.propagate(0.05, 2)
    torch.cuda.synchronize()
    for (_, a), (_, c) in zip(alone, batched):
        assert torch.equal(a.download(), c.download())
    batched[1][0].set_tuning(8, 4, x_shape=0)         # a system changed shape: the batch is stale
    with pytest.raises(ks.KSError) as e:
        b.propagate(0.05, 1)
    assert e.value.status == ks.KS_EINVAL
    b.close()
    with pytest.raises(ks.KSError) as e:              # mixed shapes
        ks.Batch([st for _, st in batched])
    assert e.value.status == ks.KS_EINVAL
    torch.cuda.synchronize()


def test_shape_switch_without_memory_keeps_the_system(ks):
    """A shape switch builds the new tables before it frees the old ones: in
    a pool with no room for them it fails with KS_ENOMEM and the system keeps
    its shape, tables and results."""
    print("[case] shape switch out of memory", file=sys.stderr, flush=True)
    n, L, natoms = GRIDS[0]
    spec = _spec(n, L, natoms)
    sysm = synth.system(spec)
    c = orbitals_device(spec)
    big = ks.Pool(512 << 20)
    a = ks.system_from_synth(sysm, pool=big)
    used = big.usage()[0]
    ref = a.ham_apply(c).clone()
    a.close()
    big.close()
    tight = ks.Pool(used + 4096)
    b = ks.system_from_synth(sysm, pool=tight)
    with pytest.raises(ks.KSError) as e:
        b.set_tuning(8, 4, x_shape=1)
    assert e.value.status == ks.KS_ENOMEM
    assert b.info()["x_shape"] == 0
    assert torch.equal(b.ham_apply(c), ref)
    b.close()
    tight.close()
