"""Launches at the y extent of a grid (65535): a system of 70000 orbitals
applies H in passes of at most 65535 orbitals, and a batch whose projection
sums need more than 65535 launch rows (one per orbital) is launched in slices
of rows.  Each orbital of the input repeats one of three base orbitals, so
every output must equal its base orbital's output bit for bit, wherever it
sits in a pass or slice; the base orbitals are checked against the FP64
oracle at 1e-12 and the batch against each state stepped alone.
"""
import sys

import numpy as np
import pytest

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth

from gpu_common import oracle_ham, orbitals_device, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRID_Y = 65535


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2106_03872_amd import ks as ksmod
    return ksmod


def _spec(natoms, seed):
    return synth.Spec(name=f"w{natoms}", n=(8, 12, 12), L=(4.8, 7.2, 7.2), ecut=10.0, norb=3, natoms=natoms,
                      seed=seed)


def _tiled(c, norb):
    reps = (norb + c.shape[0] - 1) // c.shape[0]
    return c.repeat(reps, 1, 1, 1)[:norb].contiguous()


def _check_tiled(out, nbase, picks):
    for i in picks:
        assert torch.equal(out[i], out[i % nbase]), i


def test_pass_limit_and_h_over_70000_orbitals(ks):
    norb = 70000
    print(f"[case] H psi over {norb} orbitals, 8x12x12", file=sys.stderr, flush=True)
    spec = _spec(1, 8130)
    sysm = synth.system(spec)
    c = orbitals_device(spec)
    gs = ks.system_from_synth(sysm, max_norb=norb)
    assert gs.info()["chunk"] == GRID_Y                 # the default pass is capped
    with pytest.raises(ks.KSError) as e:
        gs.set_chunk(GRID_Y + 1)
    assert e.value.status == ks.KS_EINVAL
    assert gs.info()["chunk"] == GRID_Y
    g2 = ks.system_from_synth(sysm, max_norb=norb, chunk=100000)
    assert g2.info()["chunk"] == GRID_Y                 # an explicit chunk is capped as well
    g2.close()
    psi = _tiled(c, norb)
    out = gs.ham_apply(psi)
    torch.cuda.synchronize()
    ref = ko.ham_apply(oracle_ham(sysm), c.cpu().numpy())
    assert rel_err(out[:3].cpu().numpy(), ref) < 1e-12
    rng = np.random.default_rng(8131)
    picks = [3, 4, 5, 34998, 34999, 35000, 35001, 65534, 65535, 65536, norb - 1] + list(rng.integers(3, norb, 64))
    _check_tiled(out, 3, picks)
    gs.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_rows_beyond_grid_limit(ks, precision):
    """Two states of 40000 orbitals: 80000 projection-sum rows, launched as
    65535 + 14465; bit-identical to each state stepped alone."""
    norb = 40000
    print(f"[case] batch of 2 x {norb} orbitals, precision {precision}", file=sys.stderr, flush=True)
    specs = [_spec(1, 8140), _spec(2, 8141)]

    def states():
        out = []
        for sp in specs:
            gs = ks.system_from_synth(synth.system(sp), max_norb=norb, precision=precision)
            assert gs.info()["chunk"] == norb
            st = ks.State(gs, norb)
            st.upload(_tiled(orbitals_device(sp), norb))
            out.append((gs, st))
        return out

    alone, batched = states(), states()
    for _, st in alone:
        st.propagate(0.05, 1)
    b = ks.Batch([st for _, st in batched])
    b.propagate(0.05, 1)
    torch.cuda.synchronize()
    for (_, a), (_, x) in zip(alone, batched):
        da, dx = a.download(), x.download()
        assert torch.equal(da, dx)
        _check_tiled(dx, 3, [3, 4, 5, 25534, 25535, 25536, norb - 1])
        del da, dx
    b.close()
    for gs, st in alone + batched:
        st.close()
        gs.close()
    torch.cuda.synchronize()
