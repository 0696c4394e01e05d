"""Serving loop on the GPU: requests that arrive while others run are
admitted as memory frees up, their steps overlap on the device, and each
result is the same alone and in the mix."""
import sys

import numpy as np
import pytest

from paper_2106_03872_amd import serve, synth

pytestmark = pytest.mark.gpu
NSTEPS = 50
torch = pytest.importorskip("torch")


def _requests():
    sizes = [(40, 48, 2), (32, 40, 3), (48, 32, 2), (40, 56, 4), (32, 64, 2), (48, 40, 3),
             (40, 36, 2), (32, 48, 3), (48, 44, 4), (40, 60, 2), (32, 52, 2), (48, 36, 3)]
    specs = [synth.cubic_spec(f"s{i}", n, 0.33 * n, norb, nat, 3100 + i) for i, (n, norb, nat) in enumerate(sizes)]
    arrivals = np.cumsum(np.random.default_rng(9).exponential(0.002, len(specs)))
    return [serve.Request(rid=i, arrival=float(t), spec=s, nsteps=NSTEPS) for i, (t, s) in enumerate(zip(arrivals, specs))]


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _run(reqs, budget=None, use_graphs=True, pool_bytes=None, batched=False, chunk=None):
    cls = serve.BatchedHipBackend if batched else serve.HipBackend
    be = cls(use_graphs=use_graphs, pool_bytes=pool_bytes, chunk=chunk)
    be.prepare(reqs)
    if budget is None:
        budget = sum(be.footprint(r) for r in reqs) * 2
    srv = serve.Server(be, budget, keep_orbitals=True)
    done = srv.run(reqs)
    assert not srv.failed, [r.error for r in srv.failed]
    srv.be = be
    return {r.rid: r for r in done}, srv


def test_serving_alone_equals_mix(gpu):
    """Twelve requests on 4 streams with a budget that keeps at least 8 of
    them resident at once but not all (so the rest queue); systems come from a
    device pool.  Every result is bit-identical to the request run alone."""
    print("[case] serving mix", file=sys.stderr, flush=True)
    reqs = _requests()
    be = serve.HipBackend()
    be.prepare(reqs, pretune=False)
    fps = sorted(be.footprint(r) for r in reqs)
    budget = sum(fps[-9:])                           # any 9 fit, not all 12
    mix, srv = _run(_requests(), budget, pool_bytes=budget + (64 << 20))
    assert len(mix) == len(reqs) and srv.max_used <= budget
    assert srv.max_resident >= 8, srv.max_resident
    rep = serve.Server.report(list(mix.values()), srv.elapsed, serve.hpsi_per_step)
    print(f"[serve] {rep}", file=sys.stderr)
    for r in _requests():
        print(f"[case] serving alone {r.rid}", file=sys.stderr, flush=True)
        alone, _ = _run([serve.Request(rid=r.rid, arrival=0.0, spec=r.spec, nsteps=r.nsteps)])
        a = alone[r.rid].result["orbitals"]
        m = mix[r.rid].result["orbitals"]
        assert np.array_equal(a, m), np.abs(a - m).max()
        assert abs(alone[r.rid].result["energy"] - mix[r.rid].result["energy"]) == 0.0


def test_serving_batched_equals_alone(gpu):
    """The same trace with ragged-batched steps (one launch per kernel for
    the resident requests of a grid): every result bit-identical to the
    request run alone with its own kernels."""
    print("[case] serving batched mix", file=sys.stderr, flush=True)
    reqs = _requests()
    be = serve.HipBackend()
    be.prepare(reqs, pretune=False)
    budget = sum(be.footprint(r) for r in reqs) * 2
    mix, srv = _run(_requests(), budget, use_graphs=False, pool_bytes=budget + (64 << 20), batched=True)
    assert len(mix) == len(reqs)
    assert srv.be.batched_steps < sum(r.nsteps for r in reqs)       # steps were shared
    assert max(srv.be.batch_sizes) >= 2
    for r in _requests():
        print(f"[case] serving batched alone {r.rid}", file=sys.stderr, flush=True)
        alone, _ = _run([serve.Request(rid=r.rid, arrival=0.0, spec=r.spec, nsteps=r.nsteps)])
        assert np.array_equal(alone[r.rid].result["orbitals"], mix[r.rid].result["orbitals"])
        assert alone[r.rid].result["energy"] == mix[r.rid].result["energy"]


def test_serving_batched_passes_equal_alone(gpu):
    """Requests whose systems hold a pass of at most 16 orbitals (their
    batched steps run in passes; every system's workspace is a quarter of the
    default or less): results bit-identical to each request alone with its own
    default one-pass system, and the footprints smaller."""
    print("[case] serving batched passes", file=sys.stderr, flush=True)
    reqs = _requests()[:6]
    be = serve.BatchedHipBackend(chunk=16)
    be.prepare(reqs, pretune=False)
    one = serve.BatchedHipBackend()
    one.prepare(reqs, pretune=False)
    assert all(be.footprint(r) < one.footprint(r) for r in reqs)
    budget = sum(be.footprint(r) for r in reqs) * 2
    mix, srv = _run(_requests()[:6], budget, use_graphs=False, pool_bytes=budget + (64 << 20), batched=True,
                    chunk=16)
    assert max(srv.be.batch_sizes) >= 2
    for r in _requests()[:6]:
        alone, _ = _run([serve.Request(rid=r.rid, arrival=0.0, spec=r.spec, nsteps=r.nsteps)])
        assert np.array_equal(alone[r.rid].result["orbitals"], mix[r.rid].result["orbitals"])
        assert alone[r.rid].result["energy"] == mix[r.rid].result["energy"]


def test_graph_replay_equals_direct_steps(gpu):
    print("[case] serving graphs vs direct", file=sys.stderr, flush=True)
    reqs = _requests()[:3]
    g, _ = _run(reqs, use_graphs=True)
    d, _ = _run(_requests()[:3], use_graphs=False)
    for rid in g:
        assert np.array_equal(g[rid].result["orbitals"], d[rid].result["orbitals"])


def test_pooled_system_equals_plain_and_releases(gpu):
    from paper_2106_03872_amd import ks
    print("[case] pooled system", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    sysm = synth.system(spec)
    pool = ks.Pool(256 << 20)
    a = ks.system_from_synth(sysm)
    b = ks.system_from_synth(sysm, pool=pool)
    c = torch.from_numpy(synth.orbitals_box(spec)).cuda()
    assert torch.equal(a.ham_apply(c), b.ham_apply(c))
    st = ks.State(b, spec.norb)
    st.upload(c)
    st.propagate(0.05, 2)
    used, peak, _ = pool.usage()
    assert 0 < used <= peak <= 256 << 20
    st.close()
    b.close()
    used, _, largest = pool.usage()
    assert used == 0 and largest == pool.nbytes       # every range returned and merged
    with pytest.raises(ks.KSError) as e:              # an exhausted pool fails cleanly
        ks.System((64, 64, 64), (20.0,) * 3, 10.0, 512, pool=ks.Pool(1 << 20))
    assert e.value.status == ks.KS_ENOMEM
    a.close()
    pool.close()


def test_replay_after_retune_is_rejected(gpu):
    from paper_2106_03872_amd import ks
    print("[case] stale graph", file=sys.stderr, flush=True)
    spec = synth.CONFIGS["t24"]
    gs = ks.system_from_synth(synth.system(spec))
    st = ks.State(gs, spec.norb)
    st.upload(torch.from_numpy(synth.orbitals_box(spec)).cuda())
    s = torch.cuda.Stream()
    st.capture(0.05, stream=s)
    st.replay(s)
    gs.set_tuning(4, 2)                               # launch shapes changed: the graph is stale
    with pytest.raises(ks.KSError) as e:
        st.replay(s)
    assert e.value.status == ks.KS_EINVAL
    st.capture(0.05, stream=s)                        # captured again: replays work
    st.replay(s)
    torch.cuda.synchronize()
    st.close()
    gs.close()
