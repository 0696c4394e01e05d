"""Serving loop on the GPU: requests that arrive while others run are
admitted as memory frees up, their steps overlap on the device, and each
result is the same alone and in the mix."""
import sys

import numpy as np
import pytest

from paper_2106_03872_amd import serve, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests():
    specs = [
        synth.cubic_spec("s0", 24, 7.92, 8, 2, 3100, nsteps=4),
        synth.cubic_spec("s1", 32, 10.56, 12, 3, 3101, nsteps=4),
        synth.cubic_spec("s2", 24, 7.92, 16, 2, 3102, nsteps=4),
        synth.cubic_spec("s3", 40, 13.2, 8, 4, 3103, nsteps=4),
        synth.cubic_spec("s4", 32, 10.56, 10, 2, 3104, nsteps=4),
        synth.cubic_spec("s5", 24, 7.92, 9, 3, 3105, nsteps=4),
    ]
    arrivals = np.cumsum(np.random.default_rng(9).exponential(0.002, len(specs)))
    return [serve.Request(rid=i, arrival=float(t), spec=s, nsteps=4) for i, (t, s) in enumerate(zip(arrivals, specs))]


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _run(reqs, budget=None, use_graphs=True):
    be = serve.HipBackend(use_graphs=use_graphs)
    be.prepare(reqs)
    if budget is None:
        budget = sum(be.footprint(r) for r in reqs) * 2
    srv = serve.Server(be, budget, keep_orbitals=True)
    done = srv.run(reqs)
    return {r.rid: r for r in done}, srv


def test_serving_alone_equals_mix(gpu):
    print("[case] serving mix", file=sys.stderr, flush=True)
    reqs = _requests()
    be = serve.HipBackend()
    be.prepare(reqs)
    fps = sorted(be.footprint(r) for r in reqs)
    budget = fps[-1] + fps[-2]                       # at most ~2 resident: forces queueing
    mix, srv = _run(_requests(), budget)
    assert len(mix) == len(reqs) and srv.max_used <= budget
    rep = serve.Server.report(list(mix.values()), srv.elapsed, serve.hpsi_per_step)
    print(f"[serve] {rep}", file=sys.stderr)
    for r in _requests():
        print(f"[case] serving alone {r.rid}", file=sys.stderr, flush=True)
        alone, _ = _run([serve.Request(rid=r.rid, arrival=0.0, spec=r.spec, nsteps=r.nsteps)])
        a = alone[r.rid].result["orbitals"]
        m = mix[r.rid].result["orbitals"]
        assert np.array_equal(a, m), np.abs(a - m).max()
        assert abs(alone[r.rid].result["energy"] - mix[r.rid].result["energy"]) == 0.0


def test_graph_replay_equals_direct_steps(gpu):
    print("[case] serving graphs vs direct", file=sys.stderr, flush=True)
    reqs = _requests()[:3]
    g, _ = _run(reqs, use_graphs=True)
    d, _ = _run(_requests()[:3], use_graphs=False)
    for rid in g:
        assert np.array_equal(g[rid].result["orbitals"], d[rid].result["orbitals"])
