"""Benchmark of the Kohn-Sham hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3_96]

One step = one pass of the whole hot path over the orbital batch: a Taylor-4
propagation step (4 H psi per orbital: FFT passes, local potential, KB
non-local, kinetic, Taylor accumulation), the density sum_i f_i |psi_i|^2 of
the new orbitals and their norms.  The K timed steps are one propagation call
that returns the K densities and norms.  Default workload: 96^3 grid, L = 30 bohr,
512 orbitals (f = 2), 128 atoms x 4 KB projectors, dt = 0.05, FP64.  Inputs
are seeded synthetic data resident in HBM before timing starts.

Prints ONE JSON line with the throughput (orbital.H psi applications/s), the
roofline of the dominant kernel (HIP events on the library's stream over the
timed region) and a CPU baseline (the FP64 oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
METRIC = "orbital·Hψ applications/s at 96³ grid vs roofline; serving p50/p99 step latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(info, spec, kernel, S=16):
    """Algorithmic HBM bytes of one kernel class: (per orbital, per launch).

    Per orbital: each kernel's own inputs read once and outputs written once
    (S bytes per complex element); per launch: data shared by all orbitals of
    the launch (potential, projector tables) read once."""
    N = int(np.prod(spec.n))
    npl = spec.n[1] * spec.n[2]
    box_planes = info["nplanes"] * npl * S
    npw = info["npw"] * S
    beta = info["npoints"] * info["nproj"] * 8 + info["nruns"] * 3 * 4
    parts = info["nslots"] * info["nproj"] * S
    if kernel == "plane_inv":
        return npw + box_planes, 0
    if kernel == "xproj":
        return box_planes + parts, beta
    if kernel == "proj_reduce":
        return parts + info["natoms"] * info["nproj"] * S, 0
    if kernel == "xapply":
        return 2 * box_planes, N * 8 + beta
    if kernel == "plane_fwd":       # Taylor mode: U, w_in, acc read+write, w_out for 3 of 4 powers
        return box_planes + npw + 2 * npw + 0.75 * npw, 0
    if kernel == "xdens":
        return box_planes, 2 * N * 8
    if kernel == "pack":
        return 2 * npw, 0
    if kernel == "unpack":
        return npw + N * S, 0
    if kernel == "dots":
        return npw, 0
    if kernel == "gproj":           # packed input, DP out; the split table (hi + lo BF16) once per launch
        return npw + info["natoms"] * info["nproj"] * 16, gproj_table_bytes(info)
    return 0, 0


def gproj_shape(info):
    """(columns, padded k) of the reciprocal-space projection product."""
    P = info["natoms"] * info["nproj"]
    return 2 * (-(-P // 64) * 64), -(-2 * info["npw"] // 32) * 32


def gproj_table_bytes(info):
    ncol, kpad = gproj_shape(info)
    return ncol * kpad * 4


def gproj_summary(info, spec, kt):
    """The split-BF16 projection product per launch: time, MFMA rate (three
    BF16 products per real multiply-add) against the 2.5 PFLOP/s dense BF16
    peak, and algorithmic HBM bytes (input, table, DP) per second."""
    ms, n = kt.get("gproj", (0.0, 0))
    if n == 0:
        return None
    nb = orbitals_per_pass(spec, info)
    ncol, kpad = gproj_shape(info)
    us = 1e3 * ms / n
    flop = 6.0 * nb * ncol * kpad
    po, pl = alg_bytes(info, spec, "gproj", S=8)
    byt = po * nb + pl
    return {"avg_us": round(us, 2), "launches": n, "orbitals": nb, "columns": ncol, "k": kpad,
            "mfma_tflops": round(flop / (us * 1e-6) / 1e12, 1), "mfma_peak_tflops": 2500.0,
            "mfma_frac": round(flop / (us * 1e-6) / 2.5e15, 4), "alg_bytes": int(byt),
            "alg_GBs": round(byt / (us * 1e-6) / 1e9, 1)}


def plain_copy_bandwidth(reps=5):
    """Read + write GB/s of a plain 1 GiB device copy (torch), timed with
    events after one untimed copy; its dispatches also calibrate the HBM
    traffic counters."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2.0 * (1 << 30) / (ms * 1e-3) / 1e9, 1)


def measured_traffic(kernel, workload, orbitals_per_pass, info):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE runs, scaled by the copy-kernel
    calibration; written by `python -m paper_2106_03872_amd.profiling
    traffic`), or None when the summary is missing, was taken on other
    sources or another pass size, or on another x-tile shape."""
    from paper_2106_03872_amd.profiling import csrc_fingerprint
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_fp64.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("csrc_sha256") != csrc_fingerprint() or rec.get("orbitals_per_pass") != orbitals_per_pass:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    shape = "XShapeAlt" if info.get("x_shape", 0) >= 2 else "XShape"   # shapes 2, 3: second radix plan
    if kernel.startswith("x") and f"{shape}<{info['x_tile']}, {info['x_threads']}>" not in k.get("kernel", ""):
        return None
    return k["bytes_per_launch"]


def cpu_baseline(spec, sysm, norb_sample=128):
    """The FP64 oracle, unchanged, on a bounded sample of the workload:
    norb_sample orbitals through one Taylor-4 step and the density."""
    from oracle import ks_oracle as ko
    from paper_2106_03872_amd import synth
    g = ko.Grid(spec.n, spec.L, spec.ecut)
    ham = ko.Hamiltonian(g, sysm.vloc, [sysm.proj.atom(i) for i in range(spec.natoms)], sysm.proj.d)
    c = synth.orbitals_box(spec, norb_sample)
    t0 = time.perf_counter()
    c1 = ko.taylor4_step(ham, c, spec.dt, 1)
    ko.density(ham, c1, np.full(norb_sample, spec.occ))
    dt = time.perf_counter() - t0
    # the same on one thread, over a smaller slice
    n1 = max(1, norb_sample // 16)
    workers = ko.WORKERS
    ko.WORKERS = 1
    try:
        t0 = time.perf_counter()
        c1 = ko.taylor4_step(ham, c[:n1], spec.dt, 1)
        ko.density(ham, c1, np.full(n1, spec.occ))
        dt1 = time.perf_counter() - t0
    finally:
        ko.WORKERS = workers
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": 4 * norb_sample / dt, "unit": "orbital·Hψ/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{norb_sample} of {spec.norb} orbitals, one Taylor-4 step (4 H psi each) + density, "
                      f"{spec.n[0]}^3 grid, {spec.natoms} atoms; {dt:.1f} s",
            "one_thread": {"value": 4 * n1 / dt1, "sample": f"{n1} orbitals, same step; {dt1:.1f} s"},
            "cpu_model": model}


def setup_workload(spec, precision, chunk=0):
    """System + orthonormalised resident orbitals of one workload."""
    import torch

    from paper_2106_03872_amd import ks, synth
    sysm = synth.system(spec)
    dev = torch.device("cuda:0")
    gs = ks.system_from_synth(sysm, precision=precision)
    if chunk:
        gs.set_chunk(chunk)
    sel, vals = synth.orbital_values(spec)
    c = torch.zeros((spec.norb, spec.npoints), dtype=torch.complex128, device=dev)
    c[:, torch.from_numpy(sel).to(dev)] = torch.from_numpy(vals).to(dev)
    c = c.reshape((spec.norb,) + tuple(spec.n))
    del vals
    torch.cuda.synchronize()
    gs.set_kernel_timing(True)
    t0 = time.perf_counter()
    gs.orthonormalize(c)                 # Cholesky of the overlap (set-up)
    torch.cuda.synchronize()
    ortho_ms = (time.perf_counter() - t0) * 1e3
    gemm_ms = gs.kernel_times()["gemm"][0]
    gs.set_kernel_timing(False)
    # overlap (tiles on and below the diagonal) and triangular apply: about
    # n^2 npw complex MACs together, 8 real flops each
    flop = 8.0 * spec.norb ** 2 * gs.npw
    gs.ortho = {"ms": round(ortho_ms, 3), "gemm_ms": round(gemm_ms, 3),
                "gemm_tflops": round(flop / (gemm_ms * 1e-3) / 1e12, 2) if gemm_ms > 0 else None,
                "gemm_peak_tflops": 78.6, "orbitals": spec.norb}
    state = ks.State(gs, spec.norb)
    state.upload(c)
    del c
    gs.tuning = gs.autotune(spec.norb)   # launch schedule (x-tile shape, orbital-group caps), timed on the device
    torch.cuda.synchronize()
    return sysm, gs, state


def run_steps(spec, gs, state, steps, warmup, timing=True):
    """Warm up, then time `steps` steps in one propagation call: Taylor-4,
    the density and the orbital norms after every step."""
    import torch
    occ = torch.full((spec.norb,), float(spec.occ), dtype=torch.float64, device="cuda")
    rho = torch.empty((max(steps, warmup, 1),) + tuple(spec.n), dtype=torch.float64, device="cuda")
    nrm = torch.empty((max(steps, warmup, 1), spec.norb), dtype=torch.float64, device="cuda")
    norms0, e0 = state.reduce(occ)
    if warmup:
        state.propagate(spec.dt, warmup, occ, rho, nrm)
    torch.cuda.synchronize()
    if timing:
        gs.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.propagate(spec.dt, steps, occ, rho, nrm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = gs.kernel_times() if timing else {}
    if timing:
        gs.set_kernel_timing(False)
    norms1, e1 = state.reduce(occ)
    nel = float(occ.sum().item())
    phys = {"norm_drift_max": float(torch.max(torch.abs(norms1 / norms0 - 1.0)).item()),
            "band_energy_per_electron_start": e0.item() / nel, "band_energy_per_electron_end": e1.item() / nel,
            "steps_total": warmup + steps}
    return (t1 - t0) * 1e3 / steps, kt, phys, rho


def orbitals_per_pass(spec, info):
    passes = -(-spec.norb // info["chunk"])
    return -(-spec.norb // passes)          # balanced passes


def kernel_table(info, spec, ktimes, steps, ms_step):
    """Per kernel class: time, launches, and achieved algorithmic GB/s (every
    launch of the timed call covers one pass of orbitals_per_pass orbitals)."""
    per_pass = orbitals_per_pass(spec, info)
    es = 16 if info["precision"] == 0 else 8
    kernels = {}
    for name, (ms, n) in ktimes.items():
        if n == 0:
            continue
        po, pl = alg_bytes(info, spec, name, S=es)
        byt = (po * per_pass + pl) * n
        kernels[name] = {"ms_total": round(ms, 3), "launches": n, "avg_us": round(1e3 * ms / n, 2),
                         "share": round(ms / (ms_step * steps), 4), "alg_GBs": round(byt / (ms * 1e-3) / 1e9, 1)}
    return kernels


def run_etrs(spec, gs, state, steps):
    """ETRS steps under the density-dependent Hamiltonian (V_loc + periodic
    Hartree + local-density exchange-correlation): 8 H psi, 2 densities, 2
    Poisson solves and 2 xc evaluations per step."""
    import torch
    from paper_2106_03872_amd import ks
    gs.set_xc(ks.KS_XC_LDA)
    occ = torch.full((spec.norb,), float(spec.occ), dtype=torch.float64, device="cuda")
    rho = torch.empty((steps,) + tuple(spec.n), dtype=torch.float64, device="cuda")
    nrm = torch.empty((steps, spec.norb), dtype=torch.float64, device="cuda")
    state.propagate_etrs(spec.dt, 1, occ)                      # warm-up (allocates the predictor)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.propagate_etrs(spec.dt, steps, occ, rho, nrm)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # one Poisson solve (5 full-box FFT launches) timed on its own
    v = torch.empty(tuple(spec.n), dtype=torch.float64, device="cuda")
    gs.hartree(rho[-1], add_vloc=True, out=v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        gs.hartree(rho[-1], add_vloc=True, out=v)
    torch.cuda.synchronize()
    hms = (time.perf_counter() - t0) * 1e3 / 20
    gs.set_xc(ks.KS_XC_NONE)
    return {"ms_per_step": round(ms, 3), "hpsi_per_step": 8 * spec.norb,
            "orbital_hpsi_per_s": round(8 * spec.norb / (ms * 1e-3), 1), "hartree_ms": round(hms, 4),
            "electrons": float(occ.sum().item()), "norm_drift_max": float((nrm[-1] - 1.0).abs().max().item()),
            "steps": steps, "density_dependent": "V_loc + periodic Hartree + LDA xc (Slater, Perdew-Zunger)"}


def run_ground(spec, gs, state, iters):
    """Steepest-descent eigensolver iterations on the resident orbitals: per
    iteration 2 H psi per orbital, the Rayleigh-Ritz product, two rotation
    products, the Jacobi subspace eigenproblem, the residual/preconditioner
    and line-minimisation kernels and the Cholesky orthonormalisation."""
    import torch
    state.eigensolve(1)                                    # warm-up (allocates the work blocks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, resid = state.eigensolve(iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / iters
    gs.set_kernel_timing(True)                             # per-class breakdown in a second timed run
    state.eigensolve(iters)
    torch.cuda.synchronize()
    kt = gs.kernel_times()
    gs.set_kernel_timing(False)
    npw, n = gs.npw, spec.norb
    # complex MACs of the dense products per iteration: Rayleigh-Ritz n^2 npw,
    # two rotations 2 n^2 npw, overlap (lower half) n^2 npw / 2, triangular
    # apply n^2 npw / 2; 8 real flops per complex MAC
    gemm_flop = 8.0 * n * n * npw * 4.0
    parts = {k: round(v[0] / iters, 3) for k, v in kt.items() if v[1] > 0}
    launches = {k: v[1] // iters for k, v in kt.items() if v[1] > 0}
    gemm_ms = kt["gemm"][0] / iters
    return {"ms_per_iteration": round(ms, 3), "iterations": iters, "orbitals": n,
            "ms_per_iteration_by_class": parts, "launches_per_iteration": launches,
            "hpsi_ms_per_iteration": round(sum(parts.get(k, 0.0) for k in
                                               ("plane_inv", "xproj", "proj_reduce", "xapply", "plane_fwd")), 3),
            "gemm_tflops": round(gemm_flop / (gemm_ms * 1e-3) / 1e12, 2) if gemm_ms > 0 else None,
            "gemm_peak_tflops": 78.6,
            "ritz_sum_first_last": [float(eig[0].sum().item()), float(eig[-1].sum().item())],
            "residual_max_last": float(resid[-1].max().item())}


def run_mixed_large(steps, log):
    """The mixed-precision configuration's larger system (120^3 grid, 1024
    orbitals, 256 atoms): FP64 and mixed steps from the same orthonormalised
    start, the speedup and the orbital error of the mixed path."""
    from paper_2106_03872_amd import ks, synth
    spec = synth.CONFIGS["cfg4_120"]
    sample = list(range(0, spec.norb, 64))
    res, psi = {}, {}
    for name, prec in (("fp64", ks.KS_FP64), ("mixed", ks.KS_MIXED)):
        _, g, st = setup_workload(spec, prec)
        # mixed: the split-BF16 reciprocal-space projections (1), then the
        # real-space sums (0) from the same start
        projs = (1, 0) if prec == ks.KS_MIXED else (0,)
        start = st.download() if len(projs) > 1 else None
        for proj in projs:
            key = name if proj == projs[0] else f"{name}_projection_0"
            if prec == ks.KS_MIXED:
                g.set_tuning(g.tuning["x_group"], g.tuning["plane_group"], projection=proj)
                st.upload(start)
            ms, kt, phys, _ = run_steps(spec, g, st, steps, 1)
            psi[key] = st.download()[sample].clone()
            res[key] = {"ms_per_step": round(ms, 3), "value": round(4 * spec.norb / (ms * 1e-3), 1),
                        "chunk": g.info()["chunk"], "norm_drift_max": phys["norm_drift_max"], "tuning": g.tuning,
                        "projection": proj, "kernels": kernel_table(g.info(), spec, kt, steps, ms)}
            if proj == 1:
                res[key]["gproj"] = gproj_summary(g.info(), spec, kt)
            log(f"[bench] 120^3 / {spec.norb} orbitals {key}: {ms:.2f} ms/step, {res[key]['value']:.0f} "
                f"orbital.Hpsi/s, tuning {g.tuning}")
        del start
        st.close()
        g.close()
    b = psi["fp64"]
    err = {}
    for key in ("mixed", "mixed_projection_0"):
        d = (psi[key] - b).reshape(len(sample), -1).norm(dim=1) / b.reshape(len(sample), -1).norm(dim=1)
        err[key] = float(d.max().item())
    res["mixed_projection_0"]["orbital_rel_err_vs_fp64_max"] = err["mixed_projection_0"]
    res["mixed_projection_0"]["speedup_vs_fp64"] = round(
        res["fp64"]["ms_per_step"] / res["mixed_projection_0"]["ms_per_step"], 3)
    res["mixed"]["projection_0"] = res.pop("mixed_projection_0")
    return {"workload": f"{spec.n[0]}^3, {spec.norb} orbitals, {spec.natoms} atoms", "steps": 1 + steps,
            "fp64": res["fp64"], "mixed": res["mixed"],
            "speedup_vs_fp64": round(res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"], 3),
            "orbital_rel_err_vs_fp64_max": err["mixed"], "orbitals_compared": len(sample)}


def run_serving(nreq, nsteps, budget_gb, log, batched=True, max_active=256, lockstep=True, chunk=None):
    """The serving trace: Poisson arrivals of small systems, continuous
    batching under an HBM budget.  batched: the resident requests of a grid
    are stepped by shared launches (ks_batch); otherwise each request replays
    its own captured step.  lockstep: global rounds (every resident request
    advances once per round).  Systems live in a device pool of 1.25 times
    the budget (fragmentation slack); launch schedules are tuned per grid
    bucket before the trace.  chunk: orbitals per pass of each request's
    system (None: one pass)."""
    from paper_2106_03872_amd import serve, synth
    trace = synth.serving_trace(nreq, 200.0, 2000)
    reqs = [serve.Request(rid=i, arrival=t, spec=sp, nsteps=nsteps) for i, (t, sp) in enumerate(trace)]
    import torch
    torch.cuda.empty_cache()                    # the earlier sections' cached blocks
    budget = int(budget_gb * 2 ** 30)
    pool = int(1.25 * budget) + (256 << 20)     # slack for the pool's fragmentation
    if batched:
        be = serve.BatchedHipBackend(pool_bytes=pool, lockstep=lockstep, chunk=chunk)
    else:
        be = serve.HipBackend(pool_bytes=pool, chunk=chunk)
    log(f"[bench] serving ({'batched launches' if batched else 'one graph per request'}): preparing {nreq} requests")
    be.prepare(reqs)
    srv = serve.Server(be, budget, max_active=max_active)
    done = srv.run(reqs)
    rep = serve.Server.report(done, srv.elapsed, serve.hpsi_per_step)
    rep.update({"mode": ("batched launches per grid" + (", global rounds" if lockstep else "")) if batched
                else "captured graph per request", "max_active": max_active,
                "hbm_budget_GiB": budget_gb, "max_reserved_GiB": round(srv.max_used / 2 ** 30, 2),
                "pool_peak_GiB": round(be.pool.usage()[1] / 2 ** 30, 2) if be.pool is not None else None,
                "max_resident_requests": srv.max_resident, "failed": len(srv.failed), "requeued": srv.requeued,
                "pretune_s": round(be.tuning_s, 2), "orbitals_per_pass": chunk,
                "precision": "mixed", "steps_per_request": nsteps, "arrivals": "Poisson, mean 200/s",
                "drift_max": max(float(abs(r.result["norms"] - 1.0).max()) for r in done)})
    if batched:
        sz = np.asarray(be.batch_sizes, float)
        rep.update({"batched_launch_steps": be.batched_steps, "requests_per_batched_step_mean": round(float(sz.mean()), 2),
                    "requests_per_batched_step_max": int(sz.max())})
    if be.pool is not None:
        be.pool.close()
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3_96")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-etrs", action="store_true")
    ap.add_argument("--etrs-steps", type=int, default=3)
    ap.add_argument("--no-ground", action="store_true")
    ap.add_argument("--no-mixed-120", action="store_true")
    ap.add_argument("--ground-iters", type=int, default=2)
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-steps", type=int, default=50)
    ap.add_argument("--serving-budget-gb", type=float, default=32.0)
    ap.add_argument("--serving-pass", type=int, default=64,
                    help="orbitals per pass of each request's system under the capped budget (0: one pass; "
                         "the one-pass run is then the only capped run)")
    ap.add_argument("--serving-full-budget-gb", type=float, default=160.0,
                    help="also run the trace with a budget the whole trace fits in (0: skip)")
    ap.add_argument("--serving-compare", action="store_true",
                    help="also run the trace with one captured graph per request")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "multi-GPU sharding by orbital is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_03872_amd import ks, synth
    spec = synth.CONFIGS[args.workload]
    torch.cuda.set_device(0)
    log(f"[bench] workload {spec.name}: n={spec.n} L={spec.L} norb={spec.norb} natoms={spec.natoms}")
    sysm, gs, state = setup_workload(spec, ks.KS_FP64, args.chunk)
    info = gs.info()
    log(f"[bench] FP64 set-up done, chunk {info['chunk']}, npw {info['npw']}, tuning {gs.tuning}")
    ortho = gs.ortho
    log(f"[bench] orthonormalisation of {spec.norb} orbitals: {ortho['ms']:.2f} ms, "
        f"products {ortho['gemm_tflops']} TFLOP/s")
    ms_step, ktimes, phys, rho64 = run_steps(spec, gs, state, args.steps, args.warmup)
    hpsi_per_step = 4 * spec.norb
    value = hpsi_per_step / (ms_step * 1e-3)
    log(f"[bench] FP64 {args.steps} steps: {ms_step:.2f} ms/step, {value:.1f} orbital.Hpsi/s")
    kernels = kernel_table(info, spec, ktimes, args.steps, ms_step)
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    dk = kernels[dom]
    po, pl = alg_bytes(info, spec, dom)
    per_pass = orbitals_per_pass(spec, info)    # orbitals per launch
    roof = {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dk["alg_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, spec.name, per_pass, gs.info()), "avg_launch_us": dk["avg_us"],
            "alg_bytes_per_orbital": po, "alg_bytes_per_launch_shared": pl,
            "alg_bytes_per_launch": po * per_pass + pl, "orbitals_per_launch": per_pass}
    psi64 = state.download()
    etrs = None if args.no_etrs else run_etrs(spec, gs, state, args.etrs_steps)
    if etrs:
        log(f"[bench] ETRS (V_loc + Hartree + LDA xc): {etrs['ms_per_step']:.2f} ms/step, "
            f"{etrs['orbital_hpsi_per_s']:.1f} orbital.Hpsi/s, Hartree solve {etrs['hartree_ms']:.3f} ms")
    ground = None if args.no_ground else run_ground(spec, gs, state, args.ground_iters)
    if ground:
        log(f"[bench] ground state (steepest descent): {ground['ms_per_iteration']:.2f} ms/iteration, "
            f"by class {ground['ms_per_iteration_by_class']}, products {ground['gemm_tflops']} TFLOP/s")
    state.close()
    gs.close()

    mixed = None
    if not args.no_mixed:
        _, gm, sm = setup_workload(spec, ks.KS_MIXED, 0)
        start = sm.download()        # the orthonormalised start, again for the second projection mode
        runs = {}
        # projection 1: the split-BF16 reciprocal-space product; 0: real-space sums in the x-pass
        for proj in (1, 0):
            gm.set_tuning(gm.tuning["x_group"], gm.tuning["plane_group"], projection=proj)
            sm.upload(start)
            ms_m, kt_m, phys_m, _ = run_steps(spec, gm, sm, args.steps, args.warmup)
            psim = sm.download()
            # compare after the same number of steps from the same orthonormalised start
            d = (psim - psi64).reshape(spec.norb, -1).norm(dim=1) / psi64.reshape(spec.norb, -1).norm(dim=1)
            runs[proj] = {"value": round(hpsi_per_step / (ms_m * 1e-3), 1), "ms_per_step": round(ms_m, 3),
                          "speedup_vs_fp64": round(ms_step / ms_m, 3), "projection": proj,
                          "orbital_rel_err_vs_fp64_max": float(d.max().item()),
                          "band_energy_per_electron_diff_vs_fp64":
                              abs(phys_m["band_energy_per_electron_end"] - phys["band_energy_per_electron_end"]),
                          "kernels": kernel_table(gm.info(), spec, kt_m, args.steps, ms_m),
                          "chunk": gm.info()["chunk"], "tuning": gm.tuning}
            if proj == 1:
                runs[proj]["gproj"] = gproj_summary(gm.info(), spec, kt_m)
            log(f"[bench] mixed, projection {proj}: {ms_m:.2f} ms/step ({runs[proj]['speedup_vs_fp64']}x), "
                f"err vs FP64 {runs[proj]['orbital_rel_err_vs_fp64_max']:.2e}")
            del psim
        mixed = runs[1]
        mixed["projection_0"] = {k: runs[0][k] for k in ("value", "ms_per_step", "speedup_vs_fp64",
                                                         "orbital_rel_err_vs_fp64_max", "kernels")}
        if mixed["gproj"]:
            log(f"[bench] split-BF16 projection product: {mixed['gproj']['avg_us']:.1f} us/launch, "
                f"{mixed['gproj']['mfma_tflops']} TFLOP/s MFMA ({mixed['gproj']['mfma_frac']:.3f} of BF16 peak)")
        sm.close()
        gm.close()
        del start
    del psi64

    mixed_120 = None if (args.no_mixed or args.no_mixed_120) else run_mixed_large(3, log)

    serving = None
    if not args.no_serving:
        # under the capped budget every request's system holds one pass of at
        # most args.serving_pass orbitals, so the whole trace can reside
        serving = run_serving(args.serving_requests, args.serving_steps, args.serving_budget_gb, log,
                              chunk=args.serving_pass or None)
        log(f"[bench] serving (passes of {args.serving_pass}): p50 {serving['step_latency_ms_p50']:.2f} ms, "
            f"p99 {serving['step_latency_ms_p99']:.2f} ms, first step p99 {serving['time_to_first_step_ms_p99']:.0f} ms, "
            f"{serving['orbital_hpsi_per_s']:.0f} orbital.Hpsi/s over {serving['makespan_s']:.1f} s, "
            f"{serving['max_resident_requests']} resident at most")
        if args.serving_pass:
            one = run_serving(args.serving_requests, args.serving_steps, args.serving_budget_gb, log)
            log(f"[bench] serving (one pass per request): p50 {one['step_latency_ms_p50']:.2f} ms, "
                f"p99 {one['step_latency_ms_p99']:.2f} ms, first step p99 {one['time_to_first_step_ms_p99']:.0f} ms, "
                f"{one['orbital_hpsi_per_s']:.0f} orbital.Hpsi/s, {one['max_resident_requests']} resident at most")
            serving["one_pass"] = {k: one[k] for k in (
                "step_latency_ms_p50", "step_latency_ms_p99", "time_to_first_step_ms_p50",
                "time_to_first_step_ms_p99", "admission_ms_p99", "orbital_hpsi_per_s", "makespan_s",
                "max_resident_requests", "max_reserved_GiB", "failed")}
        if args.serving_full_budget_gb > 0:
            full = run_serving(args.serving_requests, args.serving_steps, args.serving_full_budget_gb, log)
            log(f"[bench] serving ({args.serving_full_budget_gb:.0f} GiB budget): p50 {full['step_latency_ms_p50']:.2f} ms, "
                f"p99 {full['step_latency_ms_p99']:.2f} ms, first step p99 {full['time_to_first_step_ms_p99']:.0f} ms, "
                f"{full['orbital_hpsi_per_s']:.0f} orbital.Hpsi/s")
            serving["full_budget"] = {k: full[k] for k in (
                "hbm_budget_GiB", "step_latency_ms_p50", "step_latency_ms_p99", "time_to_first_step_ms_p50",
                "time_to_first_step_ms_p99", "admission_ms_p99", "orbital_hpsi_per_s", "makespan_s",
                "max_resident_requests", "max_reserved_GiB", "failed")}
        if args.serving_compare:
            alt = run_serving(args.serving_requests, args.serving_steps, args.serving_budget_gb, log, batched=False,
                              max_active=64, lockstep=False)
            log(f"[bench] serving (graph per request): p50 {alt['step_latency_ms_p50']:.2f} ms, "
                f"p99 {alt['step_latency_ms_p99']:.2f} ms, {alt['orbital_hpsi_per_s']:.0f} orbital.Hpsi/s")
            serving["graph_per_request"] = {k: alt[k] for k in (
                "step_latency_ms_p50", "step_latency_ms_p99", "time_to_first_step_ms_p50",
                "time_to_first_step_ms_p99", "orbital_hpsi_per_s", "makespan_s", "max_resident_requests")}

    # a plain 1 GiB device copy: the reference kernel of the HBM traffic
    # counters, and the read + write bandwidth a streaming kernel reaches
    roof["plain_copy_GBs"] = plain_copy_bandwidth()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(spec, sysm)
        log(f"[bench] CPU oracle: {cpu['value']:.2f} orbital.Hpsi/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "orbital·Hψ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian potential, KB projectors and orbitals; no pseudopotential files)",
        "config": {"workload": f"{spec.name}: {spec.n[0]}x{spec.n[1]}x{spec.n[2]} grid, L={spec.L[0]} bohr, "
                               f"{spec.norb} orthonormalised orbitals (f={spec.occ}), {spec.natoms} atoms x 4 KB "
                               f"projectors, E_cut={spec.ecut} Ha; step = Taylor-4 (dt={spec.dt}) + density + norms "
                               f"on HBM-resident orbitals",
                   "global_batch": spec.norb, "grid": list(spec.n), "npw": info["npw"],
                   "chunk": info["chunk"], "orbitals_per_pass": per_pass,
                   "tuning": {k: gs.tuning[k] for k in ("x_group", "plane_group", "x_shape")},
                   "hpsi_per_step": hpsi_per_step,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernels": kernels,
        "physics": phys,
        "mixed": mixed,
        "mixed_120": mixed_120,
        "etrs": etrs,
        "ground_state": ground,
        "orthonormalisation": ortho,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
