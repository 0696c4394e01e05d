"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2106_03872_amd.profiling stats <kernel_stats.csv> [--top N]
      markdown table of a --kernel-trace --stats run (per kernel: calls,
      total and average time, share)
  python -m paper_2106_03872_amd.profiling traffic <fetch_dir> <write_dir> <out.json> --orbitals N [--workload W]
      HBM bytes per launch of each pass from a --pmc FETCH_SIZE run and a
      --pmc WRITE_SIZE run of the benchmark, scaled by what the counters read
      for the plain 1 GiB device copy every benchmark run times
  python -m paper_2106_03872_amd.profiling counters <dir> [<dir> ...]
      markdown table of per-dispatch SQ counters (mean over the dispatches of
      each kernel's most frequent launch shape)
  python -m paper_2106_03872_amd.profiling waves <dir> [<dir> ...]
      the same runs as fractions of SQ_WAVE_CYCLES (issuing, waiting on
      counters or barriers, waiting on dependencies, VALU and LDS active) and
      LDS bank-conflict cycles per LDS instruction, per pass
  python -m paper_2106_03872_amd.profiling mfma <dir> [--match S] [--model-flops F]
      matrix-core use per dispatch of the kernels that issue MFMAs: BF16
      flops counted (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512), busy fraction
      SQ_VALU_MFMA_BUSY_CYCLES / (SIMDs x GRBM_GUI_ACTIVE / XCDs), LDS
      bank-conflict cycles per LDS instruction
  python -m paper_2106_03872_amd.profiling durations <kernel_trace.csv> --match S [--split-at M]
      launch durations of the kernels whose names contain S, grouped by name
      and by whether the dispatch comes before the first kernel whose name
      contains M
  python -m paper_2106_03872_amd.profiling kerneltraffic <fetch_dir> <write_dir> --match S --scale-from <record.json>
      FETCH_SIZE / WRITE_SIZE per dispatch of the kernels whose names contain
      S, scaled by the calibration factors of a traffic record

Each pass is keyed by its class (xapply, xproj, ...); the launch counted is
the (kernel, grid) pair with the most dispatches, which in a benchmark run is
the tuned schedule of the timed steps (the autotuner times each candidate
three times, the timed steps run it more often).  The calibration copy is
the largest device copy of the run (by counter value).
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLASSES = ("gproj_gemm", "gproj_reduce", "gproj_table", "plane_inv", "xproj", "proj_reduce", "xapply", "plane_fwd", "xdens", "dens_sum", "dots", "unpack",
           "pack_kernel", "bj_solve", "bj_apply", "zgemm", "potrf", "trsm", "trinv", "herk", "sd_direction", "sd_update")
COPY_KIB = 1048576.0   # the calibration copy moves 1 GiB each way


def csrc_fingerprint():
    """sha256 over the library's kernel and runtime sources (csrc/, sorted)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2106_03872_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name):
    """Kernel name without namespaces, argument list and vector type noise."""
    n = name.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*\)$", "", n)
    n = n.replace("void ", "").replace("ks::", "")
    n = n.replace("HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")
    return n


def kernel_class(name):
    for k in CLASSES:
        if k in name:
            return k.replace("_kernel", "")
    if "copyBuffer" in name:
        return "copy"
    return None


def stats_table(path, top=20):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _counter_rows(d, counter=None):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if counter is None or r.get("Counter_Name") == counter:
                    rows.append(r)
    return rows


def _grid(r):
    return int(float(r.get("Grid_Size", r.get("grid_size", 0)) or 0))


def per_launch(rows):
    """class -> (kernel name, grid, dispatches, mean counter value) for the
    (name, grid) pair of the class with the most dispatches."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        k = kernel_class(r["Kernel_Name"])
        if k is not None:
            acc[k][(r["Kernel_Name"], _grid(r))].append(float(r["Counter_Value"]))
    out = {}
    for k, groups in acc.items():
        if k == "copy":
            # the calibration copy: the copy dispatches within a factor two
            # of the largest count (the small copies of the run share its grid)
            top = max(max(v) for v in groups.values())
            (name, grid), v = max(groups.items(), key=lambda kv: max(kv[1]))
            v = [x for x in v if x >= 0.5 * top]
        else:
            (name, grid), v = max(groups.items(), key=lambda kv: (len(kv[1]), kv[0][1]))
        out[k] = (name, grid, len(v), sum(v) / len(v))
    return out


def traffic_record(fetch_dir, write_dir, orbitals, workload):
    F = per_launch(_counter_rows(fetch_dir, "FETCH_SIZE"))
    W = per_launch(_counter_rows(write_dir, "WRITE_SIZE"))
    fs = COPY_KIB / F["copy"][3] if "copy" in F else None
    ws = COPY_KIB / W["copy"][3] if "copy" in W else None
    if fs is None or ws is None:
        raise SystemExit("the runs hold no calibration copy (a 1 GiB device copy)")
    rec = {"workload": workload, "orbitals_per_pass": orbitals, "csrc_sha256": csrc_fingerprint(),
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4), "kernels": {}}
    for k in sorted(set(F) & set(W)):
        if k == "copy":
            continue
        name, grid, n, fk = F[k]
        wk = W[k][3]
        rec["kernels"][k] = {"kernel": short_name(name), "grid": grid, "dispatches": n, "fetch_kib": round(fk, 1),
                             "write_kib": round(wk, 1), "bytes_per_launch": int(round((fk * fs + wk * ws) * 1024))}
    return rec


def counters_table(dirs):
    rows = []
    for d in dirs:
        rows += _counter_rows(d)
    names = sorted({r["Counter_Name"] for r in rows})
    by = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(list)))
    for r in rows:
        k = kernel_class(r["Kernel_Name"])
        if k is not None and k != "copy":
            by[k][(r["Kernel_Name"], _grid(r))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["| kernel | grid | " + " | ".join(names) + " |", "|---|---:|" + "---:|" * len(names)]
    for k in sorted(by):
        (name, grid), cs = max(by[k].items(), key=lambda kv: (max(len(v) for v in kv[1].values()), kv[0][1]))
        vals = []
        for c in names:
            v = cs.get(c)
            vals.append(f"{sum(v) / len(v):.4g}" if v else "")
        out.append(f"| `{short_name(name)}` | {grid} | " + " | ".join(vals) + " |")
    return "\n".join(out)


SIMDS, XCDS = 1024, 8   # MI355X: 256 compute units of 4 SIMDs in 8 XCDs


def _by_kernel(dirs, match=None):
    """short kernel name -> counter -> values, over the counter runs in dirs."""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in _counter_rows(d):
            if match is None or match in r["Kernel_Name"]:
                out[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def waves_table(dirs, classes=("plane_inv", "xproj", "xapply", "plane_fwd", "xdens"), match=None):
    """Per pass class, the most frequent (kernel, grid) of the counter runs in
    dirs (only kernels whose short name, template arguments included,
    contains `match`, when given)."""
    rows = []
    for d in dirs:
        rows += _counter_rows(d)
    by = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(list)))
    for r in rows:
        if match is not None and match not in short_name(r["Kernel_Name"]):
            continue
        k = kernel_class(r["Kernel_Name"])
        if k is not None and k != "copy":
            by[k][(r["Kernel_Name"], _grid(r))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["| kernel | issuing (`ACTIVE_INST_ANY`) | waiting on counters or barriers (`WAIT_ANY`) | "
           "waiting on dependencies (`WAIT_INST_ANY`) | VALU active | LDS active | "
           "LDS bank-conflict cycles per LDS instruction |", "|---|---:|---:|---:|---:|---:|---:|"]
    for k in classes:
        if k not in by:
            continue
        (name, grid), cs = max(by[k].items(), key=lambda kv: (max(len(v) for v in kv[1].values()), kv[0][1]))
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        wc = m["SQ_WAVE_CYCLES"]
        out.append(f"| `{short_name(name)}` | {m['SQ_ACTIVE_INST_ANY'] / wc:.3f} | {m['SQ_WAIT_ANY'] / wc:.3f} | "
                   f"{m['SQ_WAIT_INST_ANY'] / wc:.3f} | {m['SQ_ACTIVE_INST_VALU'] / wc:.3f} | "
                   f"{m['SQ_ACTIVE_INST_LDS'] / wc:.3f} | "
                   f"{m['SQ_LDS_BANK_CONFLICT'] / max(1.0, m['SQ_INSTS_LDS']):.3f} |")
    return "\n".join(out)


def _clock_ghz(d, match=None):
    """short kernel name -> mean clock over its dispatches in GHz: the GPU's
    active cycles per XCD (`GRBM_GUI_ACTIVE` / 8) over the dispatch's own
    duration, where the counter rows carry the dispatch's timestamps."""
    out = collections.defaultdict(list)
    for r in _counter_rows(d, "GRBM_GUI_ACTIVE"):
        if match is not None and match not in r["Kernel_Name"]:
            continue
        try:
            ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        except (KeyError, TypeError, ValueError):
            continue
        if ns > 0:
            out[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]) / XCDS / ns)
    return {k: sum(v) / len(v) for k, v in out.items()}


def clock_table(d, matches):
    """The clock each matching kernel ran at (`_clock_ghz`), one row per name."""
    out = ["| kernel | clock GHz (`GRBM_GUI_ACTIVE` / 8 / dispatch time) |", "|---|---:|"]
    for m in matches:
        for k, v in sorted(_clock_ghz(d, m).items()):
            out.append(f"| `{k}` | {v:.2f} |")
    return "\n".join(out)


def mfma_table(d, match=None, model_flops=None):
    by = _by_kernel([d], match)
    clk = _clock_ghz(d, match)
    out = ["| kernel | dispatches | BF16 MFMA flops (`MOPS_BF16` x 512) | model flops | MFMA busy "
           "(`SQ_VALU_MFMA_BUSY_CYCLES` / (1024 SIMDs x `GRBM_GUI_ACTIVE` / 8 XCDs)) | "
           "LDS bank-conflict cycles per LDS instruction | clock GHz (`GRBM_GUI_ACTIVE` / 8 / dispatch time) |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(by):
        m = {c: sum(v) / len(v) for c, v in by[k].items()}
        if m.get("SQ_INSTS_MFMA", 0.0) == 0.0:
            continue
        fl = m.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) * 512
        busy = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * m["GRBM_GUI_ACTIVE"] / XCDS)
        mf = f"{model_flops:.4g}" if model_flops else ""
        ck = f"{clk[k]:.2f}" if k in clk else ""
        out.append(f"| `{k}` | {len(by[k]['SQ_INSTS_MFMA'])} | {fl:.4g} | {mf} | {busy:.3f} | "
                   f"{m['SQ_LDS_BANK_CONFLICT'] / max(1.0, m['SQ_INSTS_LDS']):.2f} | {ck} |")
    return "\n".join(out)


def durations_table(trace, match, split_at=None, labels=("before", "after")):
    rows = sorted(csv.DictReader(open(trace)), key=lambda r: int(r["Dispatch_Id"]))
    cut = None
    if split_at:
        cut = next((int(r["Dispatch_Id"]) for r in rows if split_at in r["Kernel_Name"]), None)
    dur = collections.defaultdict(list)
    for r in rows:
        if match in r["Kernel_Name"]:
            ph = labels[0] if cut is None or int(r["Dispatch_Id"]) < cut else labels[1]
            dur[(ph, short_name(r["Kernel_Name"]))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| part of the run | kernel | launches | mean us | min us | max us |", "|---|---|---:|---:|---:|---:|"]
    for (ph, k), v in sorted(dur.items()):
        out.append(f"| {ph} | `{k}` | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    return "\n".join(out)


def kernel_traffic_table(fetch_dir, write_dir, match, record):
    rec = json.load(open(record))
    fs, ws = rec["fetch_scale"], rec["write_scale"]
    F, W = _by_kernel([fetch_dir], match), _by_kernel([write_dir], match)
    out = ["| kernel | dispatches | FETCH KiB | WRITE KiB | counted MB per launch |", "|---|---:|---:|---:|---:|"]
    for k in sorted(set(F) & set(W)):
        f = sum(F[k]["FETCH_SIZE"]) / len(F[k]["FETCH_SIZE"])
        w = sum(W[k]["WRITE_SIZE"]) / len(W[k]["WRITE_SIZE"])
        out.append(f"| `{k}` | {len(F[k]['FETCH_SIZE'])} | {f:.0f} | {w:.0f} | {(f * fs + w * ws) * 1024 / 1e6:.1f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--orbitals", type=int, required=True)
    b.add_argument("--workload", default="cfg3_96")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    w = sub.add_parser("waves")
    w.add_argument("dirs", nargs="+")
    w.add_argument("--match", default=None)
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("--match", default=None)
    m.add_argument("--model-flops", type=float, default=None)
    u = sub.add_parser("durations")
    u.add_argument("trace")
    u.add_argument("--match", required=True)
    u.add_argument("--split-at", default=None)
    u.add_argument("--labels", nargs=2, default=("before", "after"))
    k = sub.add_parser("clock")
    k.add_argument("dir")
    k.add_argument("--match", nargs="+", required=True)
    t = sub.add_parser("kerneltraffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--match", required=True)
    t.add_argument("--scale-from", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.csv, args.top))
    elif args.cmd == "traffic":
        rec = traffic_record(args.fetch_dir, args.write_dir, args.orbitals, args.workload)
        with open(args.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
    elif args.cmd == "counters":
        print(counters_table(args.dirs))
    elif args.cmd == "waves":
        print(waves_table(args.dirs, match=args.match))
    elif args.cmd == "mfma":
        print(mfma_table(args.dir, args.match, args.model_flops))
    elif args.cmd == "clock":
        print(clock_table(args.dir, args.match))
    elif args.cmd == "durations":
        print(durations_table(args.trace, args.match, args.split_at, tuple(args.labels)))
    else:
        print(kernel_traffic_table(args.fetch_dir, args.write_dir, args.match, args.scale_from))


if __name__ == "__main__":
    main()
