"""Summaries of rocprofv3 output (csv) in the form kept under profiles/.

  python -m paper_2411_04776_amd.profsum trace --dir D --command CMD --out F
      kernel-trace statistics: per kernel launches, total, mean and median
      duration, share of kernel time.
  python -m paper_2411_04776_amd.profsum valu --pmc D1 --trace D2 --calib D3 --commands ... --out F
      VALU flop rates of kernels from SQ_INSTS_VALU_FLOPS_FP32/FP64 (scaled
      by a calibration run of known elementwise adds) over their durations.
  python -m paper_2411_04776_amd.profsum pmc --fetch D1 --write D2 --copy-fetch D3 --copy-write D4
         --json J --leg LEG --kernel NAME --commands C1 C2 C3 C4 --out F
      HBM traffic of one kernel: FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch) summed over every dispatch of the kernel, each scaled by what
      the same counter reads for a device copy of known size, against the
      algorithmic bytes the library counted for the same launches
      (bench.py's JSON line of the same command: roofline.all_launches).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PCG_SOURCES = ("paper_2411_04776_amd/csrc/k_solver.hip", "paper_2411_04776_amd/csrc/incidence.h",
               "paper_2411_04776_amd/csrc/device_util.h", "paper_2411_04776_amd/csrc/ipc_internal.h")


def source_hash(files=PCG_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(d, suffix):
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f) as fh:
            yield from csv.DictReader(fh)


def counter(d, name, kernel_substr):
    vals = [float(r["Counter_Value"]) for r in _rows(d, "counter_collection.csv")
            if r.get("Counter_Name") == name and kernel_substr in r["Kernel_Name"]]
    return vals


def dispatches(d, name, kernel_substr):
    """(counter value, grid size, duration s) per dispatch of a kernel."""
    return [(float(r["Counter_Value"]), int(r["Grid_Size"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
            for r in _rows(d, "counter_collection.csv")
            if r.get("Counter_Name") == name and kernel_substr in r["Kernel_Name"]]


def trace(args):
    per = {}
    for r in _rows(args.dir, "kernel_trace.csv"):
        per.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in per.values())
    lines = [f"# Kernel time: {args.title}", "", "Command (repository root, MI355X):", "```", args.command, "```", "",
             f"Total kernel time {tot / 1e3:.1f} ms over {sum(len(v) for v in per.values())} dispatches.", "",
             "| kernel | launches | total ms | share | mean us | median us |", "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:args.top]:
        name = k.split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {len(v)} | {sum(v) / 1e3:.2f} | {100 * sum(v) / tot:.1f} % | "
                     f"{statistics.mean(v):.2f} | {statistics.median(v):.2f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def pmc(args):
    cf = counter(args.copy_fetch, "FETCH_SIZE", "copyBuffer")
    cw = counter(args.copy_write, "WRITE_SIZE", "copyBuffer")
    copy_kib = args.copy_mib * 1024.0
    sf = copy_kib / cf[0]
    sw = copy_kib / cw[0]
    f = counter(args.fetch, "FETCH_SIZE", args.kernel + "<")
    w = counter(args.write, "WRITE_SIZE", args.kernel + "<")
    line = json.load(open(args.json))
    leg = line if args.leg == "headline" else line[args.leg]
    roof = leg["roofline"]
    k = roof if roof["kernel"].startswith(args.kernel) else roof["other_pcg_kernel"]
    n_alg = k["all_launches"]["launches"]
    alg = k["all_launches"]["algorithmic_bytes_per_launch"]
    tf = sum(f) * 1024.0 * sf
    tw = sum(w) * 1024.0 * sw
    per = (tf + tw) / max(len(f), 1)
    ratio = per / alg if alg else float("nan")
    # the full-list dispatches (grid of at least 90 % of the largest): their
    # traffic over their durations in the FETCH run
    fd = dispatches(args.fetch, "FETCH_SIZE", args.kernel + "<")
    wd = dispatches(args.write, "WRITE_SIZE", args.kernel + "<")
    gmax = max(g for _, g, _ in fd)
    bf = [(v, t) for v, g, t in fd if g >= 0.9 * gmax]
    bw = [v for v, g, _ in wd if g >= 0.9 * gmax]
    full = []
    if bf and bw:
        fb = statistics.mean(v for v, _ in bf) * 1024.0 * sf + statistics.mean(bw) * 1024.0 * sw
        fus = statistics.median(t for _, t in bf) * 1e6
        full = ["", f"Full-list dispatches (grid of at least 90 % of the largest, {gmax} threads): {len(bf)} in the "
                    f"FETCH run; {fb / 2**20:.1f} MiB of HBM traffic per dispatch over a median {fus:.1f} us "
                    f"(durations from the counter run) = {fb / (fus * 1e-6) / 1e9:.0f} GB/s.", "",
                f"full_list_dispatches: {len(bf)}", f"full_list_traffic_bytes: {int(fb)}", f"full_list_us: {fus:.2f}",
                f"full_list_hbm_gbs: {fb / (fus * 1e-6) / 1e9:.1f}"]
    lines = [f"# HBM traffic of {args.kernel}: {args.title}", "",
             "Commands (repository root, MI355X box), one counter per run:", "```", *args.commands, "```", "",
             f"Calibration: a {args.copy_mib} MiB device copy (`__amd_rocclr_copyBuffer`) reads FETCH_SIZE = "
             f"{cf[0]:.1f} KiB and WRITE_SIZE = {cw[0]:.1f} KiB, so FETCH_SIZE is scaled by {sf:.4f} and WRITE_SIZE "
             f"by {sw:.4f}.", "",
             f"{args.kernel} over {len(f)} dispatches (FETCH run) / {len(w)} (WRITE run): summed FETCH_SIZE "
             f"{sum(f):.0f} KiB, WRITE_SIZE {sum(w):.0f} KiB; scaled: {tf / 2**20:.1f} MiB read + "
             f"{tw / 2**20:.1f} MiB written, {per / 2**20:.3f} MiB per dispatch (median FETCH "
             f"{statistics.median(f):.1f} KiB, WRITE {statistics.median(w):.1f} KiB).", "",
             f"Algorithmic bytes the library counted for the same launches ({n_alg} launches in the JSON line of the "
             f"FETCH run): {alg / 2**20:.3f} MiB per launch.", "",
             f"traffic_bytes_per_launch: {int(per)}",
             f"traffic_over_algorithmic: {ratio:.3f}", *full,
             f"kernel_source_sha256: `{source_hash()}`", "",
             "(the hash covers the PCG kernel sources; bench.py reports `traffic` only while it matches)"]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"{args.kernel}: {per / 2**20:.3f} MiB per dispatch, algorithmic {alg / 2**20:.3f}, ratio {ratio:.3f}")


ELASTIC_SOURCES = ("paper_2411_04776_amd/csrc/k_elastic.hip", "paper_2411_04776_amd/csrc/device_util.h",
                   "paper_2411_04776_amd/csrc/ipc_internal.h")
PEAK_TFLOPS = {"FP32": 157.3, "FP64": 78.6}


def valu(args):
    """VALU flop rate of the assembly kernels: SQ_INSTS_VALU_FLOPS_FP32/FP64
    summed over every dispatch, scaled by what the same counters read for
    elementwise adds of a known count (the calibration run), over the
    kernels' summed durations in a kernel-trace run of the same command."""
    cal = {}
    for r in _rows(args.calib, "counter_collection.csv"):
        if "CUDAFunctor_add<float" in r["Kernel_Name"] and r["Counter_Name"] == "SQ_INSTS_VALU_FLOPS_FP32":
            cal["FP32"] = args.calib_adds / float(r["Counter_Value"])
        if "CUDAFunctor_add<double" in r["Kernel_Name"] and r["Counter_Name"] == "SQ_INSTS_VALU_FLOPS_FP64":
            cal["FP64"] = args.calib_adds / float(r["Counter_Value"])
    fl = {}
    for r in _rows(args.pmc, "counter_collection.csv"):
        k = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("ipcg::", "")
        fl.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    dur = {}
    for r in _rows(args.trace, "kernel_trace.csv"):
        k = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("ipcg::", "")
        dur.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    lines = [f"# VALU flop rate of the assembly kernels: {args.title}", "", "Commands (repository root, MI355X):",
             "```", *args.commands, "```", "",
             f"Calibration: elementwise adds of {args.calib_adds} elements read SQ_INSTS_VALU_FLOPS_FP32 / FP64 = "
             f"{args.calib_adds / cal['FP32']:.0f} / {args.calib_adds / cal['FP64']:.0f}, so the counters are scaled by "
             f"{cal['FP32']:.2f} (FP32) and {cal['FP64']:.2f} (FP64) flops per count.", "",
             "| kernel | dispatches | FP32 GFLOP | FP64 GFLOP | time ms | FP32 TFLOP/s | FP64 TFLOP/s | of FP32 peak | of FP64 peak |",
             "|---|---|---|---|---|---|---|---|---|"]
    keys = []
    for k in sorted(fl):
        f32 = sum(fl[k].get("SQ_INSTS_VALU_FLOPS_FP32", [])) * cal["FP32"]
        f64 = sum(fl[k].get("SQ_INSTS_VALU_FLOPS_FP64", [])) * cal["FP64"]
        t = sum(dur.get(k, []))
        r32, r64 = (f32 / t / 1e12, f64 / t / 1e12) if t > 0 else (0.0, 0.0)
        lines.append(f"| `{k}` | {len(dur.get(k, []))} | {f32 / 1e9:.1f} | {f64 / 1e9:.1f} | {1e3 * t:.2f} | {r32:.2f} | "
                     f"{r64:.2f} | {r32 / PEAK_TFLOPS['FP32']:.3f} | {r64 / PEAK_TFLOPS['FP64']:.3f} |")
        base = k.split("<")[0]
        keys.append((f"{base}_fp32_tflops", f"{r32:.3f}"))
        keys.append((f"{base}_fp64_tflops", f"{r64:.3f}"))
        keys.append((f"{base}_valu_utilisation", f"{r32 / PEAK_TFLOPS['FP32'] + r64 / PEAK_TFLOPS['FP64']:.4f}"))
    lines += ["", "(utilisation: the FP32 rate over the FP32 peak plus the FP64 rate over the FP64 peak)", ""]
    lines += [f"{k}: {v}" for k, v in keys]
    lines += [f"kernel_source_sha256: `{source_hash(ELASTIC_SOURCES)}`"]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--top", type=int, default=25)
    t.add_argument("--out", required=True)
    p = sub.add_parser("pmc")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--json", "--kernel", "--out"):
        p.add_argument(a, required=True)
    p.add_argument("--leg", default="headline")
    p.add_argument("--copy-mib", type=int, default=256)
    p.add_argument("--commands", nargs="+", required=True)
    p.add_argument("--title", default="")
    v = sub.add_parser("valu")
    for a in ("--pmc", "--trace", "--calib", "--out"):
        v.add_argument(a, required=True)
    v.add_argument("--calib-adds", type=int, default=16 << 20)
    v.add_argument("--commands", nargs="+", required=True)
    v.add_argument("--title", default="")
    args = ap.parse_args()
    {"trace": trace, "pmc": pmc, "valu": valu}[args.what](args)


if __name__ == "__main__":
    main()
