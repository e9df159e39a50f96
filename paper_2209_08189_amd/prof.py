"""Summaries of rocprofv3 CSV output (kernel statistics, memory counters).

  python -m paper_2209_08189_amd.prof stats <kernel_stats.csv> <title> <command>
      -> markdown table of per-kernel calls / total / average time
  python -m paper_2209_08189_amd.prof counters <out.md> <title> <command> <dir> [<dir> ...]
      -> markdown table of per-kernel counter means from --pmc runs
  python -m paper_2209_08189_amd.prof mfma <trace_dir> <pmc_dir> <title> <trace command> <pmc command>
      -> markdown table of per-kernel time and BF16 MFMA rate (the
         SQ_INSTS_VALU_MFMA_MOPS_BF16 counter counts units of 512 FLOPs)
  python -m paper_2209_08189_amd.prof traffic <fetch_dir> <write_dir> <copy_MiB> <out.json> <command>
      -> HBM bytes per launch of the SL kernels from FETCH_SIZE / WRITE_SIZE
         runs, scaled by what the same counters read for the library's plain
         copy kernel (k_copy4) of a known size; stamped with the SHA-1 of the
         transport kernel source so stale numbers are not reused.
"""
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
TRANSPORT_SRC = os.path.join(HERE, "csrc", "k_transport.hip")


def short(name):
    """Kernel name without namespace, return type and parameter list."""
    n = name.replace("clh::(anonymous namespace)::", "").replace("void ", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def stats_md(path, title, command):
    rows = list(csv.DictReader(open(path)))
    out = ["# %s" % title, "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        if float(r["Percentage"]) < 0.05:
            continue
        out.append("| %s | %s | %.1f | %.2f | %.2f |" % (short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
                                                        float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def counter_means(directory, counter):
    path = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)[0]
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]) * 1024.0)   # KiB -> bytes
    return {k: sum(v) / len(v) for k, v in acc.items()}


# tiled SL kernels of the solver in FP32: k_sl_tile<field, output, mode,
# interpolation order, interleaved feet>
SL_NAMES = {"sl_state": "k_sl_tile<float, float, 0, 3, true>", "sl_adjoint": "k_sl_tile<float, float, 1, 3, true>",
            "sl_inc": "k_sl_tile<float, float, 2, 3, true>",
            "sl_adjoint_trilinear": "k_sl_tile<float, float, 1, 1, true>",
            "sl_inc_trilinear": "k_sl_tile<float, float, 2, 1, true>"}


def traffic(fetch_dir, write_dir, copy_mib, command):
    fetch = counter_means(fetch_dir, "FETCH_SIZE")
    write = counter_means(write_dir, "WRITE_SIZE")
    nbytes = copy_mib * (1 << 20)
    fs = nbytes / fetch["k_copy4"]
    ws = nbytes / write["k_copy4"]
    rec = {"source_sha1": hashlib.sha1(open(TRANSPORT_SRC, "rb").read()).hexdigest(),
           "fetch_scale": fs, "write_scale": ws,
           "calibration": "k_copy4 over %d MiB: FETCH_SIZE %.0f B, WRITE_SIZE %.0f B" % (copy_mib, fetch["k_copy4"],
                                                                                       write["k_copy4"]),
           "command": command, "kernels": {}}
    for k, kn in SL_NAMES.items():
        if kn in fetch and kn in write:
            rec["kernels"][k] = {"fetch_bytes": fetch[kn], "write_bytes": write[kn],
                                 "hbm_bytes_scaled": fetch[kn] * fs + write[kn] * ws}
    return rec


def counters_md(dirs, title, command, copy_mib=256, min_us=20.0):
    """Per-kernel means over dispatches of every counter in the passes' CSVs
    (one rocprofv3 --pmc run per directory).  FETCH_SIZE / WRITE_SIZE are
    reported in bytes per launch, scaled by what the same counter reads for
    the library's copy kernel k_copy4 over copy_mib MiB."""
    vals = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(list)
    for d in dirs:
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        for r in csv.DictReader(open(path)):
            k = short(r["Kernel_Name"])
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            if r.get("Start_Timestamp") and r.get("End_Timestamp"):
                dur[k].append((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3)
    names = sorted({c for k in vals for c in vals[k]})
    mean = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}
    scale = {}
    nbytes = copy_mib * (1 << 20)
    if "k_copy4" in mean:
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            if c in mean["k_copy4"] and mean["k_copy4"][c] > 0:
                scale[c] = nbytes / (mean["k_copy4"][c] * 1024.0)
    out = ["# %s" % title, "", "Command (one run per counter set):", "", "```", command, "```", ""]
    if scale:
        out += ["FETCH_SIZE / WRITE_SIZE: bytes per launch, each scaled by the factor that makes the counter "
                "read %d MiB for the plain copy kernel k_copy4 (%s)." % (copy_mib, ", ".join(
                    "%s x%.3f" % (c, f) for c, f in scale.items())), ""]
    out += ["| kernel | " + " | ".join(names) + " |", "|---|" + "---:|" * len(names)]
    order = sorted(mean, key=lambda k: -max(dur.get(k, [0.0]) or [0.0]))
    for k in order:
        if dur.get(k) and max(dur[k]) < min_us and k != "k_copy4":
            continue
        cells = []
        for c in names:
            v = mean[k].get(c)
            if v is None:
                cells.append("")
            elif c in scale:
                cells.append("%.1f MB" % (v * 1024.0 * scale[c] / 1e6))
            else:
                cells.append("%.4g" % v)
        out.append("| %s | %s |" % (k, " | ".join(cells)))
    return "\n".join(out) + "\n"


def mfma_md(trace_dir, pmc_dir, title, trace_cmd, pmc_cmd, peak_tflops=2500.0):
    """Per-kernel duration (kernel trace run) and BF16 MFMA FLOPs per
    dispatch (counter run: SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512) -> TFLOP/s
    against the dense BF16 peak."""
    dur, calls = defaultdict(float), defaultdict(int)
    path = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)[0]
    for r in csv.DictReader(open(path)):
        k = short(r["Kernel_Name"])
        dur[k] += (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
        calls[k] += 1
    mops, n = defaultdict(float), defaultdict(int)
    path = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)[0]
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == "SQ_INSTS_VALU_MFMA_MOPS_BF16":
            k = short(r["Kernel_Name"])
            mops[k] += float(r["Counter_Value"])
            n[k] += 1
    total = sum(dur.values())
    out = ["# %s" % title, "", "Kernel trace:", "", "```", trace_cmd, "```", "", "MFMA counters (separate run):", "",
           "```", pmc_cmd, "```", "",
           "| kernel | calls | avg us | %% of kernel time | MFMA GFLOP / dispatch | TFLOP/s | %% of %.0f TFLOP/s |" % peak_tflops,
           "|---|---:|---:|---:|---:|---:|---:|"]
    fl_all = t_all = 0.0
    for k in sorted(dur, key=lambda k: -dur[k]):
        if dur[k] < 0.005 * total:
            continue
        avg = dur[k] / calls[k]
        if n.get(k) and mops[k] > 0:
            fl = mops[k] / n[k] * 512.0
            tf = fl / (avg * 1e-6) / 1e12
            fl_all += fl * calls[k]
            t_all += dur[k]
            out.append("| %s | %d | %.1f | %.1f | %.2f | %.1f | %.1f |" % (k, calls[k], avg, 100 * dur[k] / total,
                                                                         fl / 1e9, tf, 100 * tf / peak_tflops))
        else:
            out.append("| %s | %d | %.1f | %.1f | | | |" % (k, calls[k], avg, 100 * dur[k] / total))
    if t_all:
        out += ["", "MFMA kernels together: %.1f TFLOP/s over %.1f ms (%.1f %% of all kernel time)." % (
            fl_all / (t_all * 1e-6) / 1e12, t_all / 1e3, 100 * t_all / total)]
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        sys.stdout.write(stats_md(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "counters":
        # counters <out.md> <title> <command> <dir> [<dir> ...]
        open(sys.argv[2], "w").write(counters_md(sys.argv[5:], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "mfma":
        sys.stdout.write(mfma_md(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6]))
    elif sys.argv[1] == "traffic":
        rec = traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[6])
        json.dump(rec, open(sys.argv[5], "w"), indent=1)
        print(json.dumps(rec, indent=1))
