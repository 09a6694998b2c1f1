"""Summaries of rocprofv3 CSV output for the hot-path kernels.

    python -m paper_2303_11557_amd.profiling stats <kernel_stats.csv>
        per-kernel dispatch count and average / min / max duration (markdown)

    python -m paper_2303_11557_amd.profiling counters <counter_collection.csv> ...
        average value per dispatch of each collected counter, per hot-path kernel

    python -m paper_2303_11557_amd.profiling traffic <fetch.csv> <write.csv> [--out traffic.json]
        HBM bytes per dispatch of each hot-path kernel from FETCH_SIZE and
        WRITE_SIZE counter runs.  Both counters are scaled by what they read for
        the largest device-to-device copy in the same run (a copy of known size:
        bytes read = bytes written = its buffer size), so that the figures are
        bytes, whatever unit and sampling the counters use.

The traffic file records, per kernel, the SHA-256 prefix of the kernel's source
file, so that a reader can tell whether the figures still describe the code.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = {
    "fengine": os.path.join(HERE, "csrc", "fengine.hip"),
    "fft6400": os.path.join(HERE, "csrc", "fft6400.hip"),
    "beamform": os.path.join(HERE, "csrc", "beamform.hip"),
    "xengine": os.path.join(HERE, "csrc", "xengine.hip"),
    "pack": os.path.join(HERE, "csrc", "pack.hip"),
    "weights": os.path.join(HERE, "csrc", "weights.hip"),
    "average": os.path.join(HERE, "csrc", "average.hip"),
}
PREC = {"0": "fp32", "1": "fp16", "2": "int8"}


def source_sha(family):
    with open(SOURCES[family], "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short_name(name):
    """Kernel name without namespaces and argument lists, template arguments kept."""
    n = name.replace("mwax::(anonymous namespace)::", "").replace("mwax::", "")
    n = re.sub(r"^void ", "", n)
    depth, out = 0, []
    for ch in n:           # drop the parenthesised argument list (outside templates)
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def kernel_key(name):
    """Stable key of a hot-path kernel ('fengine_int8', 'xengine_int8', ...), or None."""
    s = short_name(name)
    m = re.match(r"fengine_(batch_)?kernel<(\d+), (\d), (false|true)(, (false|true))?>", s)
    if m:
        return (f"fengine_{'batch_' if m.group(1) else ''}{PREC[m.group(3)]}"
                + ("_stats" if m.group(4) == "true" else "") + ("_delay" if m.group(6) == "true" else ""))
    m = re.match(r"fft6400_kernel<(\d), (false|true), (false|true)>", s)
    if m:
        return (f"fft6400_{PREC[m.group(1)]}" + ("_stats" if m.group(2) == "true" else "")
                + ("_delay" if m.group(3) == "true" else ""))
    m = re.match(r"corner_turn_kernel<(\d)>", s)
    if m:
        return "fft6400_corner_turn_" + {"1": "int8", "2": "fp16", "4": "fp32"}[m.group(1)]
    if s.startswith("beamform_kernel"):
        return "beamform_coherent"
    if s.startswith("incoherent_kernel"):
        return "beamform_incoherent"
    m = re.match(r"xengine_(mfma|batch|avg)<(\d)>", s)
    if m:
        return f"xengine_{'' if m.group(1) == 'mfma' else m.group(1) + '_'}{PREC[m.group(2)]}"
    if s.startswith("xengine_f32"):
        return "xengine_fp32"
    if s.startswith("pack_"):
        return s.split("<")[0]
    if s.startswith("apply_weights_kernel"):
        return "weights_apply"
    if s.startswith("vis_weights_kernel"):
        return "weights_occupancy"
    if s.startswith("fscrunch_kernel"):
        return "average_fscrunch"
    return None


def stats_table(path):
    rows = list(csv.DictReader(open(path)))
    lines = ["| kernel | dispatches | avg ms | min ms | max ms | total ms |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| {} | {} | {:.4f} | {:.4f} | {:.4f} | {:.3f} |".format(
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6,
            float(r["MaxNs"]) / 1e6, float(r["TotalDurationNs"]) / 1e6))
    return "\n".join(lines)


def counter_per_dispatch(path, counter):
    vals = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
        vals[k] = vals.get(k, 0.0) + float(r["Counter_Value"])
    return vals


def traffic(fetch_csv, write_csv, copy_bytes):
    fetch = counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = counter_per_dispatch(write_csv, "WRITE_SIZE")

    def copy_factor(vals):
        copies = [v for (d, n), v in vals.items() if "copyBuffer" in n]
        if not copies:
            raise SystemExit("no device-to-device copy in the counter run (bench.py --copy-probe)")
        return copy_bytes / max(copies)

    ff, wf = copy_factor(fetch), copy_factor(write)
    per = collections.defaultdict(lambda: {"fetch": [], "write": []})
    for (d, n), v in fetch.items():
        k = kernel_key(n)
        if k:
            per[k]["fetch"].append(v * ff)
    for (d, n), v in write.items():
        k = kernel_key(n)
        if k:
            per[k]["write"].append(v * wf)
    out = {"copy_probe_bytes": copy_bytes, "fetch_factor_bytes_per_unit": ff,
           "write_factor_bytes_per_unit": wf}
    for k, v in per.items():
        fam = k.split("_")[0]
        fb = sum(v["fetch"]) / max(len(v["fetch"]), 1)
        wb = sum(v["write"]) / max(len(v["write"]), 1)
        out[k] = {"source_sha": source_sha(fam) if fam in SOURCES else None,
                  "dispatches": len(v["fetch"]), "fetch_bytes_per_launch": fb,
                  "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb}
    return out


def counters_table(paths):
    """Average value per dispatch of every counter in the given counter-collection
    CSVs, per hot-path kernel (markdown)."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    names = []
    for path in paths:
        vals = collections.defaultdict(float)
        for r in csv.DictReader(open(path)):
            vals[(int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"])] += float(r["Counter_Value"])
        for (d, n, c), v in vals.items():
            k = kernel_key(n)
            if k:
                per[k][c].append(v)
                if c not in names:
                    names.append(c)
    lines = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for k in sorted(per):
        cols = [per[k][c] for c in names]
        nd = max(len(x) for x in cols if x)
        lines.append(f"| {k} | {nd} | " + " | ".join(
            f"{sum(x) / len(x):.4g}" if x else "-" for x in cols) + " |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-bytes", type=float, default=float(4 << 30))
    t.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv))
    elif a.cmd == "counters":
        print(counters_table(a.csv))
    else:
        tr = traffic(a.fetch_csv, a.write_csv, a.copy_bytes)
        txt = json.dumps(tr, indent=1, sort_keys=True)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt + "\n")
        print(txt)


if __name__ == "__main__":
    sys.exit(main())
