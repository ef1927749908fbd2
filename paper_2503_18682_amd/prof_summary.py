"""Text summaries of rocprofv3 output (the files kept under profiles/).

Kernel durations (a ``--kernel-trace --stats --output-format csv`` run):

    python -m paper_2503_18682_amd.prof_summary stats --csv X_kernel_stats.csv \
        --out profiles/<name>.txt --workload "..." --command "..."

Per-dispatch SQ counter averages of one kernel (any number of counter runs):

    python -m paper_2503_18682_amd.prof_summary counters --csv A.csv B.csv \\
        --kernel k_blend --out profiles/<name>.txt --workload "..." --command "..."

HBM traffic of one kernel from two counter runs:

    python -m paper_2503_18682_amd.prof_summary traffic --fetch F.csv --write W.csv \
        --kernel k_blend --copy-mib 1024 --out profiles/<name>.txt [--command "..."]

HBM traffic and bandwidth per frame of every kernel of the path (the same two
counter runs plus the kernel-trace statistics for durations):

    python -m paper_2503_18682_amd.prof_summary traffic-table --fetch F.csv --write W.csv \
        --stats X_kernel_stats.csv --copy-mib 1024 --out profiles/<name>.txt

F.csv / W.csv are the ``*_counter_collection.csv`` files of two runs of the
same program with ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``.  Both runs
must also execute one plain device copy of ``--copy-mib`` MiB (bench.py
``--copy-calibration``): the copy reads and writes exactly that many bytes,
so bytes / counter for the copy is the scale factor of each counter on this
machine.  The kernel's traffic per dispatch is then

    FETCH_SIZE x 1024 x fetch_scale + WRITE_SIZE x 1024 x write_scale.

The summary records a hash of the kernel's sources (``SOURCES``); bench.py
reports the traffic only while the hash still matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# translation units and headers the compositing kernels are built from
SOURCES = {"k_blend": ["csrc/blend.hip", "csrc/internal.h", "csrc/binning.h"],
           "k_blend_bwd": ["csrc/blend.hip", "csrc/internal.h", "csrc/binning.h"]}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _per_dispatch(path, counter):
    """{kernel name: [counter value per dispatch]} (values summed over the
    hardware instances rocprofv3 lists separately)."""
    acc = collections.defaultdict(float)
    names = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            d = int(row["Dispatch_Id"])
            acc[d] += float(row["Counter_Value"])
            names[d] = row["Kernel_Name"]
    out = collections.defaultdict(list)
    for d in sorted(acc):
        out[names[d]].append(acc[d])
    return out


def _pick(per, pattern):
    hits = {k: v for k, v in per.items() if re.search(pattern, k)}
    if not hits:
        raise SystemExit(f"no dispatch matches {pattern!r}")
    return hits


def summarise(fetch_csv, write_csv, kernel, copy_mib):
    copy_bytes = copy_mib * (1 << 20)
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _per_dispatch(path, counter)
        copies = _pick(per, r"copyBuffer|elementwise|CopyKernel")
        # the calibration copy is the copy dispatch with the largest count
        copy_kib = max(max(v) for v in copies.values())
        ks = _pick(per, re.escape(kernel) + r"\b")
        vals = [x for v in ks.values() for x in v]
        avg_kib = sum(vals) / len(vals)
        scale = copy_bytes / (copy_kib * 1024.0)
        res[counter] = dict(copy_kib=copy_kib, scale=scale, kernel_kib=avg_kib, dispatches=len(vals),
                            kernel_names=sorted(ks), bytes=avg_kib * 1024.0 * scale)
    res["traffic_bytes"] = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    return res


def write_summary(res, kernel, out, command, workload):
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    lines = [
        f"# HBM traffic of {kernel} ({workload})",
        "#",
        "# Commands (repository root R on the GPU box, run from /tmp with TMPDIR=/tmp):",
    ]
    lines += [f"#   {c}" for c in command.split(" ;; ")]
    lines += [
        "#",
        f"# Calibration: one device copy of {res['copy_mib']} MiB in the same process.",
        f"#   FETCH_SIZE of the copy = {f['copy_kib']:.0f} KiB -> scale {f['scale']:.4f} bytes per counted byte",
        f"#   WRITE_SIZE of the copy = {w['copy_kib']:.0f} KiB -> scale {w['scale']:.4f}",
        "#",
        f"kernel: {kernel}",
        f"kernel_names: {', '.join(f['kernel_names'])}",
        f"dispatches: {f['dispatches']} (fetch run), {w['dispatches']} (write run)",
        f"fetch_kib_per_dispatch: {f['kernel_kib']:.1f}",
        f"write_kib_per_dispatch: {w['kernel_kib']:.1f}",
        f"fetch_scale: {f['scale']:.6f}",
        f"write_scale: {w['scale']:.6f}",
        f"traffic_bytes_per_dispatch: {res['traffic_bytes']:.0f}",
        f"source_sha256: {source_hash(kernel)}",
    ]
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def read_traffic(path, kernel):
    """Traffic per dispatch from a summary, or None when the file is missing
    or the kernel's sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash(kernel):
        return None
    return float(vals["traffic_bytes_per_dispatch"])


def write_traffic_table(fetch_csv, write_csv, stats_csv, copy_mib, out, command, workload,
                        frame_kernel="k_preprocess"):
    """Per frame: dispatches, HBM bytes (scaled counters) and trace duration of
    every kernel, and the bandwidth they imply.  Frames are counted by the
    dispatches of `frame_kernel` (one per frame) in each run."""
    copy_bytes = copy_mib * (1 << 20)
    per_frame = {}
    scales = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _per_dispatch(path, counter)
        copies = _pick(per, r"copyBuffer|elementwise|CopyKernel")
        scale = copy_bytes / (max(max(v) for v in copies.values()) * 1024.0)
        scales[counter] = scale
        frames = sum(len(v) for k, v in per.items() if re.search(re.escape(frame_kernel) + r"\b", k))
        for name, v in per.items():
            m = re.search(r"(k_\w+)", name)
            if not m:
                continue
            e = per_frame.setdefault(m.group(1), {})
            e[counter] = sum(v) * 1024.0 * scale / max(frames, 1)
            e["calls_" + counter] = len(v) / max(frames, 1)
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    calls = collections.defaultdict(float)
    total_ns = collections.defaultdict(float)
    for r in rows:
        m = re.search(r"(k_\w+)", r["Name"])
        if m:
            calls[m.group(1)] += float(r["Calls"])
            total_ns[m.group(1)] += float(r["TotalDurationNs"])
    trace_frames = calls.get(frame_kernel, 1.0)
    lines = [f"# HBM traffic and bandwidth per frame, every kernel ({workload})", "#",
             "# Commands (repository root R on the GPU box, run from /tmp with TMPDIR=/tmp):"]
    lines += [f"#   {c}" for c in command.split(" ;; ")]
    lines += ["#",
              f"# bytes = FETCH_SIZE x 1024 x {scales['FETCH_SIZE']:.4f} + WRITE_SIZE x 1024 x "
              f"{scales['WRITE_SIZE']:.4f} (a {copy_mib} MiB device copy calibrates both), per frame;",
              "# duration = kernel-trace total per frame; GB/s = bytes / duration",
              "#",
              "# kernel | dispatches per frame | fetch MB | write MB | us per frame | GB/s"]
    for k in sorted(per_frame, key=lambda k: -total_ns.get(k, 0.0)):
        e = per_frame[k]
        fb, wb = e.get("FETCH_SIZE", 0.0), e.get("WRITE_SIZE", 0.0)
        us = total_ns.get(k, 0.0) / trace_frames / 1e3
        gbs = (fb + wb) / (us * 1e-6) / 1e9 if us > 0 else 0.0
        lines.append(f"{k} | {e.get('calls_FETCH_SIZE', 0.0):.2g} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {us:.1f} | "
                     f"{gbs:.0f}")
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^>(]*>)?", name)
    if not m:
        return name.split("(")[0][:48]
    return m.group(1) + (m.group(2) or "")


def write_stats(csv_path, out, command, workload):
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel durations: {workload}", "#",
             "# Commands (repository root R on the GPU box, run from /tmp with TMPDIR=/tmp):"]
    lines += [f"#   {c}" for c in command.split(" ;; ")]
    lines += ["#", "# kernel | calls | average us | min us | max us | total ms | percent"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{short_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {100 * float(r['TotalDurationNs']) / total:.1f}")
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def write_counters(csv_paths, kernel, out, command, workload, clock_ghz=2.4, simds=1024):
    """Per-dispatch averages of every counter in the given counter runs for
    one kernel, with the VALU issue figure: SQ_INSTS_VALU wave instructions
    take 4 cycles each on a 16-lane SIMD, so the chip issues at most
    simds * clock / 4 of them per second."""
    vals = collections.defaultdict(list)
    ns = []
    for path in csv_paths:
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        dur = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if not re.search(re.escape(kernel) + r"\b", row["Kernel_Name"]):
                    continue
                d = int(row["Dispatch_Id"])
                acc[d][row["Counter_Name"]] += float(row["Counter_Value"])
                dur[d] = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
        for d, c in acc.items():
            for k, v in c.items():
                vals[k].append(v)
            ns.append(dur[d])
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    t = sum(ns) / len(ns) * 1e-9
    lines = [f"# SQ counters of {kernel} ({workload}), averages per dispatch", "#",
             "# Commands (repository root R on the GPU box, run from /tmp with TMPDIR=/tmp):"]
    lines += [f"#   {c}" for c in command.split(" ;; ")]
    lines += ["#", f"duration_us_under_counters: {t * 1e6:.1f}"]
    lines += [f"{k}: {v:.4g}" for k, v in sorted(avg.items())]
    if "SQ_INSTS_VALU" in avg:
        issue_s = avg["SQ_INSTS_VALU"] * 4 / (simds * clock_ghz * 1e9)
        lines += [f"valu_issue_time_us (SQ_INSTS_VALU x 4 cycles / {simds} SIMDs at {clock_ghz} GHz): "
                  f"{issue_s * 1e6:.1f}",
                  f"valu_issue_fraction_of_duration: {issue_s / t:.3f}"]
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    cn = sub.add_parser("counters")
    cn.add_argument("--csv", nargs="+", required=True)
    cn.add_argument("--kernel", default="k_blend")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", default="k_blend")
    t.add_argument("--copy-mib", type=int, required=True)
    st = sub.add_parser("stats")
    st.add_argument("--csv", required=True)
    tt = sub.add_parser("traffic-table")
    tt.add_argument("--fetch", required=True)
    tt.add_argument("--write", required=True)
    tt.add_argument("--stats", required=True)
    tt.add_argument("--copy-mib", type=int, required=True)
    for p in (t, st, cn, tt):
        p.add_argument("--out", required=True)
        p.add_argument("--workload", default="")
        p.add_argument("--command", default="", help="commands that produced the input (';;'-separated)")
    a = ap.parse_args()
    if a.cmd == "traffic":
        res = summarise(a.fetch, a.write, a.kernel, a.copy_mib)
        res["copy_mib"] = a.copy_mib
        write_summary(res, a.kernel, a.out, a.command, a.workload)
    elif a.cmd == "counters":
        write_counters(a.csv, a.kernel, a.out, a.command, a.workload)
    elif a.cmd == "traffic-table":
        write_traffic_table(a.fetch, a.write, a.stats, a.copy_mib, a.out, a.command, a.workload)
    else:
        write_stats(a.csv, a.out, a.command, a.workload)
    print(open(a.out).read())


if __name__ == "__main__":
    main()
