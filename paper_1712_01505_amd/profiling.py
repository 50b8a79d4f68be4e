"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1712_01505_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1712_01505_amd.profiling traffic <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir>
                                              <copy_mib> <out.json> "<commands>"

    python -m paper_1712_01505_amd.profiling shapes <trace_dir> <fetch_dir> <write_dir> <case_log>
                                              <copy_fetch_dir> <copy_write_dir> <copy_mib> <out.md> "<commands>"

``shapes`` pairs the stencil dispatches of ``profile_cases shapes`` (three per
launch shape, in the order the case printed its JSON lines) with their
duration (``--kernel-trace``) and calibrated HBM bytes, against the
compulsory bytes the case states.
``stats`` turns a ``--kernel-trace --stats`` kernel_stats CSV into a short
markdown table.  ``traffic`` reads the counter_collection CSVs of four
``--pmc`` runs (FETCH_SIZE and WRITE_SIZE of the benchmark, then of the
calibration copy) and writes, per kernel, the mean KiB per dispatch and the
HBM bytes per dispatch after scaling each counter by known-copy-bytes /
counter-reading of the copy kernel.  The summary records a hash of the
kernel sources; the benchmark reports the traffic only while it matches.
"""
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/wl_stencil.hip", "csrc/wl_stencil_kern.h", "csrc/wl_stencil_dev.h", "csrc/wl_brick.h",
                  "csrc/wl_brick_multi.hip",
                  "csrc/wl_hop.h", "csrc/wl_hop16.h", "csrc/wl_common.h", "csrc/wl_blas.hip"]


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name):
    return name.split("(")[0].replace("void ", "").strip()


def stats(csv_path, out_md, command):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:25]:
        lines.append("| {} | {} | {:.3f} | {:.2f} | {:.2f} | {:.2f} | {:.2f} |".format(
            short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    open(out_md, "w").write("\n".join(lines) + "\n")


def _counter_means(d, counter):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    acc = defaultdict(list)
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] == counter:
                acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib, out_json, command):
    f, nf = _counter_means(fetch_dir, "FETCH_SIZE")
    w, _ = _counter_means(write_dir, "WRITE_SIZE")
    cf, _ = _counter_means(cfetch_dir, "FETCH_SIZE")
    cw, _ = _counter_means(cwrite_dir, "WRITE_SIZE")
    copy_kib = float(copy_mib) * 1024.0
    kf = copy_kib / cf["wl::stream_copy_kernel"]
    kw = copy_kib / cw["wl::stream_copy_kernel"]
    kernels = {}
    for k in sorted(set(f) | set(w)):
        if k.startswith("wl::") and any(n in k for n in ("stencil", "twalk", "brick", "multi", "blas")):
            fb = f.get(k, 0.0) * kf * 1024
            wb = w.get(k, 0.0) * kw * 1024
            kernels[k] = {"dispatches": nf.get(k, 0), "FETCH_SIZE_KiB": round(f.get(k, 0.0), 1),
                          "WRITE_SIZE_KiB": round(w.get(k, 0.0), 1), "hbm_read_bytes": round(fb),
                          "hbm_write_bytes": round(wb), "hbm_bytes": round(fb + wb)}
    out = {"command": command, "copy_calibration": {"copy_MiB": copy_mib, "FETCH_SIZE_KiB": cf["wl::stream_copy_kernel"],
                                                    "WRITE_SIZE_KiB": cw["wl::stream_copy_kernel"],
                                                    "fetch_factor": kf, "write_factor": kw},
           "source_hash": source_hash(), "kernels": kernels}
    json.dump(out, open(out_json, "w"), indent=1)


def _per_dispatch(d, counter):
    out = []
    for fn in glob.glob(os.path.join(d, "**", "*.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            k = r.get("Kernel_Name", "")
            if not any(n in k for n in ("stencil_kernel", "twalk_kernel", "brick_kernel")):
                continue
            if counter is None:
                if "End_Timestamp" in r and "Counter_Name" not in r:
                    out.append((int(r["Dispatch_Id"]), short(k), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
            elif r.get("Counter_Name") == counter:
                out.append((int(r["Dispatch_Id"]), short(k), float(r["Counter_Value"])))
    acc = {}
    for i, k, v in out:  # counters come per XCD or per shader engine: sum per dispatch
        acc.setdefault(i, [k, 0.0])[1] += v
    return [acc[i] for i in sorted(acc)]


def shapes(trace_dir, fetch_dir, write_dir, case_log, cfetch_dir, cwrite_dir, copy_mib, out_md, command):
    rows = [json.loads(l) for l in open(case_log) if l.startswith("{")]
    t = _per_dispatch(trace_dir, None)
    f = _per_dispatch(fetch_dir, "FETCH_SIZE")
    w = _per_dispatch(write_dir, "WRITE_SIZE")
    cf, _ = _counter_means(cfetch_dir, "FETCH_SIZE")
    cw, _ = _counter_means(cwrite_dir, "WRITE_SIZE")
    kf = float(copy_mib) * 1024.0 / cf["wl::stream_copy_kernel"]
    kw = float(copy_mib) * 1024.0 / cw["wl::stream_copy_kernel"]
    n = 3 * len(rows)
    if not (len(t) == len(f) == len(w) == n):
        raise SystemExit(f"dispatch counts differ: trace {len(t)} fetch {len(f)} write {len(w)} shapes x 3 = {n}")
    lines = ["# Launch shapes: time and HBM traffic per launch", "", f"Commands: `{command}`", "",
             f"Counters scaled by the copy calibration (FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f}); each shape "
             "is launched three times and the three are averaged.  `launch` = (block, rhs_per_thread, xcd_remap, "
             "variant, rhs_lanes, brick x, y, z, t_steps, wg_per_cu, rhs_major).", "",
             "| case | launch | kernel | us | HBM read MB | read / compulsory | HBM write MB | write / compulsory | "
             "achieved TB/s |", "|---|---|---|---|---|---|---|---|---|"]
    for j, r in enumerate(rows):
        sl = slice(3 * j, 3 * j + 3)
        us = sum(x[1] for x in t[sl]) / 3
        rb = sum(x[1] for x in f[sl]) / 3 * kf * 1024
        wb = sum(x[1] for x in w[sl]) / 3 * kw * 1024
        lines.append("| {} | {} | `{}` | {:.1f} | {:.0f} | {:.2f} | {:.0f} | {:.2f} | {:.2f} |".format(
            r["case"], tuple(r["launch"]), t[3 * j][0], us, rb / 1e6, rb / r["compulsory_read"], wb / 1e6,
            wb / r["compulsory_write"], (rb + wb) / (us * 1e-6) / 1e12))
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    elif sys.argv[1] == "shapes":
        shapes(*sys.argv[2:11])
    elif sys.argv[1] == "hash":
        print(source_hash())
