"""Summaries of rocprofv3 output for the profiles/ directory.

Reads the CSV files rocprofv3 writes (--kernel-trace --stats, and --pmc
FETCH_SIZE or WRITE_SIZE runs) and writes short text summaries:

  python -m paper_2404_10861_amd.profiling stats DIR --out FILE.md --cmd "..."
  python -m paper_2404_10861_amd.profiling traffic --fetch DIR --write DIR
        --copy-bytes B --kernel step_kernel --bytes-per-launch X
        --out FILE.json --md FILE.md --cmd "..." --cmd "..."
  python -m paper_2404_10861_amd.profiling counters --fetch DIR --write DIR
        --kernel NAME --bytes-per-launch X --md FILE.md --cmd "..."
  python -m paper_2404_10861_amd.profiling sq DIR1 DIR2 --kernel NAME
        --md FILE.md --cmd "..."

The traffic summary scales each counter by what the same counter reads for
the plain copy kernel of known size (bytes read, bytes written), giving HBM
bytes per launch of the step kernel.  The counters summary reports the raw
per-dispatch medians of one kernel (KiB) next to its algorithmic bytes, for
runs without the copy kernel (WRITE_SIZE reads 1.000 of the copy kernel's
written bytes, FETCH_SIZE 0.5000 of its read bytes, on MI355X).  The sq
summary derives, from SQ and GRBM counters of two passes, an estimate of
the VALU issue fraction, the mean resident waves per SIMD and the share of wave time spent
waiting (SQ_* cycle counters count 4-cycle units; GRBM_GUI_ACTIVE sums the
8 XCDs; 1,024 SIMDs).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2404_10861_amd", "csrc", f)
                  for f in ("hsga_kernels.hip", "hsga_device.hpp")]


QUERY_SOURCES = [os.path.join(ROOT, "paper_2404_10861_amd", "csrc", f)
                 for f in ("hsga_query.hip", "hsga_device.hpp")]


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed, so that a
    comment edit does not mark a profile stale (string literals in these
    files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash(sources=None) -> str:
    """Hash of the code (comments and layout aside) of the step kernel's
    sources, or of the given files."""
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def kernel_stats(d: str):
    rows = []
    with open(_find(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append(r)
    return rows


def counter_values(d: str, counter: str):
    """{kernel name: [value per dispatch]} of one counter."""
    out: dict[str, list[float]] = {}
    with open(_find(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _pick(values: dict, needle: str):
    keys = [k for k in values if needle in k]
    if not keys:
        raise KeyError(f"no kernel matching {needle!r}: {list(values)}")
    vals = []
    for k in keys:
        vals.extend(values[k])
    return keys, vals


def cmd_stats(a):
    rows = kernel_stats(a.dir)
    lines = [f"# rocprofv3 kernel statistics: {a.title}", "", "Command:", ""]
    for c in a.cmd:
        lines.append(f"    {c}")
    lines += ["", "| kernel | calls | average us | min us | max us | total ms | % |",
              "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


def cmd_traffic(a):
    fetch = counter_values(a.fetch, "FETCH_SIZE")
    write = counter_values(a.write, "WRITE_SIZE")
    _, cf = _pick(fetch, "probe_copy")
    _, cw = _pick(write, "probe_copy")
    copy_kib = a.copy_bytes / 1024.0
    f_factor = copy_kib / statistics.median(cf)
    w_factor = copy_kib / statistics.median(cw)
    names, sf = _pick(fetch, a.kernel)
    _, sw = _pick(write, a.kernel)
    k = a.dispatches_per_launch
    if k == 1:
        # the first dispatch of a run reads no outboxes; use the median
        fetch_kib, write_kib = statistics.median(sf), statistics.median(sw)
    else:
        # a launch (a generation) of k dispatches side by side: the mean
        # dispatch times k
        fetch_kib, write_kib = k * statistics.fmean(sf), k * statistics.fmean(sw)
    fetch_b = fetch_kib * 1024.0 * f_factor
    write_b = write_kib * 1024.0 * w_factor
    rec = {
        "kernel": a.kernel,
        "kernel_names": names,
        "kernel_hash": kernel_hash(),
        "fetch_kib_per_dispatch_median": statistics.median(sf),
        "write_kib_per_dispatch_median": statistics.median(sw),
        "dispatches": len(sf),
        "copy_bytes": a.copy_bytes,
        "copy_fetch_kib_median": statistics.median(cf),
        "copy_write_kib_median": statistics.median(cw),
        "fetch_scale": f_factor,
        "write_scale": w_factor,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": a.bytes_per_launch,
        "traffic_over_algorithmic": (fetch_b + write_b) / a.bytes_per_launch,
        "design_bytes_per_launch": a.design_bytes_per_launch,
        "commands": a.cmd,
    }
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# HBM traffic of `{a.kernel}`: {a.title}", "", "Commands:", ""]
    for c in a.cmd:
        lines.append(f"    {c}")
    lines += ["",
              f"- copy kernel of {a.copy_bytes} bytes: FETCH_SIZE {rec['copy_fetch_kib_median']:.0f} KiB, "
              f"WRITE_SIZE {rec['copy_write_kib_median']:.0f} KiB per dispatch -> scale "
              f"{f_factor:.4f} (fetch), {w_factor:.4f} (write)",
              f"- step kernel ({len(sf)} dispatches, median): FETCH_SIZE "
              f"{rec['fetch_kib_per_dispatch_median']:.0f} KiB, WRITE_SIZE "
              f"{rec['write_kib_per_dispatch_median']:.0f} KiB" +
              (f"; {k} dispatches per launch, counted as {k} x the mean dispatch"
               if k > 1 else ""),
              f"- HBM bytes per launch: read {fetch_b / 1e6:.1f} MB + write {write_b / 1e6:.1f} MB "
              f"= {(fetch_b + write_b) / 1e6:.1f} MB",
              f"- algorithmic bytes per launch: {a.bytes_per_launch / 1e6:.1f} MB; measured / "
              f"algorithmic = {rec['traffic_over_algorithmic']:.3f}"]
    if a.design_bytes_per_launch:
        lines.append(f"- design bytes per launch (what this code has to move): "
                     f"{a.design_bytes_per_launch / 1e6:.1f} MB; measured / design = "
                     f"{(fetch_b + write_b) / a.design_bytes_per_launch:.3f}")
    lines += [f"- kernel source hash: {rec['kernel_hash']}", ""]
    with open(a.md, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def cmd_counters(a):
    fetch = counter_values(a.fetch, "FETCH_SIZE")
    write = counter_values(a.write, "WRITE_SIZE")
    names, sf = _pick(fetch, a.kernel)
    _, sw = _pick(write, a.kernel)
    f_kib, w_kib = statistics.median(sf), statistics.median(sw)
    lines = [f"# HBM counters of `{a.kernel}`: {a.title}", "", "Commands:", ""]
    for c in a.cmd:
        lines.append(f"    {c}")
    lines += ["",
              f"- dispatches: {len(sf)} ({', '.join(n[:60] for n in names)})",
              f"- FETCH_SIZE median {f_kib:.1f} KiB per dispatch, WRITE_SIZE median "
              f"{w_kib:.1f} KiB per dispatch",
              f"- algorithmic bytes per dispatch: {a.bytes_per_launch / 1e6:.1f} MB; "
              f"WRITE_SIZE bytes / algorithmic = {w_kib * 1024 / a.bytes_per_launch:.3f}",
              f"- query kernel source hash: {kernel_hash(QUERY_SOURCES)}", ""]
    with open(a.md, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def cmd_sq(a):
    vals = {}
    names = []
    for d in a.dirs:
        with open(_find(d, "counter_collection.csv")) as f:
            per = {}
            for r in csv.DictReader(f):
                if a.kernel not in r["Kernel_Name"]:
                    continue
                if r["Kernel_Name"] not in names:
                    names.append(r["Kernel_Name"])
                per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for k, v in per.items():
            vals[k] = statistics.median(v)
    cycles = vals["GRBM_GUI_ACTIVE"] / 8            # per XCD
    simds = 1024
    valu = vals["SQ_ACTIVE_INST_VALU"] * 4 / (simds * cycles)
    waves = vals["SQ_WAVE_CYCLES"] * 4 / (simds * cycles)
    wait = vals["SQ_WAIT_INST_ANY"] / vals["SQ_WAVE_CYCLES"]
    per_wave = vals["SQ_INSTS_VALU"] / vals["SQ_WAVES"]
    lines = [f"# SQ counters of `{a.kernel}`: {a.title}", "", "Commands:", ""]
    for c in a.cmd:
        lines.append(f"    {c}")
    lines += ["", f"- kernel: {names[0][:90] if names else a.kernel}",
              "- medians per dispatch: " + ", ".join(f"{k} {v:.0f}" for k, v in sorted(vals.items())),
              f"- duration: {cycles:.0f} cycles per XCD ({cycles / 2.4e3:.1f} us at 2.4 GHz, "
              "counters on)",
              f"- VALU issue estimate: {100 * valu:.0f} % of SIMD cycles (SQ_ACTIVE_INST_VALU "
              "x 4 cycles; an upper estimate, since some wave64 VALU instructions issue in "
              f"fewer cycles); VALU instructions per wave: {per_wave:.0f}",
              f"- resident waves per SIMD (mean): {waves:.1f}",
              f"- wave time spent waiting (s_waitcnt): {100 * wait:.0f} %",
              f"- kernel source hash: {kernel_hash()}", ""]
    with open(a.md, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    if a.json:
        rec = {"kernel": a.kernel, "kernel_names": names, "kernel_hash": kernel_hash(),
               "valu_issue_estimate": valu, "valu_instructions_per_wave": per_wave,
               "resident_waves_per_simd": waves, "wave_time_waiting": wait,
               "medians_per_dispatch": vals, "commands": a.cmd}
        with open(a.json, "w") as f:
            json.dump(rec, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--cmd", action="append", default=[])
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--kernel", default="step_kernel")
    t.add_argument("--bytes-per-launch", type=float, required=True)
    t.add_argument("--design-bytes-per-launch", type=float, default=0.0)
    t.add_argument("--dispatches-per-launch", type=int, default=1,
                   help="dispatches that make one launch's work (a pool generation's "
                        "launch groups)")
    t.add_argument("--out", required=True)
    t.add_argument("--md", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--cmd", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True, help="a query kernel (hsga_query.hip)")
    c.add_argument("--bytes-per-launch", type=float, required=True)
    c.add_argument("--md", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--cmd", action="append", default=[])
    q = sub.add_parser("sq")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--kernel", required=True)
    q.add_argument("--md", required=True)
    q.add_argument("--json", default="", help="also write the figures as JSON")
    q.add_argument("--title", default="")
    q.add_argument("--cmd", action="append", default=[])
    a = ap.parse_args(argv)
    if a.what == "sq":
        cmd_sq(a)
        return
    if a.what == "stats":
        cmd_stats(a)
    elif a.what == "counters":
        cmd_counters(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    sys.exit(main())
