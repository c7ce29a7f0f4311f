"""Short text summaries of rocprofv3 CSV output (kernel statistics, HBM counters).

  python -m paper_2306_11544_amd.rocprof_summary stats <..._kernel_stats.csv> --command "<cmd>"
  python -m paper_2306_11544_amd.rocprof_summary pmc <counter_collection.csv>... --kernel k_force_cells
      --command "<cmd of the first csv>" --command ... [--candidates <per launch>]
  python -m paper_2306_11544_amd.rocprof_summary traffic --fetch <fetch counter_collection.csv>
      --write <write counter_collection.csv> --kernel k_force_cells --copy-kernel neg_kernel
      --copy-bytes <bytes read = bytes written by the copy> --command-fetch "<cmd>" --command-write "<cmd>"

`traffic` scales the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of a kernel by what the
same counters read for a streaming copy of known size, and records the SHA-256 of the
kernel source's code (comments and blank space removed) so a reader can tell whether the
figure still describes the current code.  A summary file may hold several blocks (one
per launch configuration), separated by blank lines.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import sys

SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "mech.hip")


def code_of(text: str) -> str:
    """The source without comments and blank space: edits to comments or layout leave
    it, and so the figures taken on it, unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    return " ".join("".join(out).split())


def source_sha256(path: str = SOURCE) -> str:
    """SHA-256 of a kernel source's code (comments and blank space removed)."""
    with open(path, encoding="utf-8") as f:
        return hashlib.sha256(code_of(f.read()).encode()).hexdigest()


def source_line(path: str = SOURCE) -> str:
    return f"source_sha256(csrc/{os.path.basename(path)} code): {source_sha256(path)}"


def _short(name: str) -> str:
    """Kernel name without return type and template arguments' noise."""
    s = name
    if s.startswith("void "):
        s = s[5:]
    return s if len(s) <= 110 else s[:107] + "..."


def last_dispatches(trace_path: str, kernel: str, n: int) -> str:
    """Mean, min and max duration of the last n dispatches (by start time) of the kernels
    whose name contains `kernel`, from a kernel-trace CSV: the launches a run times last."""
    d = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
         for r in csv.DictReader(open(trace_path)) if kernel in r["Kernel_Name"]]
    if len(d) < n:
        raise SystemExit(f"{len(d)} dispatches of {kernel!r}, fewer than {n}")
    last = [dt for _, dt in sorted(d)[-n:]]
    return (f"last {n} dispatches of {kernel}: mean {sum(last) / n / 1e3:.3f} us, "
            f"min {min(last) / 1e3:.3f}, max {max(last) / 1e3:.3f}")


def stats(path: str, command: str, top: int = 25, sources=(SOURCE,), last=None) -> str:
    """Per-kernel totals of a kernel-stats CSV; with last = (kernel-trace CSV, kernel, n)
    also the mean of that kernel's last n dispatches."""
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"command: {command}", *[source_line(x) for x in sources],
           f"kernels: {len(rows)}  total kernel time: {total / 1e6:.3f} ms", "",
           f"{'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  name"]
    for r in rows[:top]:
        out.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.3f} "
                   f"{float(r['MinNs']) / 1e3:10.3f} {float(r['MaxNs']) / 1e3:10.3f} "
                   f"{100.0 * float(r['TotalDurationNs']) / total:6.2f}  {_short(r['Name'])}")
    if last is not None:
        out += ["", last_dispatches(*last)]
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    """{kernel name: [counter value per dispatch, ...]} (values summed over the counter's
    instances within a dispatch)."""
    acc = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    by = collections.defaultdict(list)
    for key, v in acc.items():
        by[names[key]].append(v)
    return by


def _pick(by, sub: str):
    hits = {k: v for k, v in by.items() if sub in k}
    if not hits:
        raise SystemExit(f"no dispatch of a kernel matching {sub!r}")
    vals = [x for v in hits.values() for x in v]
    return sorted(hits), vals


def traffic(a) -> str:
    f_by = _per_dispatch(a.fetch, "FETCH_SIZE")
    w_by = _per_dispatch(a.write, "WRITE_SIZE")
    kn, kf = _pick(f_by, a.kernel)
    _, kw = _pick(w_by, a.kernel)
    cn, cf = _pick(f_by, a.copy_kernel)
    _, cw = _pick(w_by, a.copy_kernel)
    # the copy's largest dispatches are the calibration copies (other matches are small)
    cf_kib = max(cf)
    cw_kib = max(cw)
    sf = a.copy_bytes / (cf_kib * 1024.0)
    sw = a.copy_bytes / (cw_kib * 1024.0)
    kf_kib = sum(kf) / len(kf)
    kw_kib = sum(kw) / len(kw)
    fetch_b = kf_kib * 1024.0 * sf
    write_b = kw_kib * 1024.0 * sw
    lines = [
        f"command (FETCH_SIZE): {a.command_fetch}",
        f"command (WRITE_SIZE): {a.command_write}",
        source_line(a.source),
        f"kernel: {a.kernel}  ({len(kf)} dispatches; {'; '.join(_short(k) for k in kn)})",
        f"workload: {a.workload}",
        f"tuning: {a.tuning}",
        f"copy kernel: {'; '.join(_short(k) for k in cn)}  bytes read = bytes written = {a.copy_bytes}",
        f"copy FETCH_SIZE KiB/dispatch: {cf_kib:.1f}  scale: {sf:.4f}",
        f"copy WRITE_SIZE KiB/dispatch: {cw_kib:.1f}  scale: {sw:.4f}",
        f"kernel FETCH_SIZE KiB/dispatch (mean): {kf_kib:.1f}  min {min(kf):.1f} max {max(kf):.1f}",
        f"kernel WRITE_SIZE KiB/dispatch (mean): {kw_kib:.1f}  min {min(kw):.1f} max {max(kw):.1f}",
        f"fetch_bytes_per_launch: {fetch_b:.0f}",
        f"write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    return "\n".join(lines) + "\n"


def pmc(paths, kernel: str, commands, candidates=None, source=SOURCE) -> str:
    """Mean per dispatch of every counter in the counter-collection CSVs, for the
    dispatches of kernels whose name contains `kernel`; with `candidates` (the candidate
    pairs one launch tests, from the run's own counters) the summary records it, so that
    VALU instructions per tested candidate can be derived."""
    lines = [f"command: {c}" for c in commands]
    lines.append(source_line(source))
    lines.append(f"kernel: {kernel}")
    if candidates is not None:
        lines.append(f"candidates_per_launch: {candidates:.6g}")
    mean = {}
    for path in paths:
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        name = {}
        for r in csv.DictReader(open(path)):
            if kernel not in r["Kernel_Name"]:
                continue
            acc[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
            name[r["Dispatch_Id"]] = r["Kernel_Name"]
        for counter in sorted(acc):
            vals = list(acc[counter].values())
            mean[counter] = sum(vals) / len(vals)
            lines.append(f"{counter}: {mean[counter]:.6g}  ({len(vals)} dispatches)")
    # derived figures: lane use is thread-cycles of VALU work over 64 lanes of the
    # cycles with a VALU instruction issued; per candidate, a wave instruction counts
    # once per lane
    if "SQ_THREAD_CYCLES_VALU" in mean and mean.get("SQ_ACTIVE_INST_VALU"):
        util = mean["SQ_THREAD_CYCLES_VALU"] / (64.0 * mean["SQ_ACTIVE_INST_VALU"])
        lines.append(f"derived lane_utilisation: {util:.3f}")
        if candidates and "SQ_INSTS_VALU" in mean:
            per = mean["SQ_INSTS_VALU"] * 64.0 / candidates
            lines.append(f"derived valu_lane_insts_per_candidate: {per:.2f}")
            lines.append(f"derived active_valu_lane_insts_per_candidate: {per * util:.2f}")
    return "\n".join(lines) + "\n"


def sections(path: str):
    """The blocks of a summary file: one per profiled launch configuration, separated by
    blank lines."""
    return [b for b in open(path).read().split("\n\n") if b.strip()]


def read_traffic(path: str):
    """[(traffic bytes per launch, source sha256, workload, tuning), ...], one per block
    of a file of `traffic` summaries."""
    out = []
    for block in sections(path):
        vals = {}
        for line in block.splitlines():
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
        if "traffic_bytes_per_launch" in vals:
            sha = next((v for k, v in vals.items() if k.startswith("source_sha256(")), "")
            out.append((float(vals["traffic_bytes_per_launch"]), sha, vals.get("workload", ""),
                        vals.get("tuning", "")))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--source", action="append", default=None,
                   help="kernel source(s) whose code hash the summary records (default csrc/mech.hip)")
    s.add_argument("--last", nargs=3, metavar=("TRACE_CSV", "KERNEL", "N"), default=None,
                   help="also the mean of KERNEL's last N dispatches in the kernel-trace CSV")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--tuning", default="", help="launch configuration the run used, as K,W,U,G,L")
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--source", default=SOURCE, help="the kernel's source file (default csrc/mech.hip)")
    m = sub.add_parser("pmc")
    m.add_argument("csvs", nargs="+")
    m.add_argument("--kernel", required=True)
    m.add_argument("--command", action="append", default=[])
    m.add_argument("--candidates", type=float, default=None, help="candidate pairs tested per launch")
    m.add_argument("--source", default=SOURCE)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        last = None if a.last is None else (a.last[0], a.last[1], int(a.last[2]))
        sys.stdout.write(stats(a.csv, a.command, a.top, tuple(a.source or (SOURCE,)), last))
    elif a.cmd == "traffic":
        sys.stdout.write(traffic(a))
    else:
        sys.stdout.write(pmc(a.csvs, a.kernel, a.command, a.candidates, a.source))


if __name__ == "__main__":
    main()
