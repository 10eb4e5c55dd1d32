"""Summaries of rocprofv3 output for the committed profiles.

Three summaries, all from CSV output (``rocprofv3 ... -f csv -d DIR -o NAME``):

* ``trace``: the per-kernel statistics of a ``--kernel-trace --stats`` run
  (``NAME_kernel_stats.csv``) as a Markdown table.
* ``traffic``: HBM bytes per dispatch of one kernel from two PMC runs
  (``--pmc FETCH_SIZE``, then ``--pmc WRITE_SIZE``; KiB per dispatch),
  each scaled by what the same counter reads for a plain copy kernel of
  known size (``python -m paper_2405_16634_amd.profile_copy``, which copies
  ``--mb`` MiB per dispatch): factor = bytes the copy must move / bytes the
  counter reports.  Written as JSON with the digest of the traversal sources
  the counters were taken on; bench.py reports the figure only while the
  digest matches.
* ``sq``: instruction counters (SQ_INSTS_VALU, ...) per dispatch of one
  kernel, and the fraction of the chip's wave64 vector-issue ceiling they
  take over the kernel's traced duration.
* ``moments``: the traffic of one moment-pass call (chunk pass plus
  straddler pass) on one workload, with their traced times and counters.

``python -m paper_2405_16634_amd.profiling trace --csv F --cmd "..." --out F``
``python -m paper_2405_16634_amd.profiling traffic --fetch F --write F
    --cal-fetch F --cal-write F --mb 512 --kernel REGEX --cmd "..." --out F``
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
TRAVERSAL_SOURCES = [os.path.join(HERE, "csrc", "traverse.hip"),
                     os.path.join(HERE, "csrc", "epilogue.h"),
                     os.path.join(HERE, "csrc", "layout.h"),
                     os.path.join(HERE, "csrc", "wave.h")]


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed (string
    literals in these sources hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def traversal_digest() -> str:
    """Digest of the code (comments and layout ignored) of the sources that
    define the traversal kernel."""
    h = hashlib.sha256()
    for p in TRAVERSAL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _grid(r) -> int:
    """Threads in the dispatch (PMC CSV: Grid_Size; kernel trace: Grid_Size_X)."""
    return int(float(r.get("Grid_Size") or r.get("Grid_Size_X") or 0))


def _match(r, rx, grid) -> bool:
    """The row is a dispatch of a kernel matching rx (and of `grid` threads,
    when given: one workload among several that the command ran)."""
    return bool(rx.search(r["Kernel_Name"])) and (grid is None or _grid(r) == grid)


def counter_per_dispatch(path: str, counter: str, kernel: str, grid=None) -> tuple[float, int]:
    """Mean value of `counter` over the dispatches of kernels matching the
    regex `kernel` (one row per dispatch and counter; only dispatches of
    `grid` threads when given), and the count."""
    rx = re.compile(kernel)
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if r["Counter_Name"] == counter and _match(r, rx, grid)]
    if not vals:
        raise ValueError(f"{path}: no {counter} rows for kernels matching {kernel!r}")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, mb, kernel, cmd, grid=None):
    copy_kib = mb * 1024.0  # each copy dispatch reads and writes this much
    cal = "copyBuffer|elementwise_kernel|copy"
    cf, ncf = counter_per_dispatch(cal_fetch_csv, "FETCH_SIZE", cal)
    cw, ncw = counter_per_dispatch(cal_write_csv, "WRITE_SIZE", cal)
    # the calibration CSV may hold a small setup kernel too: use the
    # dispatches that moved about the copy's size
    rx = re.compile(cal)
    big_f = [float(r["Counter_Value"]) for r in _rows(cal_fetch_csv)
             if r["Counter_Name"] == "FETCH_SIZE" and rx.search(r["Kernel_Name"])
             and float(r["Counter_Value"]) > 0.1 * copy_kib]
    big_w = [float(r["Counter_Value"]) for r in _rows(cal_write_csv)
             if r["Counter_Name"] == "WRITE_SIZE" and rx.search(r["Kernel_Name"])
             and float(r["Counter_Value"]) > 0.1 * copy_kib]
    if big_f:
        cf, ncf = sum(big_f) / len(big_f), len(big_f)
    if big_w:
        cw, ncw = sum(big_w) / len(big_w), len(big_w)
    f_fetch = copy_kib / cf
    f_write = copy_kib / cw
    kf, nf = counter_per_dispatch(fetch_csv, "FETCH_SIZE", kernel, grid)
    kw, nw = counter_per_dispatch(write_csv, "WRITE_SIZE", kernel, grid)
    read_b = kf * 1024.0 * f_fetch
    write_b = kw * 1024.0 * f_write
    return {
        "kernel": kernel,
        "grid_threads": grid,
        "source_sha": traversal_digest(),
        "bytes_per_launch": round(read_b + write_b),
        "read_bytes_per_launch": round(read_b),
        "write_bytes_per_launch": round(write_b),
        "fetch_kib_per_dispatch": round(kf, 3), "fetch_dispatches": nf,
        "write_kib_per_dispatch": round(kw, 3), "write_dispatches": nw,
        "calibration": {"copy_mib_per_dispatch": mb,
                        "fetch_kib_per_copy": round(cf, 3), "fetch_factor": round(f_fetch, 4),
                        "write_kib_per_copy": round(cw, 3), "write_factor": round(f_write, 4),
                        "copy_dispatches": [ncf, ncw]},
        "command": cmd,
    }


def moments(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, mb, chunk_grid, strad_grid,
            cmd, sq_csv=None, trace_csv=None):
    """HBM bytes of one moment-pass call on one workload: its chunk pass
    and its straddler pass (dispatches of the given grid sizes), each from
    the two traffic counters scaled as in `traffic`; with a kernel trace
    and SQ counters, each pass's time and instructions too."""
    parts = {}
    for name, rx, grid in (("chunk", r"k_moments_chunk<[0-9], false>", chunk_grid),
                           ("straddler", r"k_moments_strad<false>", strad_grid)):
        d = traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, mb, rx, cmd, grid)
        part = {k: d[k] for k in ("kernel", "grid_threads", "bytes_per_launch",
                                   "read_bytes_per_launch", "write_bytes_per_launch",
                                   "fetch_dispatches", "write_dispatches")}
        if trace_csv:
            r_ = re.compile(rx)
            durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
                    for r in _rows(trace_csv) if _match(r, r_, grid)]
            part["trace_avg_us"] = round(sum(durs) / len(durs) * 1e6, 2)
            part["gb_per_s"] = round(d["bytes_per_launch"] / (sum(durs) / len(durs)) / 1e9, 1)
        if sq_csv:
            r_ = re.compile(rx)
            per = {}
            for r in _rows(sq_csv):
                if _match(r, r_, grid):
                    per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            part["sq"] = {k: round(sum(v) / len(v), 1) for k, v in per.items()}
        parts[name] = part
        calib = d["calibration"]
    out = {"parts": parts, "calibration": calib,
           "bytes_per_call": parts["chunk"]["bytes_per_launch"] + parts["straddler"]["bytes_per_launch"],
           "command": cmd}
    if trace_csv:
        t = parts["chunk"]["trace_avg_us"] + parts["straddler"]["trace_avg_us"]
        out["trace_us_per_call"] = round(t, 2)
        out["gb_per_s"] = round(out["bytes_per_call"] / (t * 1e-6) / 1e9, 1)
    return out


# Issue ceiling of one MI355X for wave64 vector instructions: 256 CUs x 4
# SIMDs, each issuing one wave64 instruction per 4 cycles (16 lanes), 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def sq(csv_paths, kernel: str, trace_csv: str, cmd: str, grid=None) -> dict:
    """Instruction counters (and derived metrics such as VALUBusy) per
    dispatch of the kernels matching `kernel` (of `grid` threads when
    given), from one or more --pmc runs, with the kernels' average duration
    from a kernel trace of the same command (kernel_trace CSV)."""
    rx = re.compile(kernel)
    per = {}
    for path in ([csv_paths] if isinstance(csv_paths, str) else csv_paths):
        for r in _rows(path):
            if _match(r, rx, grid):
                per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = {k: round(sum(v) / len(v), 3) for k, v in per.items()}
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
            for r in _rows(trace_csv) if _match(r, rx, grid)]
    avg = sum(durs) / len(durs)
    d = {"kernel": kernel, "grid_threads": grid, "source_sha": traversal_digest(),
         "per_dispatch": out,
         "dispatches": len(next(iter(per.values()))), "trace_avg_s": avg,
         "valu_issue_peak_per_s": VALU_ISSUE_PEAK, "command": cmd}
    if "SQ_INSTS_VALU" in out:
        d["valu_issue_frac"] = round(out["SQ_INSTS_VALU"] / avg / VALU_ISSUE_PEAK, 4)
    return d


def trace_markdown(stats_csv: str, title: str, cmd: str, groups=(), top: int = 25,
                   trace_csv=None, dispatch_groups=()) -> str:
    """groups: (label, regex) pairs; each gets the call-weighted average
    duration of the kernels whose names match.  dispatch_groups: (label,
    regex, grid) triples, averaged over the dispatches of `grid` threads in
    the per-dispatch trace (trace_csv): one workload among several that the
    command ran."""
    rows = _rows(stats_csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
           "```", cmd, "```", "",
           "Kernel statistics (rocprofv3 --kernel-trace --stats; durations in microseconds):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if groups:
        out += ["", "Kernel groups (all template instances whose names match):", "",
                "| group | regex | calls | average us |", "|---|---|---|---|"]
        for label, rx in groups:
            m = [r for r in rows if re.search(rx, r["Name"])]
            calls = sum(int(r["Calls"]) for r in m)
            tot = sum(float(r["TotalDurationNs"]) for r in m)
            avg = tot / calls / 1e3 if calls else float("nan")
            out.append(f"| {label} | `{rx}` | {calls} | {avg:.2f} |")
    if dispatch_groups:
        trows = _rows(trace_csv)
        out += ["", "Dispatches of one workload (kernel trace rows of the given grid size):", "",
                "| group | regex | grid threads | calls | average us |", "|---|---|---|---|---|"]
        for label, rx, grid in dispatch_groups:
            r_ = re.compile(rx)
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                 for r in trows if _match(r, r_, grid)]
            avg = sum(d) / len(d) if d else float("nan")
            out.append(f"| {label} | `{rx}` | {grid} | {len(d)} | {avg:.2f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--title", default="Kernel trace")
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--group", action="append", default=[], metavar="LABEL=REGEX")
    t.add_argument("--trace", help="kernel_trace CSV (per dispatch), for --dispatch-group")
    t.add_argument("--dispatch-group", action="append", default=[], metavar="LABEL=REGEX@GRID")
    q = sub.add_parser("traffic")
    for k in ("fetch", "write", "cal_fetch", "cal_write"):
        q.add_argument("--" + k.replace("_", "-"), required=True)
    q.add_argument("--mb", type=int, default=512)
    q.add_argument("--kernel", required=True)
    q.add_argument("--grid", type=int, default=None, help="only dispatches of this many threads")
    q.add_argument("--cmd", required=True)
    q.add_argument("--out", required=True)
    c = sub.add_parser("sq")
    c.add_argument("--csv", required=True, action="append")
    c.add_argument("--trace", required=True, help="kernel_trace CSV of the same workload")
    c.add_argument("--kernel", required=True)
    c.add_argument("--grid", type=int, default=None, help="only dispatches of this many threads")
    c.add_argument("--cmd", required=True)
    c.add_argument("--out", required=True)
    m = sub.add_parser("moments")
    for k in ("fetch", "write", "cal_fetch", "cal_write"):
        m.add_argument("--" + k.replace("_", "-"), required=True)
    m.add_argument("--mb", type=int, default=512)
    m.add_argument("--chunk-grid", type=int, required=True)
    m.add_argument("--strad-grid", type=int, required=True)
    m.add_argument("--sq", default=None)
    m.add_argument("--trace", default=None)
    m.add_argument("--cmd", required=True)
    m.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.what == "trace":
        dg = []
        for g in a.dispatch_group:
            label, rest = g.split("=", 1)
            rx, grid = rest.rsplit("@", 1)
            dg.append((label, rx, int(grid)))
        text = trace_markdown(a.csv, a.title, a.cmd,
                              [tuple(g.split("=", 1)) for g in a.group],
                              trace_csv=a.trace, dispatch_groups=dg)
        with open(a.out, "w") as f:
            f.write(text)
    elif a.what == "moments":
        d = moments(a.fetch, a.write, a.cal_fetch, a.cal_write, a.mb, a.chunk_grid, a.strad_grid,
                    a.cmd, a.sq, a.trace)
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
            f.write("\n")
    elif a.what == "sq":
        d = sq(a.csv, a.kernel, a.trace, a.cmd, a.grid)
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
            f.write("\n")
    else:
        d = traffic(a.fetch, a.write, a.cal_fetch, a.cal_write, a.mb, a.kernel, a.cmd, a.grid)
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
            f.write("\n")
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
