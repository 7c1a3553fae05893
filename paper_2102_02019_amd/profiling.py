"""Reading and writing the HBM-traffic summaries kept under profiles/.

A summary records, for one kernel and workload, the FETCH_SIZE and WRITE_SIZE
counters of rocprofv3 (KiB per dispatch) together with the same counters read
for a plain device-to-device copy of known size, from which a scale factor
turns counter KiB into HBM bytes. It also records a hash of the kernel's
source file so that a summary taken on an older kernel is not reported.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_source(name: str) -> str:
    return os.path.join(ROOT, "paper_2102_02019_amd", "csrc", name)


def read_counter_csv(pattern: str) -> list:
    """Rows of the rocprofv3 counter_collection CSV files matching pattern."""
    rows = []
    for path in sorted(glob.glob(pattern, recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def kernel_matches(name: str, pattern: str) -> bool:
    """pattern is a plain substring, or several substrings joined by '*'
    that must appear in that order."""
    pos = 0
    for part in pattern.split("*"):
        k = name.find(part, pos)
        if k < 0:
            return False
        pos = k + len(part)
    return True


def counter_per_dispatch(rows: list, kernel_substr: str, counter: str) -> list:
    """Values of `counter` for each dispatch whose kernel name matches
    kernel_substr (summed over the counter's dimensions), in dispatch order."""
    per = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
        if not kernel_matches(name, kernel_substr) or r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per, key=lambda s: int(s))]


# the gather kernels (apply, RK stage, filter) and their launch code
GATHER_SOURCES = ("gather.hpp", "operators.hip", "common.hpp")


def tile_nodes() -> int:
    """LABFM_TILE_NODES as the public header defines it."""
    import re

    with open(os.path.join(ROOT, "include", "labfm.h")) as f:
        return int(re.search(r"#define LABFM_TILE_NODES (\d+)", f.read()).group(1))


def sources_hash(names=GATHER_SOURCES) -> str:
    """Hash of the gather kernels' sources and of the tile size they run on."""
    h = hashlib.sha256()
    for name in names:
        with open(kernel_source(name), "rb") as f:
            h.update(f.read())
    h.update(b"tile_nodes=%d" % tile_nodes())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, kernel_name: str = None):
    """HBM bytes per dispatch of `kernel` on `workload` from a committed
    summary, or None if there is none, it was taken on other source, or (when
    kernel_name is given) on another launch variant."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("source_hash") != sources_hash():
        return None
    if kernel_name is not None and not kernel_matches(kernel_name, s["kernel_name_contains"]) \
            and s["kernel_name_contains"] != kernel_name:
        return None
    return s.get("hbm_bytes_per_dispatch")


COPY_KERNEL = "copyBuffer"        # torch's device-to-device copy (a runtime blit)
FILL_KERNEL = "FillFunctor"       # torch's fill
CALIBRATION_BYTES = 1 << 30       # 1 GiB read by the copy, 1 GiB written by fill and copy


def traffic_summary(kernel_tag: str, kernel_substr: str, workload: str, fetch_glob: str,
                    write_glob: str, command: str, last: int = 0,
                    algorithmic_bytes: float = None) -> dict:
    """Summarise FETCH_SIZE / WRITE_SIZE of one kernel (the last `last`
    matching dispatches when last > 0), scaled by the same counters read for
    the 1 GiB calibration copy of a profile run."""
    fr = read_counter_csv(fetch_glob)
    wr = read_counter_csv(write_glob)
    copy_fetch = max(counter_per_dispatch(fr, COPY_KERNEL, "FETCH_SIZE"))
    copy_write = max(counter_per_dispatch(wr, COPY_KERNEL, "WRITE_SIZE"))
    f = counter_per_dispatch(fr, kernel_substr, "FETCH_SIZE")
    w = counter_per_dispatch(wr, kernel_substr, "WRITE_SIZE")
    if not f or not w:
        raise SystemExit(f"no dispatch of a kernel matching {kernel_substr!r}")
    if last > 0:
        f, w = f[-last:], w[-last:]
    fetch_factor = CALIBRATION_BYTES / (copy_fetch * 1024.0)
    write_factor = CALIBRATION_BYTES / (copy_write * 1024.0)
    fkib = sum(f) / len(f)
    wkib = sum(w) / len(w)
    return {
        "kernel": kernel_tag,
        "kernel_name_contains": kernel_substr,
        "workload": workload,
        "dispatches": {"fetch": len(f), "write": len(w)},
        "fetch_kib_per_dispatch": fkib,
        "write_kib_per_dispatch": wkib,
        "copy_calibration": {"bytes": CALIBRATION_BYTES, "fetch_kib": copy_fetch,
                             "write_kib": copy_write, "fetch_factor": fetch_factor,
                             "write_factor": write_factor},
        "hbm_bytes_per_dispatch": fkib * 1024.0 * fetch_factor + wkib * 1024.0 * write_factor,
        "algorithmic_bytes_per_dispatch": algorithmic_bytes,
        "source_hash": sources_hash(),
        "command": command,
    }


def kernel_stats_markdown(stats_csv: str, top: int = 12) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary (short names)."""
    import re

    rows = read_counter_csv(stats_csv)
    lines = ["| kernel | calls | mean us | min us | max us | share % |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = re.sub(r"\(anonymous namespace\)::|labfm::", "", r["Name"])
        name = re.sub(r"\((int|double|float|void|signed|long|labfm|at|std).*$", "", name)
        lines.append(f"| `{name[:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def kernel_trace_markdown(trace_csv: str, min_grid: int = 0, top: int = 12,
                          max_grid: int = 0) -> str:
    """Markdown table of per-kernel durations from a rocprofv3 --kernel-trace
    CSV, counting only dispatches with Grid_Size_X >= min_grid (and <= max_grid
    when given), to separate the launches of one node set from those of
    other sizes in the same run."""
    import re

    rows = read_counter_csv(trace_csv)
    acc = {}
    for r in rows:
        g = int(r["Grid_Size_X"])
        if g < min_grid or (max_grid and g > max_grid):
            continue
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        acc.setdefault(r["Kernel_Name"], []).append(d)
    total = sum(sum(v) for v in acc.values()) or 1.0
    order = sorted(acc.items(), key=lambda kv: -sum(kv[1]))
    lines = ["| kernel | calls | mean us | min us | max us | share % |",
             "|---|---:|---:|---:|---:|---:|"]
    for name, v in order[:top]:
        name = re.sub(r"\(anonymous namespace\)::|labfm::", "", name)
        name = re.sub(r"\((int|double|float|void|signed|long|labfm|at|std|Tiles|BuildArgs).*$", "",
                      name)
        lines.append(f"| `{name[:80]}` | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | "
                     f"{max(v):.1f} | {100.0 * sum(v) / total:.2f} |")
    return "\n".join(lines)


def counters_markdown(csv_globs: list, kernel_substr: str, units: float = 0.0,
                      last: int = 0) -> str:
    """Markdown table of the counters of one kernel over several rocprofv3
    --pmc passes (one glob per pass): the mean per dispatch of each counter
    (summed over its dimensions) and, when `units` is given, per unit of
    work (per node, say). `last` > 0 keeps the last matching dispatches of
    each pass only."""
    means = {}
    for g in csv_globs:
        rows = read_counter_csv(g)
        names = sorted({r.get("Counter_Name") for r in rows})
        for c in names:
            vals = counter_per_dispatch(rows, kernel_substr, c)
            if last > 0:
                vals = vals[-last:]
            if vals:
                means[c] = (sum(vals) / len(vals), len(vals))
    if not means:
        raise SystemExit(f"no dispatch of a kernel matching {kernel_substr!r}")
    head = "| counter | dispatches | mean per dispatch |" + (" per unit |" if units else "")
    sep = "|---|---:|---:|" + ("---:|" if units else "")
    lines = [head, sep]
    for c, (v, n) in sorted(means.items()):
        row = f"| `{c}` | {n} | {v:.6g} |"
        if units:
            row += f" {v / units:.4g} |"
        lines.append(row)
    return "\n".join(lines)


def main(argv=None) -> None:
    """Command line: write a traffic summary (JSON) or a kernel-trace table
    (markdown) under profiles/ from rocprofv3 CSV output."""
    import argparse

    ap = argparse.ArgumentParser(prog="python -m paper_2102_02019_amd.profiling")
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("traffic", help="FETCH_SIZE / WRITE_SIZE summary of one kernel")
    t.add_argument("--tag", required=True, help="short kernel tag, e.g. rk_stage_f64")
    t.add_argument("--match", required=True, help="kernel name pattern ('*' joins parts)")
    t.add_argument("--workload", required=True)
    t.add_argument("--fetch", required=True, help="glob of the FETCH_SIZE counter CSV files")
    t.add_argument("--write", required=True, help="glob of the WRITE_SIZE counter CSV files")
    t.add_argument("--last", type=int, default=0, help="use the last N matching dispatches")
    t.add_argument("--algorithmic-bytes", type=float, default=None)
    t.add_argument("--command", required=True, help="the rocprofv3 commands, for the record")
    k = sub.add_parser("stats", help="markdown table of a --stats kernel summary")
    k.add_argument("--csv", required=True, help="glob of the kernel_stats CSV file")
    k.add_argument("--top", type=int, default=14)
    g = sub.add_parser("trace", help="markdown table of a --kernel-trace CSV, large grids only")
    g.add_argument("--csv", required=True, help="glob of the kernel_trace CSV file")
    g.add_argument("--min-grid", type=int, default=0, help="smallest Grid_Size_X counted")
    g.add_argument("--max-grid", type=int, default=0, help="largest Grid_Size_X counted")
    g.add_argument("--top", type=int, default=14)
    c = sub.add_parser("counters", help="markdown table of one kernel's --pmc counters")
    c.add_argument("--csv", required=True, nargs="+",
                   help="one glob of counter_collection CSV files per pass")
    c.add_argument("--match", required=True, help="kernel name pattern ('*' joins parts)")
    c.add_argument("--units", type=float, default=0.0, help="work units per dispatch")
    c.add_argument("--last", type=int, default=0)
    a = ap.parse_args(argv)
    if a.what == "traffic":
        s = traffic_summary(a.tag, a.match, a.workload, a.fetch, a.write, a.command, a.last,
                            a.algorithmic_bytes)
        path = os.path.join(PROFILES, f"{a.tag}_{a.workload}_traffic.json")
        with open(path, "w") as f:
            json.dump(s, f, indent=1)
        print(path, s["hbm_bytes_per_dispatch"])
    elif a.what == "counters":
        print(counters_markdown(a.csv, a.match, a.units, a.last))
    elif a.what == "trace":
        print(kernel_trace_markdown(a.csv, a.min_grid, a.top, a.max_grid))
    else:
        print(kernel_stats_markdown(a.csv, a.top))


if __name__ == "__main__":
    main()
