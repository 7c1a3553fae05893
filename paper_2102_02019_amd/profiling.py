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


def counter_per_dispatch(rows: list, kernel_substr: str, counter: str) -> list:
    """Values of `counter` for each dispatch whose kernel name contains
    kernel_substr (summed over the counter's dimensions)."""
    per = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
        if kernel_substr not in name or r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per, key=lambda s: int(s))]


def load_traffic(kernel: str, workload: str, source: str):
    """HBM bytes per dispatch of `kernel` on `workload` from a committed
    summary, or None if there is none or it was taken on other source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("source_hash") != source_hash(source):
        return None
    return s.get("hbm_bytes_per_dispatch")


COPY_KERNEL = "copyBuffer"        # torch's device-to-device copy (a runtime blit)
FILL_KERNEL = "FillFunctor"       # torch's fill
CALIBRATION_BYTES = 1 << 30       # 1 GiB read by the copy, 1 GiB written by fill and copy


def traffic_summary(kernel_tag: str, kernel_substr: str, workload: str, fetch_glob: str,
                    write_glob: str, source: str, command: str) -> dict:
    """Summarise FETCH_SIZE / WRITE_SIZE of one kernel, scaled by the same
    counters read for the 1 GiB calibration copy of a profile run."""
    fr = read_counter_csv(fetch_glob)
    wr = read_counter_csv(write_glob)
    copy_fetch = max(counter_per_dispatch(fr, COPY_KERNEL, "FETCH_SIZE"))
    copy_write = max(counter_per_dispatch(wr, COPY_KERNEL, "WRITE_SIZE"))
    f = counter_per_dispatch(fr, kernel_substr, "FETCH_SIZE")
    w = counter_per_dispatch(wr, kernel_substr, "WRITE_SIZE")
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
        "source_hash": source_hash(source),
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
