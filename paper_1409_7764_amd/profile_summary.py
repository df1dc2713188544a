"""Summarise rocprofv3 output of a bench.py run into a short text record.

Inputs: the directory of a `rocprofv3 --kernel-trace --stats --output-format csv` run, and
optionally the directories of two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
`bench.py --calibrate-copy` (one plain 2 GiB device-to-device copy precedes the steps); without
them the record holds the kernel trace alone.
The counters are scaled by what they read for that copy (its true traffic is known), and
the per-launch HBM bytes of the named kernel are written to profiles/traffic.json under the
workload name, together with the hash of the kernel sources they were taken on.

    python -m paper_1409_7764_amd.profile_summary --workload rmat16-exact --kernel k_msb \\
        --kt DIR --fetch DIR --write DIR --cmd "..." --out profiles/k_msb_rmat16-exact.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 * 1024 ** 3


def _rows(d, pattern):
    files = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not files:
        raise SystemExit(f"no {pattern} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def counter_per_dispatch(d, counter):
    out = []
    for r in _rows(d, "*counter_collection.csv"):
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernel", required=True, help="substring of the dominant kernel's name")
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cmd", required=True, help="the commands that produced the inputs")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    stats = _rows(a.kt, "*kernel_stats.csv")
    stats.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    lines = [f"# {a.kernel} on {a.workload}", "", "Commands:", "", "```", a.cmd.strip(), "```", "",
             "## Kernel trace (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    avg_ms = None
    for r in stats[:12]:
        name = r["Name"]
        tot = float(r["TotalDurationNs"]) / 1e6
        avg = float(r["AverageNs"]) / 1e6
        lines.append(f"| `{name[:90]}` | {r['Calls']} | {tot:.3f} | {avg:.3f} | {float(r['Percentage']):.1f} |")
        if a.kernel in name and avg_ms is None:
            avg_ms = avg

    if not (a.fetch and a.write):
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return

    def factor(rows, truth_bytes):
        copies = [v for k, g, v in rows if "copyBuffer" in k and v > 1024]
        if not copies:
            raise SystemExit("calibration copy not found (run bench.py with --calibrate-copy)")
        return truth_bytes / (max(copies) * 1024)

    fr = counter_per_dispatch(a.fetch, "FETCH_SIZE")
    wr = counter_per_dispatch(a.write, "WRITE_SIZE")
    ff = factor(fr, COPY_BYTES)
    wf = factor(wr, COPY_BYTES)
    kf = [v for k, g, v in fr if a.kernel in k]
    kw = [v for k, g, v in wr if a.kernel in k]
    if not kf or not kw:
        raise SystemExit(f"kernel {a.kernel} not found in the counter runs")
    fetch_b = sum(kf) / len(kf) * 1024 * ff
    write_b = sum(kw) / len(kw) * 1024 * wf
    lines += ["", "## HBM traffic (rocprofv3 --pmc, KiB per dispatch, scaled by a plain 2 GiB copy)", "",
              f"* calibration: FETCH_SIZE read {max(v for k, g, v in fr if 'copyBuffer' in k):.0f} KiB and "
              f"WRITE_SIZE {max(v for k, g, v in wr if 'copyBuffer' in k):.0f} KiB for 2 GiB copied "
              f"-> fetch factor {ff:.3f}, write factor {wf:.3f}",
              f"* `{a.kernel}`: fetch {fetch_b / 1e9:.2f} GB + write {write_b / 1e9:.2f} GB = "
              f"{(fetch_b + write_b) / 1e9:.2f} GB per launch"]
    if avg_ms:
        lines.append(f"* average duration {avg_ms:.3f} ms -> {(fetch_b + write_b) / (avg_ms / 1e3) / 1e9:.1f} GB/s "
                     "of HBM traffic")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    sys.path.insert(0, ROOT)
    import bench
    tj = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(tj)) if os.path.exists(tj) else {}
    rec[a.workload] = {"kernel": a.kernel, "kernel_hash": bench.kernel_source_hash(),
                       "hbm_bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b, "write_bytes": write_b,
                       "fetch_factor": ff, "write_factor": wf, "avg_kernel_ms": avg_ms}
    with open(tj, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
