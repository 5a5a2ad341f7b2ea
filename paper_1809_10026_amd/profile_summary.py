"""Summarise rocprofv3 output of ``kernel_profile`` runs as a Markdown table.

    python -m paper_1809_10026_amd.profile_summary --stats DIR [--fetch DIR --write DIR]
        [--traffic-json FILE] --command "..." > summary.md

DIR is a rocprofv3 output directory written with ``--output-format csv -o run``
(``run_kernel_stats.csv`` for --stats, ``run_counter_collection.csv`` for the
counter runs).  FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are turned into
bytes with the factors measured on the calibration kernel of the same run
(an elementwise multiply reading and writing CALIB_BYTES each), so that
traffic = counter / factor.  --traffic-json writes the per-class traffic of
the hot kernels together with a hash of the kernel sources; bench.py reports
it only while the sources still match.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 256 * 1024 * 1024
CALIB_MATCH = "MulFunctor"  # torch's elementwise multiply kernel (the calibration copy)

# kernel-name fragments -> profiling class of the library (bench.py's names)
CLASSES = [
    ("mv_outer_dma_kernel", "mv_outer"), ("mv_outer_kernel", "mv_outer"),
    ("mv_inner_slab_kernel", "mv_inner2"), ("mv_inner12_kernel", "mv_inner2"), ("mv_inner1_kernel", "mv_inner1"),
    ("fd_slab_kernel", "fd_slab"),
    ("fd_strided_kernel", None),  # fd_space or fd_time by the FUSED argument
    ("fd_mode_bf16x3_kernel", None), ("fd_mode_kernel", None),
    ("update_xr_kernel", "vec"), ("update_p_kernel", "vec"), ("dot_kernel", "vec"),
    ("finalize_kernel", "reduce"),
    ("mapped_space_kernel", "mv_mapped_space"), ("mapped_time_kernel", "mv_mapped_time"),
    ("mapped_scale_kernel", "vec"), ("mapped_assemble_kernel", "setup"),
    ("lift_class_kernel", "lift"), ("err_reduce_kernel", "norms"), ("eval_mode_kernel", "norms"),
]


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


# position of the FUSED template argument (time kernel) in the FD kernels' argument lists
FUSED_ARG = {"fd_strided_kernel": 2, "fd_mode_bf16x3_kernel": 4, "fd_mode_kernel": 6}


def _mangled_template_args(name: str, frag: str):
    """Template arguments of an Itanium-mangled name that the profiler left
    mangled: integer (``Li4E``) and boolean (``Lb1E``) literals after ``frag``."""
    rest = name.split(frag + "I", 1)[1] if frag + "I" in name else ""
    return ["true" if v == "b1" else "false" if v == "b0" else v[1:]
            for v in re.findall(r"L(i\d+|b[01])E", rest.split("EEv", 1)[0])]


def kernel_class(name: str):
    for frag, cls in CLASSES:
        if frag in name:
            if cls is not None:
                return cls
            if frag + "<" in name:
                targs = [a.strip() for a in name.split(frag + "<", 1)[1].split(">", 1)[0].split(",")]
            else:
                targs = _mangled_template_args(name, frag)
            fused = len(targs) > FUSED_ARG[frag] and targs[FUSED_ARG[frag]] == "true"
            return "fd_time" if fused else "fd_space"
    return None


def short(name: str, width: int = 110) -> str:
    return name if len(name) <= width else name[:width]


def read_stats(d):
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        return list(csv.DictReader(f))


def read_counter(d, counter):
    per = defaultdict(list)
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
    return per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--traffic-json")
    ap.add_argument("--command", required=True, help="the rocprofv3 command lines that produced DIRs")
    ap.add_argument("--title", default="Kernel statistics")
    ap.add_argument("--top", type=int, default=16)
    args = ap.parse_args()

    rows = read_stats(args.stats)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {args.title}", "", "Commands (run from the repository root):", ""]
    out += ["    " + c for c in args.command.split(";")]
    out += ["", "Durations from `run_kernel_stats.csv` (ns).", "",
            "| kernel | class | calls | avg ns | min ns | max ns | total % |", "|---|---|---|---|---|---|---|"]
    for r in rows[: args.top]:
        out.append(f"| `{short(r['Name'])}` | {kernel_class(r['Name']) or ''} | {r['Calls']} | "
                   f"{float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']} | {float(r['Percentage']):.2f} |")
    traffic = {}
    if args.fetch and args.write:
        fetch = read_counter(args.fetch, "FETCH_SIZE")
        write = read_counter(args.write, "WRITE_SIZE")
        cal_f = [v for k, vs in fetch.items() if CALIB_MATCH in k for v in vs]
        cal_w = [v for k, vs in write.items() if CALIB_MATCH in k for v in vs]
        if not cal_f or not cal_w:
            raise SystemExit("calibration kernel not found in the counter runs")
        ff = (sum(cal_f) / len(cal_f)) / CALIB_BYTES
        fw = (sum(cal_w) / len(cal_w)) / CALIB_BYTES
        out += ["", f"Calibration (elementwise multiply, {CALIB_BYTES} B read and {CALIB_BYTES} B written per launch): "
                f"FETCH_SIZE reads {ff:.4f} x the bytes read, WRITE_SIZE {fw:.4f} x the bytes written "
                f"({len(cal_f)} dispatches).  Traffic below = counter / factor.", "",
                "| kernel | class | dispatches | fetch MB/dispatch | write MB/dispatch |", "|---|---|---|---|---|"]
        agg = defaultdict(lambda: [0, 0.0, 0.0])
        for name in sorted(set(fetch) | set(write), key=lambda k: -sum(fetch.get(k, [0]))):
            cls = kernel_class(name)
            if cls is None:
                continue
            fv, wv = fetch.get(name, []), write.get(name, [])
            n = min(len(fv), len(wv))
            if n == 0:
                continue
            fb = sum(fv[:n]) / n / ff
            wb = sum(wv[:n]) / n / fw
            out.append(f"| `{short(name, 90)}` | {cls} | {n} | {fb / 1e6:.2f} | {wb / 1e6:.2f} |")
            a = agg[cls]
            a[0] += n
            a[1] += fb * n
            a[2] += wb * n
        for cls, (n, fb, wb) in agg.items():
            traffic[cls] = {"dispatches": n, "fetch_bytes": fb / n, "write_bytes": wb / n}
    print("\n".join(out))
    if args.traffic_json and traffic:
        with open(args.traffic_json, "w") as f:
            json.dump({"source_sha256": source_hash(), "command": args.command, "classes": traffic}, f, indent=1)


if __name__ == "__main__":
    main()
