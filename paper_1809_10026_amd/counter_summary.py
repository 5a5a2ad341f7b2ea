"""Summarise rocprofv3 counter runs of ``kernel_profile`` as Markdown.

    python -m paper_1809_10026_amd.counter_summary --mfma DIR --trace DIR --mode fp64 --command "..."
    python -m paper_1809_10026_amd.counter_summary --waits DIR --command "..."

--mfma: a run with SQ_INSTS_VALU_MFMA_MOPS_{BF16,F32,F64}, SQ_VALU_MFMA_BUSY_CYCLES
and GRBM_GUI_ACTIVE.  The hardware counts MFMA work in units of 512 flops
(MOPS), so flops per dispatch = MOPS * 512; with the kernel's mean duration
from the kernel-trace run of the same workload (--trace) that gives the
achieved MFMA rate, compared with MI355X's dense peak for the precision.
The busy-cycle utilisation is sum(SQ_VALU_MFMA_BUSY_CYCLES) / (GRBM_GUI_ACTIVE
per XCD * SIMDs): rocprofv3 reports GRBM_GUI_ACTIVE summed over the 8 XCDs.

--waits: a run with SQ_WAVE_CYCLES, SQ_WAIT_ANY, SQ_WAIT_INST_ANY,
SQ_ACTIVE_INST_ANY, SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS (all in the
same wave-cycle units): the share of the waves' resident cycles spent
waiting on anything (memory, dependencies), waiting to issue, and issuing.
"""
from __future__ import annotations

import argparse
import csv
import os
from collections import defaultdict

from .profile_summary import kernel_class, read_stats, short

PEAK_TF = {"BF16": 2500.0, "F32": 157.3, "F64": 78.6}
MODE_PREC = {"bf16x3": "BF16", "fp32": "F32", "fp64": "F64"}
XCDS = 8
SIMDS = 256 * 4


def read_counters(d):
    per = defaultdict(lambda: defaultdict(list))
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            per[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return per


def mfma(args):
    prec = MODE_PREC[args.mode]
    per = read_counters(args.mfma)
    dur = {r["Name"]: float(r["AverageNs"]) for r in read_stats(args.trace)} if args.trace else {}
    out = [f"# MFMA activity: {args.title}", "", "Commands (run from the repository root):", ""]
    out += ["    " + c for c in args.command.split(";")]
    out += ["", f"Flops = SQ_INSTS_VALU_MFMA_MOPS_{prec} x 512 per dispatch; duration = mean from the kernel trace; "
            f"peak = MI355X dense {prec} MFMA, {PEAK_TF[prec]} TFLOP/s.  Busy = sum(SQ_VALU_MFMA_BUSY_CYCLES) / "
            f"(GRBM_GUI_ACTIVE / {XCDS} x {SIMDS} SIMDs).", "",
            "| kernel | class | dispatches | MFMA GFLOP/dispatch | mean us | TFLOP/s | of peak | MFMA busy |",
            "|---|---|---|---|---|---|---|---|"]
    for name, cs in sorted(per.items(), key=lambda kv: -sum(kv[1].get(f"SQ_INSTS_VALU_MFMA_MOPS_{prec}", [0]))):
        mops = cs.get(f"SQ_INSTS_VALU_MFMA_MOPS_{prec}", [])
        if not mops or sum(mops) == 0:
            continue
        n = len(mops)
        flops = sum(mops) / n * 512.0
        busy = sum(cs["SQ_VALU_MFMA_BUSY_CYCLES"]) / sum(cs["GRBM_GUI_ACTIVE"]) * XCDS / SIMDS
        us = dur.get(name, 0.0) / 1e3
        tf = flops / (us * 1e-6) / 1e12 if us else float("nan")
        out.append(f"| `{short(name, 90)}` | {kernel_class(name) or ''} | {n} | {flops / 1e9:.3f} | {us:.1f} | "
                   f"{tf:.1f} | {tf / PEAK_TF[prec]:.3f} | {busy:.3f} |")
    print("\n".join(out))


def waits(args):
    per = read_counters(args.waits)
    out = [f"# Wave cycles: {args.title}", "", "Commands (run from the repository root):", ""]
    out += ["    " + c for c in args.command.split(";")]
    out += ["", "Shares of SQ_WAVE_CYCLES (summed over the waves of a dispatch, same units): waiting on anything "
            "(memory or dependencies), waiting to issue, issuing any instruction, issuing VALU, issuing LDS.", "",
            "| kernel | class | dispatches | wait any | wait issue | active any | active VALU | active LDS |",
            "|---|---|---|---|---|---|---|---|"]
    for name, cs in sorted(per.items(), key=lambda kv: -sum(kv[1].get("SQ_WAVE_CYCLES", [0]))):
        cls = kernel_class(name)
        if cls is None or "SQ_WAVE_CYCLES" not in cs:
            continue
        wc = sum(cs["SQ_WAVE_CYCLES"])
        if wc == 0:
            continue
        f = lambda c: sum(cs.get(c, [0.0])) / wc
        out.append(f"| `{short(name, 90)}` | {cls} | {len(cs['SQ_WAVE_CYCLES'])} | {f('SQ_WAIT_ANY'):.2f} | "
                   f"{f('SQ_WAIT_INST_ANY'):.2f} | {f('SQ_ACTIVE_INST_ANY'):.2f} | {f('SQ_ACTIVE_INST_VALU'):.2f} | "
                   f"{f('SQ_ACTIVE_INST_LDS'):.2f} |")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mfma")
    ap.add_argument("--trace")
    ap.add_argument("--mode", default="bf16x3", choices=sorted(MODE_PREC))
    ap.add_argument("--waits")
    ap.add_argument("--title", default="FD-preconditioned PCG, d=3, p=4, 48 el/dir (ndof 6,375,000)")
    ap.add_argument("--command", required=True)
    args = ap.parse_args()
    if args.mfma:
        mfma(args)
    elif args.waits:
        waits(args)
    else:
        raise SystemExit("--mfma or --waits required")


if __name__ == "__main__":
    main()
