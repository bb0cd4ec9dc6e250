"""Summaries of rocprofv3 output (kernel times and hardware counters) as short
markdown tables.

    python -m paper_2603_17711_amd.profile_summary kernels <results.db> [top]
    python -m paper_2603_17711_amd.profile_summary counters <counter_collection.csv> [regex]

`kernels` reads the SQLite database that `rocprofv3 --kernel-trace --stats`
writes and lists the kernels by total time.  `counters` reads the CSV that
`rocprofv3 --pmc ... --output-format csv` writes (one row per dispatch and
counter) and sums each counter per kernel, for the kernels whose name matches
the regex; for MFMA counters it adds the executed MFMA flops
(SQ_INSTS_VALU_MFMA_MOPS_F32 x 512), their rate over the summed dispatch
durations (when the CSV carries start and end timestamps) and the VALU
instructions issued per MFMA instruction.
"""
import csv
import re
import sqlite3
import sys
from collections import defaultdict


def kernels(db, top=16):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels"))
    out = ["| Kernel | Calls | Total ms | Average us | Share |", "|:--|--:|--:|--:|--:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        # the view reports microseconds
        out.append(f"| `{name[:90]}` | {calls} | {tot / 1e3:.2f} | {avg:.1f} | {pct:.1f}% |")
    return "\n".join(out)


def counters(path, pattern=r"k_apply"):
    rx = re.compile(pattern)
    acc = defaultdict(lambda: defaultdict(float))
    dur = defaultdict(dict)
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r.get("Kernel_Name") or r.get("kernel_name") or ""
            if not rx.search(name):
                continue
            key = name.split("(")[0]
            cname = r.get("Counter_Name") or r.get("counter_name")
            val = float(r.get("Counter_Value") or r.get("counter_value") or 0.0)
            acc[key][cname] += val
            did = r.get("Dispatch_Id") or r.get("dispatch_id")
            t0 = r.get("Start_Timestamp") or r.get("start_timestamp")
            t1 = r.get("End_Timestamp") or r.get("end_timestamp")
            dur[key][did] = (float(t1) - float(t0)) * 1e-9 if t0 and t1 else None
    out = []
    for k, cs in acc.items():
        n = len(dur[k])
        secs = [d for d in dur[k].values() if d is not None]
        out.append(f"### `{k}` ({n} dispatches)")
        out.append("| Counter | Sum | Per dispatch |")
        out.append("|:--|--:|--:|")
        for cn in sorted(cs):
            out.append(f"| {cn} | {cs[cn]:.6g} | {cs[cn] / max(n, 1):.6g} |")
        if "SQ_INSTS_VALU_MFMA_MOPS_F32" in cs:
            fl = cs["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512
            out.append(f"| executed MFMA flops (MOPS_F32 x 512) | {fl:.6g} | {fl / max(n, 1):.6g} |")
            if secs and len(secs) == n:
                out.append(f"| summed dispatch time (s) | {sum(secs):.6g} | "
                           f"{sum(secs) / max(n, 1):.6g} |")
                out.append(f"| executed MFMA rate (TFLOP/s) | {fl / sum(secs) / 1e12:.4g} | |")
        if "SQ_INSTS_VALU" in cs and cs.get("SQ_INSTS_MFMA"):
            out.append(f"| VALU instructions per MFMA | "
                       f"{cs['SQ_INSTS_VALU'] / cs['SQ_INSTS_MFMA']:.2f} | |")
        out.append("")
    return "\n".join(out)


def main(argv):
    if len(argv) >= 2 and argv[0] == "kernels":
        print(kernels(argv[1], int(argv[2]) if len(argv) > 2 else 16))
    elif len(argv) >= 2 and argv[0] == "counters":
        print(counters(argv[1], argv[2] if len(argv) > 2 else r"k_apply"))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
