"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2311_04648_amd.profsum stats <run_kernel_stats.csv> [<run_kernel_trace.csv>]
        markdown table of per-kernel durations (the --stats summary) and, with
        the kernel trace, the per-schedule breakdown of a bench.py run (the
        bench runs its schedules one after another; they are told apart by
        the gaps between the dynamics-kernel launches)
    python -m paper_2311_04648_amd.profsum traffic <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv>
                                                   <copy_bytes> <kernel> <source> <workload> [<variant>]
        HBM bytes per launch of one kernel (of one template variant of it,
        named exactly as in the trace, when given) from FETCH_SIZE /
        WRITE_SIZE counter runs, each scaled by what the same counter reads
        for a plain copy of a known size (JSON on stdout)
    python -m paper_2311_04648_amd.profsum kernels <fetch.csv> <write.csv> <fetch_scale> <write_scale>
        markdown table of the mean HBM bytes per launch of every kernel of a
        run (FETCH_SIZE and WRITE_SIZE scaled by the given copy-probe factors)
"""
from __future__ import annotations

import collections
import csv
import json
import os
import sys

DYN_KERNELS = ("k_step_fused", "k_fold_integrate", "k_step_free")


def _name(raw):
    n = raw.replace("(anonymous namespace)::", "")
    n = n.split("(")[0]
    return n[5:] if n.startswith("void ") else n


def stats_table(path, top=25):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| {_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def segments(trace_path, gap_ns=5e6, top=8):
    rows = list(csv.DictReader(open(trace_path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    dyn = [i for i, r in enumerate(rows) if _name(r["Kernel_Name"]).startswith(DYN_KERNELS)]
    if not dyn:
        return ""
    segs, cur = [], [dyn[0]]
    for a, b in zip(dyn, dyn[1:]):
        if int(rows[b]["Start_Timestamp"]) - int(rows[a]["End_Timestamp"]) > gap_ns:
            segs.append(cur)
            cur = []
        cur.append(b)
    segs.append(cur)
    out = []
    for k, s in enumerate(segs):
        lo, hi = s[0], s[-1]
        d = collections.defaultdict(list)
        for r in rows[lo:hi + 1]:
            d[_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        span = (int(rows[hi]["End_Timestamp"]) - int(rows[lo]["Start_Timestamp"])) / 1e6
        out.append(f"\nSegment {k + 1}: {len(s)} dynamics launches over {span:.2f} ms "
                   f"({1e3 * span / len(s):.2f} us per step)\n")
        out.append("| kernel | calls | mean us | median us | total ms |\n|---|---|---|---|---|")
        for name, v in sorted(d.items(), key=lambda kv: -sum(kv[1]))[:top]:
            v.sort()
            out.append(f"| {name} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {v[len(v) // 2] / 1e3:.2f} | "
                       f"{sum(v) / 1e6:.2f} |")
    return "\n".join(out)


def _counter(path, kernel=None, variant=None):
    """Mean counter value (KiB) per dispatch of a kernel (of one template
    variant of it when `variant` names one exactly), or of the largest
    dispatch when no kernel is named (the copy probe)."""
    vals = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        key = r["Dispatch_Id"]
        vals[key] += float(r["Counter_Value"])
        names[key] = _name(r["Kernel_Name"])
    if kernel is None:
        return max(vals.values())
    if variant:
        sel = [v for k, v in vals.items() if names[k] == variant]
    else:
        sel = [v for k, v in vals.items() if names[k].startswith(kernel)]
    return sum(sel) / len(sel)


def traffic(fetch, write, cfetch, cwrite, copy_bytes, kernel, source, workload, variant=None):
    copy_bytes = float(copy_bytes)
    cf, cw = _counter(cfetch), _counter(cwrite)
    fs, ws = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    f, w = _counter(fetch, kernel, variant), _counter(write, kernel, variant)
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.dirname(here))
    from bench import kernel_sha
    return {
        "copy_probe": {"bytes_read": copy_bytes, "bytes_written": copy_bytes, "FETCH_SIZE_KiB": cf,
                       "WRITE_SIZE_KiB": cw, "fetch_scale": fs, "write_scale": ws},
        kernel: {"source": source, "variant": variant or kernel, "FETCH_SIZE_KiB": f, "WRITE_SIZE_KiB": w,
                 "bytes_per_launch": f * 1024.0 * fs + w * 1024.0 * ws, "workload": workload,
                 "kernel_sha": kernel_sha(os.path.join(here, "csrc", source), kernel)},
    }


def kernels_traffic(fetch, write, fetch_scale, write_scale, top=20):
    def per_kernel(path):
        vals = collections.defaultdict(float)
        names = {}
        for r in csv.DictReader(open(path)):
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
            names[r["Dispatch_Id"]] = _name(r["Kernel_Name"])
        agg = collections.defaultdict(list)
        for d, v in vals.items():
            agg[names[d]].append(v)
        return agg
    f, w = per_kernel(fetch), per_kernel(write)
    fs, ws = float(fetch_scale), float(write_scale)
    rows = []
    for k in set(f) | set(w):
        fv, wv = f.get(k, []), w.get(k, [])
        fm = sum(fv) / max(len(fv), 1) * 1024.0 * fs / 1e6
        wm = sum(wv) / max(len(wv), 1) * 1024.0 * ws / 1e6
        rows.append((k, max(len(fv), len(wv)), fm, wm))
    rows.sort(key=lambda r: -(r[2] + r[3]) * r[1])
    out = ["| kernel | dispatches | read MB / launch | written MB / launch | HBM MB / launch |",
           "|---|---|---|---|---|"]
    for k, n, a, b in rows[:top]:
        out.append(f"| {k} | {n} | {a:.2f} | {b:.2f} | {a + b:.2f} |")
    return "\n".join(out)


def main(argv):
    if argv[0] == "stats":
        print(stats_table(argv[1]))
        if len(argv) > 2:
            print(segments(argv[2]))
    elif argv[0] == "kernels":
        print(kernels_traffic(*argv[1:5]))
    elif argv[0] == "traffic":
        print(json.dumps(traffic(*argv[1:10]), indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
