"""Text summaries of rocprofv3 output for the kernels of the library.

    python -m paper_2201_00804_amd.profsum stats TRACE_CSV STATS_CSV --command CMD
    python -m paper_2201_00804_amd.profsum traffic --kernel k_matvec \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --copy-bytes N --command CMD

    python -m paper_2201_00804_amd.profsum valu|issue --counters C.csv --trace TRACE_CSV \
        --command CMD [--command CMD2]

`stats` lists the per-kernel totals of `--kernel-trace --stats` and, for
each kernel, the mean over its working launches: the solver enqueues its
iterations in batches of four and launches queued after the device-side stop
flag was raised return at once (a few microseconds); launches shorter than a
quarter of the kernel's median are counted separately as idle.  `traffic` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per
dispatch) into bytes per launch, each scaled by the ratio of a plain copy
kernel's known bytes to what the same counter reads for it.

The library's HIP-event profile counts the same working launches, so the two
mean durations are comparable.
"""
import argparse
import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources whose change makes a stored traffic figure stale
TRAFFIC_SOURCES = {
    "k_matvec": ["paper_2201_00804_amd/csrc/pair.hip", "paper_2201_00804_amd/csrc/pairmath.h",
                 "paper_2201_00804_amd/csrc/common.h"],
}
IDLE_FRACTION = 0.25   # a launch under this share of the kernel's median is idle


def source_hash(kernel):
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    """'void ns::k<float, 5>(args)' -> 'k<float, 5>'."""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.replace("sibfa::", "")


def precision_of(name):
    return "mixed" if "<float" in name else "fp64"


def stats(args):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(args.trace)):
        per[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = list(csv.DictReader(open(args.stats)))
    total = sum(float(r["TotalDurationNs"]) for r in rows) / 1e3
    out = [f"# {args.title}", "", "Command:", "", "```", args.command, "```", ""]
    if args.note:
        out += [args.note, ""]
    out += [f"Total kernel time {total / 1e3:.3f} ms over {len(rows)} kernels.", "",
           "| kernel | calls | total us | avg us (rocprof) | % | working calls | "
           "working avg us | idle calls |",
           "|---|---|---|---|---|---|---|---|"]
    for r in rows[:args.top]:
        d = per.get(r["Name"], [])
        med = sorted(d)[len(d) // 2] if d else 0.0
        work = [x for x in d if x >= IDLE_FRACTION * med]
        wavg = sum(work) / len(work) if work else 0.0
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f}"
                   f" | {float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} | "
                   f"{len(work)} | {wavg:.2f} | {len(d) - len(work)} |")
    print("\n".join(out))


def counter_means(path, kernel):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if short(r["Kernel_Name"]).split("<")[0] == kernel:
            vals[precision_of(short(r["Kernel_Name"]))].append(float(r["Counter_Value"]))
    out = {}
    for p, v in vals.items():
        med = sorted(v)[len(v) // 2]
        work = [x for x in v if x >= IDLE_FRACTION * med]
        out[p] = (sum(work) / len(work), len(work), len(v))
    return out


def copy_value(path):
    v = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
         if "copyBuffer" in r["Kernel_Name"]]
    return sum(v) / len(v)


def traffic(args):
    f_copy = args.copy_bytes / (copy_value(args.copy_fetch) * 1024.0)
    w_copy = args.copy_bytes / (copy_value(args.copy_write) * 1024.0)
    fm = counter_means(args.fetch, args.kernel)
    wm = counter_means(args.write, args.kernel)
    out = [f"# HBM traffic of {args.kernel}, {args.workload}", "", "Commands:", "", "```"]
    out += args.command
    out += ["```", "",
            "FETCH_SIZE and WRITE_SIZE are KiB per dispatch.  A plain device copy of "
            f"{args.copy_bytes} bytes reads {copy_value(args.copy_fetch):.1f} KiB of FETCH_SIZE "
            f"and {copy_value(args.copy_write):.1f} KiB of WRITE_SIZE, so the counters are "
            f"scaled by {f_copy:.4f} (fetch) and {w_copy:.4f} (write) bytes per KiB/1024.  "
            "Means are over working launches (idle launches after the solver's stop flag "
            "excluded).", "",
            "| key | value |", "|---|---|",
            f"| kernel sources sha256[:16] | `{source_hash(args.kernel)}` |",
            f"| fetch scale | {f_copy:.5f} |", f"| write scale | {w_copy:.5f} |"]
    for p in sorted(fm):
        fk, nw, nall = fm[p]
        wk = wm.get(p, (0.0, 0, 0))[0]
        b = fk * 1024.0 * f_copy + wk * 1024.0 * w_copy
        out += [f"| FETCH_SIZE KiB ({p}) | {fk:.1f} ({nw} of {nall} launches) |",
                f"| WRITE_SIZE KiB ({p}) | {wk:.1f} |",
                f"| traffic bytes per launch ({p}) | {b:.0f} |"]
    print("\n".join(out))


# gfx950: 256 CUs x 4 SIMDs at 2.4 GHz; a wave64 VALU instruction occupies
# its SIMD for 4 cycles (16 lanes per cycle, FP32 unpacked and FP64 alike)
VALU_PEAK = 256 * 4 * 2.4e9 / 4


def valu(args):
    """VALU (and SALU) instructions per working dispatch from SQ_INSTS_VALU /
    SQ_INSTS_SALU, over each kernel's working mean duration in a kernel
    trace, against the issue peak."""
    inst = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(args.counters)):
        inst[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = collections.defaultdict(list)
    for r in csv.DictReader(open(args.trace)):
        dur[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) -
                                             int(r["Start_Timestamp"])) / 1e3)

    def working_mean(v):
        med = sorted(v)[len(v) // 2]
        w = [x for x in v if x >= IDLE_FRACTION * med]
        return sum(w) / len(w)

    rows = []
    for k, d in dur.items():
        if k not in inst or "SQ_INSTS_VALU" not in inst[k]:
            continue
        t = working_mean(d)
        nv = working_mean(inst[k]["SQ_INSTS_VALU"])
        ns = working_mean(inst[k]["SQ_INSTS_SALU"]) if "SQ_INSTS_SALU" in inst[k] else 0.0
        rows.append((t * len(d), k, t, nv, ns))
    rows.sort(reverse=True)
    out = ["# VALU issue of the kernels, 32,000-water box", "", "Commands:", "", "```"]
    out += args.command
    out += ["```", "",
            "Instructions are wavefront instructions per working dispatch; durations are "
            "working means from the kernel trace " + (
                "of the same run (dispatches profiled for counters run one at a time, so a "
                "kernel that normally overlaps another reads its own time alone).  "
                if os.path.dirname(os.path.abspath(args.counters)) ==
                os.path.dirname(os.path.abspath(args.trace)) else
                "(a separate run, the same workload).  ") +
            "Issue peak: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU "
            f"instruction = {VALU_PEAK / 1e9:.1f} G/s.  Transcendental and FP64 "
            "transcendental-helper instructions take longer than 4 cycles, so a kernel "
            "bound by them reads below 1.", "",
            "| kernel | working avg us | VALU instr (M) | VALU G/s | fraction of issue peak | "
            "SALU instr (M) |",
            "|---|---|---|---|---|---|"]
    for _, k, t, nv, ns in rows[:args.top]:
        rate = nv / (t * 1e-6)
        out.append(f"| `{k}` | {t:.2f} | {nv / 1e6:.2f} | {rate / 1e9:.1f} | "
                   f"{rate / VALU_PEAK:.3f} | {ns / 1e6:.2f} |")
    print("\n".join(out))


def issue(args):
    """VALU instructions per SIMD per 4 cycles on each kernel's own clock:
    GRBM_GUI_ACTIVE (summed over the 8 XCDs) over the dispatch's duration
    in the same run gives the clock the kernel ran at."""
    inst = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(args.counters)):
        inst[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = collections.defaultdict(list)
    for r in csv.DictReader(open(args.trace)):
        dur[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) -
                                             int(r["Start_Timestamp"])) / 1e3)

    def working_mean(v):
        med = sorted(v)[len(v) // 2]
        w = [x for x in v if x >= IDLE_FRACTION * med]
        return sum(w) / len(w)

    rows = []
    for k, d in dur.items():
        c = inst.get(k, {})
        if "SQ_INSTS_VALU" not in c or "GRBM_GUI_ACTIVE" not in c:
            continue
        t = working_mean(d)
        nv = working_mean(c["SQ_INSTS_VALU"])
        g = working_mean(c["GRBM_GUI_ACTIVE"]) / XCDS
        na = working_mean(c["SQ_ACTIVE_INST_VALU"]) if "SQ_ACTIVE_INST_VALU" in c else float("nan")
        rows.append((t * len(d), k, t, nv, g, na))
    rows.sort(reverse=True)
    out = ["# VALU issue on each kernel's own clock, 32,000-water box", "", "Command:", "",
           "```"] + args.command + ["```", "",
           "GRBM_GUI_ACTIVE counts GPU-busy cycles summed over the 8 XCDs, so per dispatch "
           "GRBM_GUI_ACTIVE / 8 over the dispatch's duration (kernel trace of the same run) is "
           "the clock the kernel ran at.  Issue is SQ_INSTS_VALU x 4 cycles / (1,024 SIMDs x "
           "GRBM_GUI_ACTIVE / 8): 1.0 means every SIMD issued one wave64 VALU instruction every "
           "4 cycles, the most a single VALU pipeline takes.  A value above 1 means some "
           "instructions issued beside others (the kernel's transcendentals are the "
           "candidates); SQ_ACTIVE_INST_VALU / SQ_INSTS_VALU near 1 shows that counter counts "
           "instructions here, not cycles.  The busy count also covers the dispatch's own "
           "start and drain, so for launches of tens of microseconds the clock reads above the "
           "part's 2.4 GHz and the issue figure low: the columns mean what they say for the "
           "long kernels (hundreds of microseconds).", "",
           "| kernel | working avg us | clock GHz | VALU instr (M) | issue per SIMD per 4 cycles | "
           "ACTIVE_INST / INSTS |", "|---|---|---|---|---|---|"]
    for _, k, t, nv, g, na in rows[:args.top]:
        out.append(f"| `{k}` | {t:.2f} | {g / (t * 1e3):.2f} | {nv / 1e6:.2f} | "
                   f"{nv * 4.0 / (SIMDS * g):.3f} | {na / nv:.3f} |")
    print("\n".join(out))


XCDS = 8
SIMDS = 256 * 4


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace")
    a.add_argument("stats")
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="Kernel time")
    a.add_argument("--top", type=int, default=30)
    a.add_argument("--note", default="")
    b = sub.add_parser("traffic")
    b.add_argument("--kernel", required=True, choices=sorted(TRAFFIC_SOURCES))
    b.add_argument("--workload", default="")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-fetch", required=True)
    b.add_argument("--copy-write", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--command", action="append", required=True)
    e = sub.add_parser("issue")
    e.add_argument("--counters", required=True)
    e.add_argument("--trace", required=True)
    e.add_argument("--command", action="append", required=True)
    e.add_argument("--top", type=int, default=24)
    c = sub.add_parser("valu")
    c.add_argument("--counters", required=True)
    c.add_argument("--trace", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--top", type=int, default=24)
    args = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "valu": valu, "issue": issue}[args.cmd](args)


if __name__ == "__main__":
    main(sys.argv[1:])
