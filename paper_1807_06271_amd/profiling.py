"""Summaries of rocprofv3 CSV output for the profiles/ directory.

    python -m paper_1807_06271_amd.profiling stats  <kernel_stats.csv> <out.txt> "<command>" \
        [<kernel_trace.csv> (<kernel name part> <N dispatches> <skip, -1: the last N> <largest|all|grid=G>)...]
    python -m paper_1807_06271_amd.profiling traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <out.json> "<fetch command>" "<write command>" [median|largest|max]
    python -m paper_1807_06271_amd.profiling counters <counter_collection.csv> <kernel_trace.csv> \
        <out.txt> "<command>" [largest [<kernel name part>@<grid>]...]

`stats` keeps the per-kernel call count and average / min / max durations.
`counters` keeps the median per dispatch of each SQ counter of each kernel and
derives the VALU issue utilisation: SQ_INSTS_VALU (wave instructions) over
what the chip can issue in the kernel's median duration (from the kernel
trace of the same run): one wave64 VALU instruction per clock per CU (four
SIMDs, each 16 lanes wide), 256 CUs at 2.4 GHz.
`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) into bytes per
launch of each kernel (and of each of its grid sizes, for a kernel whose
launches of different shapes do different work), scaled by what the same counter reads for the plain
copy kernel of known size that the profiled run also executes (bench.py
--calibrate-copy copies CALIBRATION_BYTES between two device buffers); the
JSON also records a hash of the kernel sources, so a reader can tell whether
the counters still describe the current kernels.
"""
from __future__ import annotations

import csv
import hashlib
import re
import json
import os
import sys
from collections import defaultdict

CALIBRATION_BYTES = 1 << 30  # 1 GiB device-to-device copy
PKG = os.path.dirname(os.path.abspath(__file__))


def _header_section(name: str, marker: str) -> bytes:
    """The shared preamble of a kernel header plus one of its "// ---- name"
    sections (what a kernel's code depends on in that header)."""
    text = open(os.path.join(PKG, "csrc", name), encoding="utf-8").read()
    cuts = [i for i in range(len(text)) if text.startswith("// ---", i) and (i == 0 or text[i - 1] == "\n")]
    pre = text[:cuts[0]] if cuts else text
    body = ""
    for a, b in zip(cuts, cuts[1:] + [len(text)]):
        if marker in text[a:text.index("\n", a)]:
            body = text[a:b]
    return (pre + body).encode()


def _code_only(text: bytes) -> bytes:
    """Source text without comments and blank-space differences, so that a
    documentation edit does not invalidate a measurement of the same code."""
    t = text.decode("utf-8")
    t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
    t = re.sub(r"//[^\n]*", " ", t)
    return " ".join(t.split()).encode()


def source_hash(files=("aggregate.hip", "stripes.hip", "device_util.h")) -> str:
    """Hash of the aggregation kernels' code (the per-direction kernel and
    the two-pass stripe kernels): their files, the device helpers and their
    sections of the kernel header (changes elsewhere in the header do not
    touch them), comments and spacing ignored."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(_code_only(fh.read()))
    h.update(_code_only(_header_section("sgm_kernels.h", "aggregation")))
    h.update(_code_only(_header_section("sgm_kernels.h", "two-pass stripes")))
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    name = name.replace("(sgmk::JobTable<sgmk::", "(").replace("void ", "")
    return name[:110]


def stats(csv_path: str, out_path: str, command: str, trace_csv: str | None = None,
          selections=()) -> None:
    """Kernel statistics; with trace_csv, also for each selection (kernel,
    first, skip, grid) the average of dispatches skip .. skip+first-1 (in
    start order; skip < 0: the last `first`) of `kernel` (a loop of the
    benchmark in which the kernel runs alone); grid True: counted among the
    dispatches with the kernel's largest grid only (e.g. its 8-frame
    launches, not single frames), an int: among those with that grid, False:
    all."""
    rows = list(csv.DictReader(open(csv_path)))
    lines = ["# rocprofv3 kernel statistics", "# command: " + command, "#",
             "%-100s %6s %12s %12s %12s %7s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct")]
    for r in rows:
        lines.append("%-100s %6s %12.1f %12.1f %12.1f %7.2f" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    if trace_csv and selections:
        trace = list(csv.DictReader(open(trace_csv)))
        lines.append("#")
        for kernel, first, skip, largest in selections:
            tr = [r for r in trace if kernel in r["Kernel_Name"]]
            tr.sort(key=lambda r: int(r["Start_Timestamp"]))
            grid = max(int(r["Grid_Size_X"]) for r in tr) if largest is True else largest
            if largest is not False:
                tr = [r for r in tr if int(r["Grid_Size_X"]) == grid]
            if skip < 0:  # the last `first` dispatches
                skip = len(tr) - first
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr][skip:skip + first]
            lines.append("# dispatches %d..%d (in start order)%s of %s: avg %.1f us, min %.1f, max %.1f"
                         % (skip, skip + len(d) - 1, " (grid %d only)" % grid if largest is not False else "", kernel,
                            sum(d) / len(d), min(d), max(d)))
    open(out_path, "w").write("\n".join(lines) + "\n")


def _per_grid(csv_path: str, counter: str):
    """{kernel name: {grid: [per-dispatch counter values]}}."""
    acc = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(csv_path)):
        if r.get("Counter_Name") == counter:
            acc[r["Kernel_Name"]][int(r["Grid_Size"])].append(float(r["Counter_Value"]))
    return acc


def _per_kernel(csv_path: str, counter: str, largest: bool = False):
    """{kernel name: [per-dispatch counter values]} from counter_collection.csv;
    with `largest`, only each kernel's dispatches with its largest grid."""
    rows = [r for r in csv.DictReader(open(csv_path)) if r.get("Counter_Name") == counter]
    big = defaultdict(int)
    for r in rows:
        big[r["Kernel_Name"]] = max(big[r["Kernel_Name"]], int(r["Grid_Size"]))
    acc = defaultdict(list)
    for r in rows:
        if not largest or int(r["Grid_Size"]) == big[r["Kernel_Name"]]:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return acc


def traffic(fetch_csv: str, write_csv: str, out_path: str, fetch_cmd: str, write_cmd: str,
            pick: str = "median") -> dict:
    """pick: "median" of each kernel's dispatches (all dispatches of one size),
    "largest" (the median over the dispatches with the kernel's largest grid,
    e.g. whole batches among single frames), or "max" (the largest dispatch)."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE", pick == "largest")
    w = _per_kernel(write_csv, "WRITE_SIZE", pick == "largest")
    copy = [k for k in f if "copy" in k.lower() or "elementwise" in k.lower()]
    # the calibration copy is the dispatch whose fetch is largest among copies
    best = None
    for k in copy:
        for v in f[k]:
            if best is None or v > best[1]:
                best = (k, v)
    if best is None:
        raise SystemExit("no copy kernel found for calibration")
    cname, cfetch = best
    cwrite = max(w.get(cname, [0.0]))
    fetch_factor = CALIBRATION_BYTES / (cfetch * 1024.0)
    write_factor = CALIBRATION_BYTES / (cwrite * 1024.0) if cwrite else None
    fg, wg = _per_grid(fetch_csv, "FETCH_SIZE"), _per_grid(write_csv, "WRITE_SIZE")
    kernels = {}
    for k in f:
        if k == cname:
            continue
        fs, ws = sorted(f[k]), sorted(w.get(k, [0.0]))
        fv = fs[-1] if pick == "max" else fs[len(fs) // 2]
        wv = ws[-1] if pick == "max" else ws[len(ws) // 2]
        grids = {}
        for g, vals in sorted(fg.get(k, {}).items()):
            fgv = sorted(vals)[len(vals) // 2]
            wgs = sorted(wg.get(k, {}).get(g, [0.0]))
            wgv = wgs[len(wgs) // 2]
            grids[str(g)] = {"dispatches": len(vals), "fetch_kib": fgv, "write_kib": wgv,
                             "fetch_bytes": fgv * 1024.0 * fetch_factor,
                             "write_bytes": wgv * 1024.0 * (write_factor or 1.0)}
        kernels[short_name(k)] = {
            "dispatches": len(f[k]),
            "fetch_kib": fv, "write_kib": wv, "pick": pick,
            "fetch_bytes": fv * 1024.0 * fetch_factor,
            "write_bytes": wv * 1024.0 * (write_factor or 1.0),
            "grids": grids,
        }
    out = {"calibration": {"kernel": short_name(cname), "bytes": CALIBRATION_BYTES,
                           "fetch_kib": cfetch, "write_kib": cwrite,
                           "fetch_factor": fetch_factor, "write_factor": write_factor},
           "source_hash": source_hash(),
           "source_hash_covers": "aggregate.hip, stripes.hip, device_util.h and the aggregation and two-pass sections of sgm_kernels.h, comments and spacing ignored",
           "fetch_command": fetch_cmd, "write_command": write_cmd,
           "kernels": kernels}
    json.dump(out, open(out_path, "w"), indent=1)
    return out


CUS, CLOCK_HZ = 256, 2.4e9


def counters(csv_path: str, trace_csv: str, out_path: str, command: str, largest: bool = False,
             extra=()) -> None:
    """Median per dispatch of each counter of each kernel; with `largest`,
    only the dispatches with the kernel's largest grid (e.g. the 8-frame
    launches of a kernel that also ran single frames), each entry labelled
    with that grid; `extra`: (kernel name part, grid) pairs summarised as
    entries of their own (a kernel's launches of another shape)."""
    def grid_ok(name, grid, biggest):
        return not largest or grid == biggest[name]

    tr = list(csv.DictReader(open(trace_csv)))
    big_tr = defaultdict(int)
    for r in tr:
        big_tr[short_name(r["Kernel_Name"])] = max(big_tr[short_name(r["Kernel_Name"])], int(r["Grid_Size_X"]))
    dur = defaultdict(list)
    for r in tr:
        k = short_name(r["Kernel_Name"])
        if grid_ok(k, int(r["Grid_Size_X"]), big_tr):
            dur[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = list(csv.DictReader(open(csv_path)))
    big = defaultdict(int)
    for r in rows:
        big[short_name(r["Kernel_Name"])] = max(big[short_name(r["Kernel_Name"])], int(r["Grid_Size"]))
    acc = defaultdict(lambda: defaultdict(list))
    for r in rows:
        k = short_name(r["Kernel_Name"])
        if grid_ok(k, int(r["Grid_Size"]), big):
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 counters (median per dispatch) and VALU issue utilisation",
             "# command: " + command,
             "# VALU util = SQ_INSTS_VALU / (%d CUs x %.1f GHz x median duration of the same run's dispatches)"
             % (CUS, CLOCK_HZ / 1e9),
             "# dispatches: " + ("only each kernel's largest grid" if largest else "all"),
             "# aggregation source hash %s" % source_hash(), "#"]
    entries = {(k + (" [grid %d]" % big[k] if largest else "")): (acc[k], dur.get(k)) for k in acc}
    for part, g in extra:
        for k in {short_name(r["Kernel_Name"]) for r in rows}:
            if part not in k:
                continue
            ca = defaultdict(list)
            for r in rows:
                if short_name(r["Kernel_Name"]) == k and int(r["Grid_Size"]) == g:
                    ca[r["Counter_Name"]].append(float(r["Counter_Value"]))
            du = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr
                  if short_name(r["Kernel_Name"]) == k and int(r["Grid_Size_X"]) == g]
            if ca:
                entries["%s [grid %d]" % (k, g)] = (ca, du)
    for name in sorted(entries, key=lambda n: -max(entries[n][0].get("SQ_INSTS_VALU", [0]))):
        ca, du = entries[name]
        med = {c: sorted(v)[len(v) // 2] for c, v in ca.items()}
        util = ""
        if du and "SQ_INSTS_VALU" in med:
            us = sorted(du)[len(du) // 2]
            util = "  VALU util %.2f (median %.1f us, %d dispatches)" % (
                med["SQ_INSTS_VALU"] / (CUS * CLOCK_HZ * us * 1e-6), us, len(du))
        lines.append(name + util)
        lines.append("    " + ", ".join("%s %d" % (c, v) for c, v in sorted(med.items())))
    open(out_path, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        # ... <trace.csv> then groups of: <kernel name part> <N dispatches> <skip (-1: the last N)> <largest|all>
        sel = sys.argv[6:]
        def mode(m):
            return True if m == "largest" else int(m[5:]) if m.startswith("grid=") else False
        groups = [(sel[i], int(sel[i + 1]), int(sel[i + 2]), mode(sel[i + 3])) for i in range(0, len(sel) - 3, 4)]
        stats(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else None, groups)
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], *sys.argv[7:8])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], len(sys.argv) > 6 and sys.argv[6] == "largest",
                 [(a.rsplit("@", 1)[0], int(a.rsplit("@", 1)[1])) for a in sys.argv[7:]])
    else:
        raise SystemExit(__doc__)
