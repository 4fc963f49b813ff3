"""Summaries of rocprofv3 output for the stepper kernels.

    python -m paper_2312_05410_amd.rocprof_summary stats DIR [--kernel SUBSTR]
    python -m paper_2312_05410_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR --kernel SUBSTR \
        [--ref-bytes N] [--out FILE] [--command TEXT]

`stats` prints the per-kernel summary of a `--kernel-trace --stats` run
(CSV output); `dbstats` the same from the SQLite database rocprofv3 writes
by default (`*_results.db`), grouped by kernel and grid.
`counters` prints SQ counter metrics (occupancy, VALU issue, wait and MFMA
fractions, LDS conflicts) of one kernel from a `--pmc` run.
`sequence` splits a `--kernel-trace` run into the launch sequences that
begin with a kernel whose name contains START (and whose next kernel's name
contains NEXT, if given) and prints, position by position, the median
duration over the sequences of the most common length (e.g. the kernels of
one network forward).
`traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the same
program, whose first large device copy (--ref-bytes bytes, read once and
written once) calibrates the counters: each counter is scaled by
ref_bytes / (its reading for that copy).  It prints (or writes) the scaled
HBM bytes per launch of the kernels whose name contains SUBSTR, tagged with
a hash of the stepper sources so that a stale summary can be recognised.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STEPPER_SOURCES = ("csrc/pf_cell.h", "csrc/pf_march.hip", "csrc/pf_step.hip", "csrc/pf_resident.hip", "csrc/pf_kernels.h")


def stepper_hash() -> str:
    h = hashlib.sha256()
    for rel in STEPPER_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def stats(d: str, kernel: str | None = None):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    out = []
    for r in rows:
        if kernel and kernel not in r["Name"]:
            continue
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
                    float(r["Percentage"])))
    return out


def sequence(d: str, start: str, nxt: str | None = None):
    rows = sorted(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_trace.csv")))),
                  key=lambda r: int(r["Start_Timestamp"]))
    heads = [i for i, r in enumerate(rows) if start in r["Kernel_Name"] and
             (nxt is None or (i + 1 < len(rows) and nxt in rows[i + 1]["Kernel_Name"]))]
    seqs = []
    for i, h in enumerate(heads):
        end = heads[i + 1] if i + 1 < len(heads) else len(rows)
        seqs.append(rows[h:end])
    if not seqs:
        raise SystemExit(f"no sequence starts with {start}")
    n = statistics.mode(len(q) for q in seqs[:-1] or seqs)
    seqs = [q[:n] for q in seqs if len(q) >= n]
    out = []
    for k in range(n):
        dur = [(int(q[k]["End_Timestamp"]) - int(q[k]["Start_Timestamp"])) / 1e3 for q in seqs]
        out.append((seqs[-1][k]["Kernel_Name"], statistics.median(dur)))
    span = statistics.median((int(q[-1]["End_Timestamp"]) - int(q[0]["Start_Timestamp"])) / 1e3 for q in seqs)
    return len(seqs), out, span


def _counter(d: str, name: str):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))))
    return [(int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
            for r in rows if r["Counter_Name"] == name]


def dbstats(d: str, kernel: str | None = None, top: int = 40):
    """(name, grid, calls, avg ns, min ns, max ns, share %) from a results
    database, largest total time first."""
    import sqlite3

    db = sqlite3.connect(_one(os.path.join(d, "**", "*results.db")))
    rows = db.execute("select name, grid_x, grid_y, grid_z, count(*), avg(end - start), min(end - start), "
                      "max(end - start), sum(end - start) from kernels group by name, grid_x, grid_y, grid_z "
                      "order by sum(end - start) desc").fetchall()
    tot = sum(r[8] for r in rows) or 1
    out = []
    for name, gx, gy, gz, calls, avg, mn, mx, sm in rows:
        if kernel and kernel not in name:
            continue
        out.append((name, f"{gx}x{gy}x{gz}", calls, avg, mn, mx, 100.0 * sm / tot))
    return out[:top]


def traffic(fetch_dir: str, write_dir: str, kernel: str, ref_bytes: int):
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    # reference: the largest copy kernel dispatch
    ref_f = max((v for _, n, _, v in f if "copyBuffer" in n or "copy" in n.lower()), default=None)
    ref_w = max((v for _, n, _, v in w if "copyBuffer" in n or "copy" in n.lower()), default=None)
    if not ref_f or not ref_w:
        raise SystemExit("no reference copy kernel in the counter runs")
    sf = ref_bytes / (ref_f * 1024.0)
    sw = ref_bytes / (ref_w * 1024.0)
    kf = [v for _, n, _, v in f if kernel in n]
    kw = [v for _, n, _, v in w if kernel in n]
    if not kf or not kw:
        raise SystemExit(f"no dispatch of a kernel matching {kernel!r}")
    return dict(fetch_kib_raw=statistics.median(kf), write_kib_raw=statistics.median(kw),
                fetch_scale=sf, write_scale=sw,
                fetch_bytes=statistics.median(kf) * 1024.0 * sf,
                write_bytes=statistics.median(kw) * 1024.0 * sw,
                launches=min(len(kf), len(kw)))


def counters(d: str, kernel: str, cus: int = 256, simds: int = 1024, xcds: int = 8):
    """Per-dispatch SQ counter metrics of the kernels whose name contains
    `kernel` (median over their dispatches).  GRBM_GUI_ACTIVE is the sum over
    the XCDs (cycles per XCD = value / xcds); SQ_*_CYCLES and SQ_WAIT_* are
    in quad-cycles (4 clocks), SQ_VALU_MFMA_BUSY_CYCLES in clocks per SIMD."""
    import collections

    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))))
    disp = collections.OrderedDict()
    for r in rows:
        if kernel not in r["Kernel_Name"]:
            continue
        e = disp.setdefault(r["Dispatch_Id"], {"us": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3,
                                               "c": collections.defaultdict(float)})
        e["c"][r["Counter_Name"]] += float(r["Counter_Value"])
    if not disp:
        raise SystemExit(f"no dispatch of a kernel matching {kernel!r}")
    out = collections.defaultdict(list)
    for e in disp.values():
        c, us = e["c"], e["us"]
        out["duration_us"].append(us)
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        if cyc:
            out["cycles_per_xcd"].append(cyc)
            out["clock_GHz"].append(cyc / us / 1e3)
        if "SQ_WAVES" in c:
            out["waves"].append(c["SQ_WAVES"])
        if cyc and "SQ_WAVE_CYCLES" in c:
            out["mean_waves_per_CU"].append(4 * c["SQ_WAVE_CYCLES"] / (cus * cyc))
        if cyc and "SQ_INSTS_VALU" in c:
            out["valu_wave_instructions"].append(c["SQ_INSTS_VALU"])
            # a wave64 FP32 VALU instruction occupies its SIMD for 2 clocks
            out["valu_issue_fraction"].append(2 * c["SQ_INSTS_VALU"] / (simds * cyc))
        for name, key in (("SQ_WAIT_ANY", "wait_any_fraction_of_wave_time"),
                          ("SQ_WAIT_INST_ANY", "wait_issue_fraction_of_wave_time"),
                          ("SQ_ACTIVE_INST_VALU", "valu_active_fraction_of_wave_time"),
                          ("SQ_ACTIVE_INST_LDS", "lds_active_fraction_of_wave_time")):
            if name in c and c.get("SQ_WAVE_CYCLES"):
                out[key].append(c[name] / c["SQ_WAVE_CYCLES"])
        if cyc and "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            out["mfma_busy_fraction"].append(c["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cyc))
        if "SQ_INSTS_MFMA" in c:
            out["mfma_instructions"].append(c["SQ_INSTS_MFMA"])
        if c.get("SQ_LDS_IDX_ACTIVE", 0) > c.get("SQ_LDS_BANK_CONFLICT", 0):
            out["lds_conflicts_per_access"].append(
                c.get("SQ_LDS_BANK_CONFLICT", 0) / (c["SQ_LDS_IDX_ACTIVE"] - c.get("SQ_LDS_BANK_CONFLICT", 0)))
        if "SQ_WAIT_INST_LDS" in c and c.get("SQ_WAVE_CYCLES"):
            out["wait_lds_issue_fraction_of_wave_time"].append(c["SQ_WAIT_INST_LDS"] / c["SQ_WAVE_CYCLES"])
    return len(disp), {k: statistics.median(v) for k, v in out.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--kernel")
    s2 = sub.add_parser("dbstats")
    s2.add_argument("dir")
    s2.add_argument("--kernel")
    s2.add_argument("--top", type=int, default=40)
    q = sub.add_parser("counters")
    q.add_argument("dir")
    q.add_argument("--kernel", required=True)
    q.add_argument("--command", default="")
    q.add_argument("--out")
    sq = sub.add_parser("sequence")
    sq.add_argument("dir")
    sq.add_argument("--start", required=True)
    sq.add_argument("--next")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--ref-bytes", type=int, default=512 * 1024 * 1024)
    t.add_argument("--out")
    t.add_argument("--command", default="")
    t.add_argument("--steps-per-launch", type=int, default=0,
                   help="steps each dispatch advances (a launch that runs a whole call): also per step")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        for name, calls, avg, mn, mx, pct in stats(a.dir, a.kernel):
            print(f"{name}\n    calls {calls}  avg {avg / 1e3:.3f} us  min {mn / 1e3:.3f}  max {mx / 1e3:.3f}  "
                  f"share {pct:.2f} %")
        return
    if a.cmd == "dbstats":
        for name, grid, calls, avg, mn, mx, pct in dbstats(a.dir, a.kernel, a.top):
            print(f"{name}\n    grid {grid}  calls {calls}  avg {avg / 1e3:.3f} us  min {mn / 1e3:.3f}  "
                  f"max {mx / 1e3:.3f}  share {pct:.2f} %")
        return
    if a.cmd == "sequence":
        n, seq, span = sequence(a.dir, a.start, a.next)
        print(f"{n} sequences of {len(seq)} launches; median duration per position (us):")
        for i, (name, us) in enumerate(seq):
            print(f"{i:3d} {us:8.2f}  {name}")
        print(f"sum of the medians {sum(u for _, u in seq):.1f} us; median span first start to last end "
              f"{span:.1f} us")
        return
    if a.cmd == "counters":
        n, m = counters(a.dir, a.kernel)
        lines = ([f"command: {a.command}"] if a.command else []) + [
            f"kernel: {a.kernel}", f"stepper_source_sha256_16: {stepper_hash()}", f"dispatches: {n}",
            "medians over the dispatches:"] + [f"{k}: {v:.4g}" for k, v in m.items()]
        text = "\n".join(lines) + "\n"
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(text)
        sys.stdout.write(text)
        return
    r = traffic(a.fetch_dir, a.write_dir, a.kernel, a.ref_bytes)
    lines = [f"kernel: {a.kernel}",
             f"stepper_source_sha256_16: {stepper_hash()}",
             f"launches_measured: {r['launches']}",
             f"FETCH_SIZE_KiB_per_launch_raw: {r['fetch_kib_raw']:.1f}",
             f"WRITE_SIZE_KiB_per_launch_raw: {r['write_kib_raw']:.1f}",
             f"fetch_scale_from_reference_copy: {r['fetch_scale']:.4f}",
             f"write_scale_from_reference_copy: {r['write_scale']:.4f}",
             f"hbm_read_bytes_per_launch: {r['fetch_bytes']:.0f}",
             f"hbm_write_bytes_per_launch: {r['write_bytes']:.0f}",
             f"hbm_bytes_per_launch: {r['fetch_bytes'] + r['write_bytes']:.0f}"]
    if a.steps_per_launch:
        lines += [f"steps_per_launch: {a.steps_per_launch}",
                  f"hbm_bytes_per_step: {(r['fetch_bytes'] + r['write_bytes']) / a.steps_per_launch:.0f}"]
    if a.command:
        lines.insert(0, f"command: {a.command}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    sys.stdout.write(text)


if __name__ == "__main__":
    main()
