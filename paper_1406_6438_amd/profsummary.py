"""Summaries of rocprofv3 output for the profiles/ notes.

  profsummary.py trace <results.db | kernel_stats.csv>
      per-kernel calls, total and average duration
  profsummary.py traffic <fetch counter_collection.csv> <write counter_collection.csv> \\
                 <kernel substring> <copy kernel substring> <copy bytes per dispatch>
      HBM bytes per dispatch of a kernel from FETCH_SIZE / WRITE_SIZE (KiB per
      dispatch), each scaled by the ratio of a plain copy kernel's known bytes to
      what the same counter reads for it.
  profsummary.py valu <kernel substring> <counter_collection.csv> [...]
      per-dispatch averages of the SQ counters and derived metrics the files hold
      for the kernel: VALU instructions, VALU-active quad-cycles, VALUBusy,
      occupancy, ...; the figures bench.py reads are printed as
      "valu_insts_per_launch", "valu_active_quad_cycles_per_launch" and
      "valu_busy_frac".
"""
from __future__ import annotations

import csv
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def kernel_stats(path: str, limit: int = 20):
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        rows = con.execute("select name, total_calls, total_duration, average, percentage "
                           "from top_kernels limit ?", (limit,)).fetchall()
        con.close()
        return [(n, c, t / 1e3 if t > 1e7 else t, a / 1e3 if a > 1e7 else a, p)
                for n, c, t, a, p in rows]
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return rows[:limit]


def counters_of(path: str):
    out = set()
    with open(path) as fh:
        for r in csv.DictReader(fh):
            out.add(r.get("Counter_Name"))
    return sorted(c for c in out if c)


def counter_per_dispatch(path: str, counter: str):
    """{kernel name: [value per dispatch]} from a counter_collection.csv."""
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def pick(d: dict, sub: str):
    keys = [k for k in d if sub in k]
    if not keys:
        raise SystemExit(f"no kernel matching {sub!r}")
    vals = [v for k in keys for v in d[k]]
    return keys[0], vals


def kernel_source_hash() -> str:
    src = os.path.join(HERE, "csrc", "lbm_vans.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def main(argv):
    if len(argv) >= 3 and argv[1] == "trace":
        print("| kernel | calls | total us | avg us | % |")
        print("|---|---|---|---|---|")
        for name, calls, total, avg, pct in kernel_stats(argv[2]):
            print(f"| {short(name)} | {calls} | {total:.1f} | {avg:.2f} | {pct:.1f} |")
        return
    if len(argv) == 7 and argv[1] == "traffic":
        fetch = counter_per_dispatch(argv[2], "FETCH_SIZE")
        write = counter_per_dispatch(argv[3], "WRITE_SIZE")
        ksub, csub, copy_bytes = argv[4], argv[5], float(argv[6])
        kf_name, kf = pick(fetch, ksub)
        _, kw = pick(write, ksub)
        _, cf = pick(fetch, csub)
        _, cw = pick(write, csub)
        # the copy dispatches of the calibration are the large ones
        cf_big = max(cf)
        cw_big = max(cw)
        sf = copy_bytes / (cf_big * 1024.0)
        sw = copy_bytes / (cw_big * 1024.0)
        f_b = sum(kf) / len(kf) * 1024.0 * sf
        w_b = sum(kw) / len(kw) * 1024.0 * sw
        print(f"kernel: {short(kf_name)}  dispatches: fetch {len(kf)}, write {len(kw)}")
        print(f"FETCH_SIZE avg KiB/dispatch: {sum(kf) / len(kf):.1f}")
        print(f"WRITE_SIZE avg KiB/dispatch: {sum(kw) / len(kw):.1f}")
        print(f"copy calibration: {copy_bytes:.0f} B read and written per dispatch; "
              f"FETCH_SIZE {cf_big:.1f} KiB -> factor {sf:.4f}; WRITE_SIZE {cw_big:.1f} KiB -> factor {sw:.4f}")
        print(f"hbm_read_bytes_per_launch: {f_b:.6e}")
        print(f"hbm_write_bytes_per_launch: {w_b:.6e}")
        print(f"hbm_bytes_per_launch: {f_b + w_b:.6e}")
        print(f"kernel_source_sha256_16: {kernel_source_hash()}")
        return
    if len(argv) >= 4 and argv[1] == "valu":
        ksub = argv[2]
        vals = {}
        name = None
        for path in argv[3:]:
            for c in counters_of(path):
                n, v = pick(counter_per_dispatch(path, c), ksub)
                name = name or n
                vals[c] = (sum(v) / len(v), len(v))
        print(f"kernel: {short(name)}")
        for c, (avg, n) in sorted(vals.items()):
            print(f"{c}: {avg:.6e}  (average of {n} dispatches)")
        if "SQ_INSTS_VALU" in vals:
            print(f"valu_insts_per_launch: {vals['SQ_INSTS_VALU'][0]:.6e}")
        if "SQ_ACTIVE_INST_VALU" in vals:
            print(f"valu_active_quad_cycles_per_launch: {vals['SQ_ACTIVE_INST_VALU'][0]:.6e}")
        if "VALUBusy" in vals:
            print(f"valu_busy_frac: {vals['VALUBusy'][0] / 100.0:.4f}")
        print(f"kernel_source_sha256_16: {kernel_source_hash()}")
        return
    print(__doc__)
    sys.exit(2)


if __name__ == "__main__":
    main(sys.argv)
