"""Turns rocprofv3 CSV output into the short summaries kept under profiles/.

  python -m paper_2007_01277_amd.rocprof_summary stats  --csv DIR/trace_kernel_stats.csv --cmd "..." --out profiles/X.md
  python -m paper_2007_01277_amd.rocprof_summary counters --dir DIR [--dir DIR ...] --match SUBSTR --cmd "..." --out profiles/Y.md
         [--key NAME --key-match SUBSTR]
  python -m paper_2007_01277_amd.rocprof_summary traffic --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR
         --copy-bytes B --match SUBSTR --key NAME --alg-bytes B --cmd "..." --out profiles/Z.md

`traffic` scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of the
matched kernel by what the same counters read for the library's copy kernel
moving a known number of bytes, and records the result, with a hash of the
kernel sources it was measured on, in profiles/traffic.json; `counters --key`
records the matched kernel's counters the same way in profiles/counters.json.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# the sources that define and launch the fused kernels: a profile stays valid
# while these are unchanged (the cost model, tuner and batch sources do not
# touch the fused kernels)
KERNEL_SOURCES = ("hf_device.hpp", "hf_bodies.hpp", "hf_hash.hpp", "hf_kernels.hpp", "hf_pairs.hip",
                  "hf_runtime.hpp", "hf_runtime.hip")


def csrc_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2007_01277_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def time_weighted(values, times):
    """Utilisation of kernels launched one after the other, aggregated over
    their run: each kernel's value weighted by its elapsed time (the paper's
    Native issue-slot column, Sec. IV-C, weighs by elapsed cycles)."""
    return sum(v * t for v, t in zip(values, times)) / sum(times)


def trace_avg_ns(csv_path, match):
    """Average duration (ns) of the kernels matching `match` in a
    --kernel-trace --stats summary CSV."""
    rows = [r for r in csv.DictReader(open(csv_path)) if all(m in r["Name"] for m in match.split("&"))]
    if not rows:
        raise SystemExit(f"no kernel matches {match!r} in {csv_path}")
    calls = sum(int(r["Calls"]) for r in rows)
    return sum(float(r["AverageNs"]) * int(r["Calls"]) for r in rows) / calls


def alone_avg_ns(trace_csv, match):
    """Average duration (ns) of the dispatches of the kernels matching `match`
    (substrings separated by '&') that overlap no other dispatch in time, from
    a --kernel-trace per-dispatch CSV: launches on two concurrent streams are
    left out, so the figure is the kernel's time when it runs alone."""
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
            for r in csv.DictReader(open(trace_csv))]
    rows.sort()
    durs = []
    for i, (s, e, name) in enumerate(rows):
        if not all(m in name for m in match.split("&")):
            continue
        before = i > 0 and max(r[1] for r in rows[:i]) > s
        after = i + 1 < len(rows) and rows[i + 1][0] < e
        if not (before or after):
            durs.append(e - s)
    if not durs:
        raise SystemExit(f"no dispatch of {match!r} runs alone in {trace_csv}")
    return sum(durs) / len(durs)


def short(name: str) -> str:
    s = name.replace("hf::", "").replace("(DevTask, DevTask, unsigned int)", "").replace("(DevTask)", "")
    return s if len(s) <= 90 else s[:87] + "..."


def stats(a):
    rows = list(csv.DictReader(open(a.csv)))
    out = [f"# Kernel trace: {a.title}", "", f"Command (from the repository root):", "", "```", a.cmd, "```", "",
           "| kernel | calls | avg us | min us | max us | % time |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if a.trace and a.timed:
        skip, k = (int(v) for v in a.timed.split(","))
        d = launches_us(a.trace, a.timed_match, skip, k)
        out += ["", f"Dispatches {skip + 1}..{skip + k} of `{short(a.timed_match)}` in the per-dispatch trace "
                f"(the {k} timed steps after {skip} warmup steps): avg {statistics.fmean(d):.2f} us, median {statistics.median(d):.2f} us, min {min(d):.2f} us, "
                f"max {max(d):.2f} us."]
    for m in (a.alone or []):
        for grid, (n, avg, lo) in sorted(alone_by_grid_us(a.trace, m).items()):
            out += ["", f"`{short(m)}` at grid {grid} lanes, dispatches that ran alone: {n}, "
                        f"avg {avg:.2f} us, min {lo:.2f} us."]
    if a.note:
        out += ["", a.note]
    open(a.out, "w").write("\n".join(out) + "\n")


def alone_by_grid_us(trace_csv, match):
    """{grid lanes: (count, avg us, min us)} over the dispatches of `match` that
    overlap no other dispatch, from a --kernel-trace per-dispatch CSV."""
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"], int(r["Grid_Size_X"]))
            for r in csv.DictReader(open(trace_csv))]
    rows.sort()
    res, end_max = {}, None
    for i, (s, e, name, g) in enumerate(rows):
        before = end_max is not None and end_max > s
        after = i + 1 < len(rows) and rows[i + 1][0] < e
        end_max = e if end_max is None else max(end_max, e)
        if match in name and not (before or after):
            res.setdefault(g, []).append((e - s) / 1e3)
    return {g: (len(v), sum(v) / len(v), min(v)) for g, v in res.items()}


def launches_us(trace_csv, match, skip, k):
    """Durations (us) of dispatches skip+1 .. skip+k, in start order, of the
    kernels whose name contains `match`, from a --kernel-trace per-dispatch CSV."""
    rows = [r for r in csv.DictReader(open(trace_csv)) if match in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if len(rows) < skip + k:
        raise SystemExit(f"only {len(rows)} dispatches match {match!r} in {trace_csv}")
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[skip:skip + k]]


def read_pmc(d):
    """{kernel name: {counter: [values per dispatch]}} of one rocprofv3 --pmc output dir."""
    res = {}
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith("counter_collection.csv"):
                for r in csv.DictReader(open(os.path.join(root, f))):
                    res.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                        float(r["Counter_Value"]))
    return res


def clock_rows(d, xcds=8, simds=1024, min_ns=100000):
    """{kernel name: (dispatches, median clock GHz, median VALU instructions per
    SIMD per cycle)} from a --pmc pass that collected GRBM_GUI_ACTIVE (summed
    over the XCDs) and SQ_INSTS_VALU: clock = GRBM_GUI_ACTIVE / xcds /
    dispatch duration (its start and end timestamps in the same CSV).
    Dispatches shorter than min_ns are left out (the busy count then spans
    more than the kernel)."""
    per = {}
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith("counter_collection.csv"):
                for r in csv.DictReader(open(os.path.join(root, f))):
                    k = (r["Kernel_Name"], r["Dispatch_Id"])
                    e = per.setdefault(k, {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
                    e[r["Counter_Name"]] = float(r["Counter_Value"])
    out = {}
    for (name, _), e in per.items():
        if e["ns"] < min_ns or "GRBM_GUI_ACTIVE" not in e:
            continue
        cyc = e["GRBM_GUI_ACTIVE"] / xcds
        out.setdefault(name, []).append((cyc / e["ns"], e.get("SQ_INSTS_VALU", 0.0) / (cyc * simds)))
    return {n: (len(v), statistics.median(x[0] for x in v), statistics.median(x[1] for x in v))
            for n, v in out.items()}


def pick(res, match):
    """Kernel names matching `match`: alternatives separated by '|', each a
    list of substrings separated by '&' that must all occur."""
    alts = [a.split("&") for a in match.split("|")]
    names = [k for k in res if any(all(m in k for m in alt) for alt in alts)]
    if not names:
        raise SystemExit(f"no kernel matches {match!r}: {list(res)}")
    return names


def counters(a):
    lines = [f"# Counters: {a.title}", "", "Commands (from the repository root), one rocprofv3 pass each:", "", "```"]
    lines += a.cmd.split(";;")
    lines += ["```", "", "| kernel | counter | dispatches | mean per dispatch |", "|---|---|---:|---:|"]
    entry = {}
    for d in a.dir:
        res = read_pmc(d)
        for n in pick(res, a.match):
            for c, v in sorted(res[n].items()):
                lines.append(f"| `{short(n)}` | {c} | {len(v)} | {statistics.mean(v):.3f} |")
        if a.key:
            for n in pick(res, a.key_match):
                for c, v in res[n].items():
                    entry[c] = round(statistics.mean(v), 3)
                entry.setdefault("kernel", [])
                if short(n) not in entry["kernel"]:
                    entry["kernel"].append(short(n))
    if a.native:
        # the two solo kernels run back to back: each counter aggregated over
        # their run, weighted by their traced durations
        ma, mb = a.native.split(";")
        if a.trace_dispatch:
            ta, tb = alone_avg_ns(a.trace_dispatch, ma), alone_avg_ns(a.trace_dispatch, mb)
        else:
            ta, tb = trace_avg_ns(a.trace_csv, ma), trace_avg_ns(a.trace_csv, mb)
        per = {}
        for d in a.dir:
            res = read_pmc(d)
            for m, t in ((ma, ta), (mb, tb)):
                for n in pick(res, m):
                    for c, v in res[n].items():
                        per.setdefault(c, {})[m] = statistics.mean(v)
        lines += ["", f"Back-to-back aggregate of the two solo kernels (time-weighted, {ta / 1e3:.1f} us and "
                      f"{tb / 1e3:.1f} us from the kernel trace"
                      f"{', launches that ran alone' if a.trace_dispatch else ''}) next to the fused kernel:", "",
                  "| counter | fused | solo kernels back to back |", "|---|---:|---:|"]
        for c in sorted(per):
            if len(per[c]) == 2:
                nat = time_weighted([per[c][ma], per[c][mb]], [ta, tb])
                entry["native_" + c] = round(nat, 3)
                lines.append(f"| {c} | {entry.get(c, float('nan')):.3f} | {nat:.3f} |")
    if a.key:
        # the fused kernel's counters, for the bench line (valid while the
        # kernel sources hash matches)
        entry["csrc_hash"] = csrc_hash()
        path = os.path.join(ROOT, "profiles", "counters.json")
        data = json.load(open(path)) if os.path.exists(path) else {}
        data[a.key] = entry
        json.dump(data, open(path, "w"), indent=1, sort_keys=True)
    if a.clock:
        lines += ["", "Clock and VALU issue per dispatch (GRBM_GUI_ACTIVE / 8 XCDs / dispatch duration; "
                      "SQ_INSTS_VALU per SIMD per cycle; medians over dispatches of at least 100 us):", "",
                  "| kernel | dispatches | clock GHz | VALU instructions / SIMD / cycle |", "|---|---:|---:|---:|"]
        for d in a.dir:
            rows = clock_rows(d)
            for n in pick(rows, a.match):
                k, ghz, ipc = rows[n]
                lines.append(f"| `{short(n)}` | {k} | {ghz:.3f} | {ipc:.4f} |")
    if a.note:
        lines += ["", a.note]
    open(a.out, "w").write("\n".join(lines) + "\n")


def traffic(a):
    def mean_of(d, counter, match):
        res = read_pmc(d)
        names = pick(res, match)
        vals = [v for n in names for v in res[n].get(counter, [])]
        return statistics.mean(vals), len(vals), names

    f_kib, nf, names = mean_of(a.fetch, "FETCH_SIZE", a.match)
    w_kib, nw, _ = mean_of(a.write, "WRITE_SIZE", a.match)
    cf_kib, _, _ = mean_of(a.copy_fetch, "FETCH_SIZE", "k_copy")
    cw_kib, _, _ = mean_of(a.copy_write, "WRITE_SIZE", "k_copy")
    sf = a.copy_bytes / (cf_kib * 1024.0)  # bytes per counted KiB, reads
    sw = a.copy_bytes / (cw_kib * 1024.0)  # bytes per counted KiB, writes
    rd = f_kib * 1024.0 * sf
    wr = w_kib * 1024.0 * sw
    entry = {"kernel": [short(n) for n in names], "fetch_kib": round(f_kib, 1), "write_kib": round(w_kib, 1),
             "copy_scale_read": round(sf, 4), "copy_scale_write": round(sw, 4),
             "hbm_read_bytes": round(rd), "hbm_write_bytes": round(wr),
             "hbm_bytes_per_launch": round(rd + wr), "algorithmic_bytes": a.alg_bytes,
             "traffic_over_algorithmic": round((rd + wr) / a.alg_bytes, 4) if a.alg_bytes else None,
             "dispatches": [nf, nw], "csrc_hash": csrc_hash()}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[a.key] = entry
    json.dump(data, open(path, "w"), indent=1, sort_keys=True)
    lines = [f"# HBM traffic: {a.title}", "", "Commands (from the repository root), one rocprofv3 pass each:", "", "```"]
    lines += a.cmd.split(";;")
    lines += ["```", "",
              f"Copy kernel reference: {a.copy_bytes} bytes read and written; FETCH_SIZE read {cf_kib:.1f} KiB "
              f"(scale {sf:.4f}), WRITE_SIZE read {cw_kib:.1f} KiB (scale {sw:.4f}).", "",
              "| quantity | value |", "|---|---:|",
              f"| FETCH_SIZE per dispatch (KiB) | {f_kib:.1f} |", f"| WRITE_SIZE per dispatch (KiB) | {w_kib:.1f} |",
              f"| HBM read per launch (scaled, bytes) | {rd:.4g} |", f"| HBM write per launch (scaled, bytes) | {wr:.4g} |",
              f"| algorithmic bytes per launch | {a.alg_bytes:.4g} |",
              f"| traffic / algorithmic | {(rd + wr) / a.alg_bytes:.3f} |" if a.alg_bytes else "",
              "", f"Kernel sources hash: `{entry['csrc_hash']}` (the bench reports this traffic only while it matches)."]
    open(a.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--trace", default="", help="the per-dispatch kernel trace CSV of the same run")
    s.add_argument("--timed", default="", help="W,K: also summarise dispatches W+1..W+K of --timed-match")
    s.add_argument("--timed-match", default="")
    s.add_argument("--alone", action="append", help="per-grid averages of this kernel's dispatches that ran alone")
    for p in (s,):
        p.add_argument("--cmd", required=True)
        p.add_argument("--out", required=True)
        p.add_argument("--title", default="")
        p.add_argument("--note", default="")
    c = sub.add_parser("counters")
    c.add_argument("--dir", action="append", required=True)
    c.add_argument("--match", required=True)
    c.add_argument("--key", default="", help="record the counters of --key-match in profiles/counters.json")
    c.add_argument("--key-match", default="")
    c.add_argument("--native", default="", help="SOLO_A;SOLO_B: also aggregate the two solo kernels")
    c.add_argument("--trace-csv", default="", help="kernel-trace stats CSV giving the solo durations")
    c.add_argument("--trace-dispatch", default="",
                   help="per-dispatch kernel trace CSV: solo durations from the launches that ran alone")
    c.add_argument("--clock", action="store_true", help="also derive clock and VALU issue per cycle")
    c.add_argument("--cmd", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "match", "key", "cmd", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--alg-bytes", type=float, default=0.0)
    t.add_argument("--title", default="")
    a = ap.parse_args()
    {"stats": stats, "counters": counters, "traffic": traffic}[a.mode](a)


if __name__ == "__main__":
    main()
