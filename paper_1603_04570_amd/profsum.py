"""Summaries of rocprofv3 CSV output (``--output-format csv``).

    python -m paper_1603_04570_amd.profsum stats KERNEL_STATS_CSV [TOP]
        per-kernel totals from ``--kernel-trace --stats`` (kt_kernel_stats.csv)

    python -m paper_1603_04570_amd.profsum bygrid KERNEL_TRACE_CSV [TOP]
        per (kernel, grid size) totals from ``--kernel-trace`` (kt_kernel_trace.csv):
        separates the multigrid levels and the grids of one kernel template

    python -m paper_1603_04570_amd.profsum ranges MARKER_TRACE_CSV
        per ROCTX range name (``--marker-trace``, marker_api_trace.csv): count,
        total, mean, median and 99th percentile of the range durations

    python -m paper_1603_04570_amd.profsum traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes BYTES --kernel SUBSTRING \
        [--kernel SUBSTRING ...] [--exclude SUBSTRING ...] [--main-grid]
        per-dispatch HBM bytes of the kernels whose name contains any SUBSTRING
        (and none of the --exclude ones)
        (with --main-grid: only their dispatches of the most dispatched grid
        size of each run, i.e. the launch shape that run used most -- autotuner
        trials and other levels excluded), from
        two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs, each scaled by
        what the same counter reads for a plain copy kernel of BYTES bytes read
        and BYTES bytes written (the copy runs of ``bench.py --calibrate-copy``).

    python -m paper_1603_04570_amd.profsum counters --csv A.csv [--csv B.csv ...] \
        --kernel SUBSTRING [--kernel SUBSTRING ...] [--grid G]
        mean value per dispatch of every counter in the ``--pmc`` runs A, B, ...
        for each kernel whose name contains a SUBSTRING, over its dispatches of
        grid size G (default: its most dispatched one), with instructions per wavefront and the
        shares of wave cycles that the SQ_* cycle counters give
"""
from __future__ import annotations

import argparse
import csv
import re
import statistics


def short_name(name: str, width: int = 110) -> str:
    n = re.sub(r"okd::\(anonymous namespace\)::", "", name).replace("okd::", "")
    return n if len(n) <= width else n[: width - 3] + "..."


def stats(path: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"total kernel time {tot / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} "
           f"dispatches", f"{'ms':>9} {'%':>5} {'calls':>6} {'avg us':>9}  kernel"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        out.append(f"{t / 1e6:9.3f} {100 * t / tot:5.1f} {int(r['Calls']):6d} "
                   f"{float(r['AverageNs']) / 1e3:9.2f}  {short_name(r['Name'])}")
    return "\n".join(out)


def bygrid(path: str, top: int = 40) -> str:
    acc = {}
    for r in csv.DictReader(open(path)):
        g = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
        t = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        k = (r["Kernel_Name"], g)
        n, s = acc.get(k, (0, 0))
        acc[k] = (n + 1, s + t)
    tot = sum(s for _, s in acc.values())
    out = [f"total kernel time {tot / 1e6:.2f} ms over {sum(n for n, _ in acc.values())} "
           f"dispatches", f"{'ms':>9} {'%':>5} {'calls':>6} {'avg us':>9} {'grid':>9}  kernel"]
    for (name, g), (n, s) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{s / 1e6:9.3f} {100 * s / tot:5.1f} {n:6d} {s / n / 1e3:9.2f} {g:9d}  "
                   f"{short_name(name, 100)}")
    return "\n".join(out)


def ranges(path: str) -> str:
    acc = {}
    for r in csv.DictReader(open(path)):
        name = r.get("Message") or r.get("Function") or ""
        t = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if t <= 0:  # instantaneous markers
            continue
        acc.setdefault(name, []).append(t)
    out = [f"{'count':>6} {'total ms':>10} {'mean us':>9} {'p50 us':>9} {'p99 us':>9}  range"]
    for name, ts in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        ts.sort()
        p99 = ts[min(len(ts) - 1, int(0.99 * len(ts)))]
        out.append(f"{len(ts):6d} {sum(ts) / 1e6:10.3f} {statistics.mean(ts) / 1e3:9.1f} "
                   f"{statistics.median(ts) / 1e3:9.1f} {p99 / 1e3:9.1f}  {name}")
    return "\n".join(out)


def _counter(path: str, counter: str, substrings=None, exclude=()):
    vals = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        if substrings is not None and not any(k in r["Kernel_Name"] for k in substrings):
            continue
        if any(k in r["Kernel_Name"] for k in exclude):
            continue
        vals.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return vals


def _copy_scale(path: str, counter: str, nbytes: int) -> float:
    """Bytes per counter unit: the copy dispatches (the largest grid) of the
    calibration run, median counter value."""
    vals = _counter(path, counter)
    big = max(g for _, g, _ in vals)
    v = statistics.median(x for _, g, x in vals if g == big)
    return nbytes / v


def traffic(fetch, write, copy_fetch, copy_write, copy_bytes, kernel, main_grid=False,
            exclude=()):
    sf = _copy_scale(copy_fetch, "FETCH_SIZE", copy_bytes)
    sw = _copy_scale(copy_write, "WRITE_SIZE", copy_bytes)
    kernels = [kernel] if isinstance(kernel, str) else list(kernel)
    f = _counter(fetch, "FETCH_SIZE", kernels, exclude)
    w = _counter(write, "WRITE_SIZE", kernels, exclude)
    if not f or not w:
        raise SystemExit(f"no dispatch of a kernel containing {kernel!r}")
    if main_grid:  # per run: the two runs may have tuned different launch shapes
        def main(vals):
            sizes = [x[1] for x in vals]
            g = max(set(sizes), key=sizes.count)
            return [x for x in vals if x[1] == g]
        f, w = main(f), main(w)
    fb = statistics.mean(x for _, _, x in f) * sf
    wb = statistics.mean(x for _, _, x in w) * sw
    names = sorted({short_name(x[0], 80) for x in f + w})
    return {"kernel": "; ".join(names), "grid_size": sorted({f[0][1], w[0][1]}),
            "dispatches": [len(f), len(w)],
            "fetch_scale_bytes_per_unit": sf, "write_scale_bytes_per_unit": sw,
            "fetch_bytes_per_dispatch": fb, "write_bytes_per_dispatch": wb,
            "traffic_bytes_per_dispatch": fb + wb}


def counters(paths, kernels, grid_size=None) -> str:
    by = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if not any(k in name for k in kernels):
                continue
            by.setdefault(name, []).append((int(r["Grid_Size"]), r["Counter_Name"],
                                            float(r["Counter_Value"])))
    if not by:
        raise SystemExit(f"no dispatch of a kernel containing {kernels!r}")
    out = []
    for name, rows in sorted(by.items()):
        sizes = [g for g, _, _ in rows]
        grid = grid_size if grid_size else max(set(sizes), key=sizes.count)
        if grid not in sizes:
            continue
        vals = {}
        for g, c, v in rows:
            if g == grid:
                vals.setdefault(c, []).append(v)
        d = {c: statistics.mean(v) for c, v in vals.items()}
        out.append(f"kernel: {short_name(name)}")
        out.append(f"  grid {grid}, dispatches per counter {min(len(v) for v in vals.values())}")
        for c in sorted(d):
            out.append(f"  {c}: {d[c]:.0f}")
        w = d.get("SQ_WAVES")
        if w:
            per = [f"{d[c] / w:.0f} {c[9:]}" for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU",
                                                         "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
                                                         "SQ_INSTS_VMEM_WR") if c in d]
            out.append("  per wavefront: " + ", ".join(per))
        wc = d.get("SQ_WAVE_CYCLES")
        if wc:
            sh = [f"{c[3:].lower()} {100 * d[c] / wc:.0f}%" for c in
                  ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_SCA",
                   "SQ_ACTIVE_INST_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY") if c in d]
            if sh:
                out.append("  of wave cycles: " + ", ".join(sh))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("top", nargs="?", type=int, default=25)
    e = sub.add_parser("counters")
    e.add_argument("--csv", action="append", required=True)
    e.add_argument("--kernel", action="append", required=True)
    e.add_argument("--grid", type=int, default=0)
    c = sub.add_parser("bygrid")
    c.add_argument("csv")
    c.add_argument("top", nargs="?", type=int, default=40)
    d = sub.add_parser("ranges")
    d.add_argument("csv")
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        b.add_argument("--" + k, required=True)
    b.add_argument("--kernel", action="append", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--main-grid", action="store_true")
    b.add_argument("--exclude", action="append", default=[])
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.top))
    elif args.cmd == "bygrid":
        print(bygrid(args.csv, args.top))
    elif args.cmd == "ranges":
        print(ranges(args.csv))
    elif args.cmd == "counters":
        print(counters(args.csv, args.kernel, args.grid))
    else:
        r = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_bytes,
                    args.kernel, args.main_grid, args.exclude)
        for k, v in r.items():
            print(f"{k}: {v}")


if __name__ == "__main__":
    main()
