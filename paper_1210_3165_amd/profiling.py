"""Summaries of rocprofv3 output for the committed profiles.

    # kernel-trace summary (markdown) of a `rocprofv3 --kernel-trace --stats
    # --output-format csv -d DIR -o PREFIX -- <command>` run
    python -m paper_1210_3165_amd.profiling trace DIR PREFIX --title T --command C

    # HBM traffic per dispatch from two counter runs (FETCH_SIZE, WRITE_SIZE),
    # scaled by what the same counters read for the plain device copy that ran
    # in the same process (16 MiB each way)
    python -m paper_1210_3165_amd.profiling traffic FETCH_CSV WRITE_CSV --kernel SUBSTR ...

    # instruction mix per dispatch from one SQ counter run (SQ_INSTS_VALU and
    # friends count wave instructions; x64 gives lane instructions)
    python -m paper_1210_3165_amd.profiling valu SQ_CSV --kernel SUBSTR --pixels N ...

Only reads CSV files; runs nothing on the GPU.
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics
import sys
from collections import defaultdict

from .build import kernel_source_sha

COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("void ", "")


def _pct(v, q: float) -> float:
    """q-th percentile of v by linear interpolation between order statistics."""
    s = sorted(v)
    if len(s) == 1:
        return s[0]
    x = (len(s) - 1) * q / 100.0
    i = int(x)
    j = min(i + 1, len(s) - 1)
    return s[i] + (s[j] - s[i]) * (x - i)


def trace_summary(d: str, prefix: str, title: str, command: str, note: str = "",
                  only: tuple[str, ...] = ("bz_", "otsu_", "__amd_rocclr_copyBuffer")) -> str:
    stats = _rows(f"{d}/{prefix}_kernel_stats.csv")
    trace = _rows(f"{d}/{prefix}_kernel_trace.csv")
    out = [f"# {title}", "", "Command (repository root, one MI355X):", "", f"    {command}", ""]
    if note:
        out += [note, ""]
    out += ["## kernel_stats.csv (this library's kernels and the device copy)", "", "| Kernel | Calls | Average ns | Min ns | Max ns | % |",
            "|---|---|---|---|---|---|"]
    for r in stats:
        if not any(o in r["Name"] for o in only):
            continue
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | "
                   f"{r['MaxNs']} | {float(r['Percentage']):.1f} |")
    groups = defaultdict(list)
    meta = {}
    for r in trace:
        if not any(o in r["Kernel_Name"] for o in only):
            continue
        key = (_short(r["Kernel_Name"]).split("(")[0], int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        groups[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        meta[key] = (r["LDS_Block_Size"], r["VGPR_Count"], r["SGPR_Count"])
    out += ["", "## per launch shape (kernel_trace.csv)", "",
            "| Kernel | grid threads | workgroup | LDS bytes | VGPR | SGPR | launches | mean us | median us "
            "| p10 us | p90 us |",
            "|---|---|---|---|---|---|---|---|---|---|---|"]
    per_name = defaultdict(list)
    for key in groups:
        per_name[key[0]].append(key)
    for name in sorted(per_name):
        keys = sorted(per_name[name], key=lambda k: -k[1])
        if len(keys) > 8:  # many launch shapes (uneven pages): one aggregate row
            v = [x for k in keys for x in groups[k]]
            lds, vg, sg = meta[keys[0]]
            out.append(f"| `{name}` | {len(keys)} shapes, {min(k[1] for k in keys)}..{max(k[1] for k in keys)} | "
                       f"{keys[0][2]} | {lds} | {vg} | {sg} | {len(v)} | {statistics.mean(v):.1f} | "
                       f"{statistics.median(v):.1f} | {_pct(v, 10):.1f} | {_pct(v, 90):.1f} |")
            continue
        for key in keys:
            v = groups[key]
            lds, vg, sg = meta[key]
            out.append(f"| `{key[0]}` | {key[1]} | {key[2]} | {lds} | {vg} | {sg} | {len(v)} | "
                       f"{statistics.mean(v):.1f} | {statistics.median(v):.1f} | {_pct(v, 10):.1f} | "
                       f"{_pct(v, 90):.1f} |")
    return "\n".join(out) + "\n"


def overlap_summary(d: str, prefix: str, kernel: str, min_launches: int = 1) -> str:
    """Runs of consecutive dispatches of one kernel and launch shape, in start
    order: per run the launches, their mean duration, the run's span (first
    start to last end), the summed durations over the span (the mean number
    of launches in flight) and the share of the span with two or more in
    flight, for runs of at least min_launches.  A markdown table."""
    rows = [r for r in _rows(f"{d}/{prefix}_kernel_trace.csv") if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    runs = []
    for r in rows:
        key = (_short(r["Kernel_Name"]).split("(")[0], int(r["Grid_Size_X"]))
        iv = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
        if runs and runs[-1][0] == key:
            runs[-1][1].append(iv)
        else:
            runs.append((key, [iv]))
    out = ["| run | kernel | grid threads | launches | mean us | span us | span / launch us "
           "| in flight (mean) | span with 2+ in flight |",
           "|---|---|---|---|---|---|---|---|---|"]
    for i, ((name, grid), ivs) in enumerate(runs):
        if len(ivs) < min_launches:
            continue
        t0, t1 = min(a for a, _ in ivs), max(b for _, b in ivs)
        busy = sum(b - a for a, b in ivs)
        ev = sorted([(a, 1) for a, _ in ivs] + [(b, -1) for _, b in ivs])
        depth, last, multi = 0, t0, 0
        for t, dlt in ev:
            if depth >= 2:
                multi += t - last
            depth += dlt
            last = t
        span = max(t1 - t0, 1)
        out.append(f"| {i} | `{name}` | {grid} | {len(ivs)} | {busy / len(ivs) / 1e3:.1f} | {span / 1e3:.1f} | "
                   f"{span / len(ivs) / 1e3:.1f} | {busy / span:.2f} | {multi / span:.2f} |")
    return "\n".join(out) + "\n"


def _counter(path, counter):
    per = defaultdict(list)
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        per[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return per


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, workload: str,
            commands: list[str], sources: tuple[str, ...]) -> dict:
    fetch = _counter(fetch_csv, "FETCH_SIZE")
    write = _counter(write_csv, "WRITE_SIZE")

    def pick(per, sub):
        vals, grids = [], {}
        names = set()
        for (n, g), v in per.items():
            if sub in n:
                vals += v
                grids.setdefault(g, []).extend(v)
                names.add(n)
        return sorted(names), vals, grids

    cf = [v for (n, _), vs in fetch.items() if n == COPY_KERNEL for v in vs]
    cw = [v for (n, _), vs in write.items() if n == COPY_KERNEL for v in vs]
    names, kf, grids = pick(fetch, kernel)
    _, kw, _ = pick(write, kernel)
    if not (cf and cw and kf and kw):
        raise SystemExit("missing copy or kernel dispatches in the counter files")
    copy_kib = copy_bytes / 1024
    fs, ws = copy_kib / statistics.median(cf), copy_kib / statistics.median(cw)
    f_raw, w_raw = statistics.mean(kf), statistics.mean(kw)
    return {
        "kernel": kernel,
        "kernels": names,
        "workload": workload,
        "source_sha": kernel_source_sha(sources),
        "fetch_kib_per_dispatch_raw": round(f_raw, 1),
        "write_kib_per_dispatch_raw": round(w_raw, 1),
        "copy_fetch_kib_raw": round(statistics.median(cf), 1),
        "copy_write_kib_raw": round(statistics.median(cw), 1),
        "copy_bytes_each_way": copy_bytes,
        "fetch_scale": round(fs, 4),
        "write_scale": round(ws, 4),
        "bytes_per_launch": int(round((f_raw * fs + w_raw * ws) * 1024)),
        "per_grid_fetch_kib_raw": {str(g): round(statistics.mean(v), 1) for g, v in sorted(grids.items())},
        "commands": commands,
    }


# Counters of the instruction-mix record (one pass); SQ_INSTS_VALU is
# required.  A second pass may add the wave-state counters (SQ_WAVE_CYCLES,
# SQ_WAIT_ANY, ...), which the record then carries too.
SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES")


def valu(sq_csvs, kernel: str, pixels: int, workload: str, commands: list[str],
         sources: tuple[str, ...]) -> dict:
    """Mean counter values per dispatch of the kernels whose name contains
    `kernel`, over one or more SQ counter runs (every counter found in them),
    and VALU lane instructions per output pixel (wave instructions x 64
    lanes / pixels per dispatch)."""
    if pixels <= 0:
        raise SystemExit("pixels per dispatch must be positive")
    if isinstance(sq_csvs, str):
        sq_csvs = [sq_csvs]
    names, means = set(), {}
    for path in sq_csvs:
        counters = sorted({r["Counter_Name"] for r in _rows(path)})
        for c in counters:
            vals = []
            for (n, _), vs in _counter(path, c).items():
                if kernel in n:
                    vals += vs
                    names.add(n)
            if vals:
                means[c] = statistics.mean(vals)
    if "SQ_INSTS_VALU" not in means:
        raise SystemExit(f"no SQ_INSTS_VALU rows for a kernel matching {kernel!r}")
    return {
        "kernel": kernel,
        "kernels": sorted(names),
        "workload": workload,
        "source_sha": kernel_source_sha(sources),
        "pixels_per_dispatch": pixels,
        "per_dispatch": {c: round(v, 1) for c, v in means.items()},
        "valu_lane_ops_per_px": round(means["SQ_INSTS_VALU"] * 64 / pixels, 3),
        "commands": commands,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("prefix")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--note", default="")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_csv")
    f.add_argument("write_csv")
    f.add_argument("--kernel", required=True, help="substring of the kernel name")
    f.add_argument("--copy-bytes", type=int, default=16 * 2**20)
    f.add_argument("--workload", required=True)
    f.add_argument("--command", action="append", default=[])
    f.add_argument("--sources", default="binarize.hip,bz_common.hpp,bz_tile.hpp")
    o = sub.add_parser("overlap")
    o.add_argument("dir")
    o.add_argument("prefix")
    o.add_argument("--kernel", required=True, help="substring of the kernel name")
    o.add_argument("--min-launches", type=int, default=1)
    v = sub.add_parser("valu")
    v.add_argument("sq_csv", nargs="+")
    v.add_argument("--kernel", required=True, help="substring of the kernel name")
    v.add_argument("--pixels", type=int, required=True, help="output pixels per dispatch")
    v.add_argument("--workload", required=True)
    v.add_argument("--command", action="append", default=[])
    v.add_argument("--sources", default="binarize.hip,bz_common.hpp,bz_tile.hpp")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        sys.stdout.write(trace_summary(a.dir, a.prefix, a.title, a.command, a.note))
    elif a.cmd == "overlap":
        sys.stdout.write(overlap_summary(a.dir, a.prefix, a.kernel, a.min_launches))
    elif a.cmd == "valu":
        rec = valu(a.sq_csv, a.kernel, a.pixels, a.workload, a.command, tuple(a.sources.split(",")))
        sys.stdout.write(json.dumps(rec, indent=1) + "\n")
    else:
        rec = traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.workload, a.command,
                      tuple(a.sources.split(",")))
        sys.stdout.write(json.dumps(rec, indent=1) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
