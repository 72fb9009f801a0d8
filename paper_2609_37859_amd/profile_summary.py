"""Summaries of rocprofv3 output for the stage kernel.

Reads the CSV files rocprofv3 writes (`--output-format csv`): the kernel
statistics of a `--kernel-trace --stats` run, and the per-dispatch
`FETCH_SIZE` / `WRITE_SIZE` counters (KiB) of two `--pmc` runs of the same
command, plus the same counters for a plain device copy of known size.  The
copy gives the factor from counter units to HBM bytes for each counter.
Writes a short text summary (and, with --json, the per-launch HBM bytes and
the hash of the kernel sources they were taken on).

  python -m paper_2609_37859_amd.profile_summary --stats DIR --fetch DIR --write DIR \
      --copy-fetch DIR --copy-write DIR --copy-bytes N --kernel stage_tiled --cmd "..." \
      --out profiles/x.md [--json profiles/x.json]
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash(family="stage"):
    """Hash of the sources the counters depend on (stage kernel or multigrid)."""
    files = ("tdh_kernels.hip", "tdh_internal.hpp") if family == "stage" else ("tdh_gravity.hip", "tdh_internal.hpp")
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2609_37859_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def family_summary(args):
    """Every kernel whose name contains args.family: calls and time, and with
    counter runs its HBM bytes (total, and per unit of work: the run's
    total divided by args.units)."""
    rows = [r for r in csv.DictReader(open(_one(args.stats, "*kernel_stats.csv"))) if args.family in r["Name"]]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {args.title}", "", "Commands:", ""] + [f"    {c}" for c in args.cmd]
    lines += ["", "Kernel statistics (rocprofv3 --kernel-trace --stats):", "",
              "| kernel | calls | average ms | total ms | HBM read MB (all calls) | HBM written MB (all calls) |",
              "|---|---|---|---|---|---|"]
    f_k = copy_factor(args.copy_fetch, "FETCH_SIZE", args.copy_bytes) if args.copy_fetch else None
    w_k = copy_factor(args.copy_write, "WRITE_SIZE", args.copy_bytes) if args.copy_write else None
    tot_r = tot_w = 0.0
    fe = {}
    wr = {}
    if args.fetch and f_k:
        for r in csv.DictReader(open(_one(args.fetch, "*counter_collection.csv"))):
            if r["Counter_Name"] == "FETCH_SIZE":
                fe[r["Kernel_Name"]] = fe.get(r["Kernel_Name"], 0.0) + float(r["Counter_Value"]) * f_k
    if args.write and w_k:
        for r in csv.DictReader(open(_one(args.write, "*counter_collection.csv"))):
            if r["Counter_Name"] == "WRITE_SIZE":
                wr[r["Kernel_Name"]] = wr.get(r["Kernel_Name"], 0.0) + float(r["Counter_Value"]) * w_k
    total_ms = 0.0
    for r in rows:
        rb, wb = fe.get(r["Name"], 0.0), wr.get(r["Name"], 0.0)
        tot_r += rb
        tot_w += wb
        total_ms += float(r["TotalDurationNs"]) / 1e6
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} |")
    out = {"family": args.family, "kernel_hash": kernel_source_hash("gravity"), "total_ms": total_ms}
    lines += ["", f"All {args.family} kernels: {total_ms:.3f} ms"]
    if fe:
        per = (tot_r + tot_w) / max(args.units, 1)
        lines += [f"HBM traffic (copy-calibrated counters, factors {f_k:.4f} / {w_k:.4f} B per unit): "
                  f"{tot_r / 1e6:.1f} MB read + {tot_w / 1e6:.1f} MB written; over {args.units} {args.unit_name}: "
                  f"{per / 1e6:.1f} MB per {args.unit_name[:-1] if args.unit_name.endswith('s') else args.unit_name}"]
        out.update({"hbm_read_bytes": tot_r, "hbm_write_bytes": tot_w, "units": args.units,
                    "hbm_bytes_per_unit": per, "ms_per_unit": total_ms / max(args.units, 1)})
    lines += ["", f"Kernel source hash: {out['kernel_hash']}"]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    print("\n".join(lines))


def _one(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits[0]


def kernel_stats(d, kernel):
    """Rows of the stats file whose name contains `kernel`; the variant with the
    most calls is the one the run used after tuning."""
    rows = [r for r in csv.DictReader(open(_one(d, "*kernel_stats.csv"))) if kernel in r["Name"]]
    if not rows:
        raise SystemExit(f"kernel {kernel} not in the stats of {d}")
    rows.sort(key=lambda r: -int(r["Calls"]))
    return rows


def _tail(vals, last):
    return vals[-last:] if last > 0 else vals


def trace_durations(d, name_exact):
    """Durations (ms) of the dispatches of one kernel in dispatch order, from
    the kernel trace."""
    rows = [r for r in csv.DictReader(open(_one(d, "*kernel_trace.csv"))) if r["Kernel_Name"] == name_exact]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows]


def counter_per_dispatch(d, name_exact, counter, last=0):
    rows = [r for r in csv.DictReader(open(_one(d, "*counter_collection.csv")))
            if r["Kernel_Name"] == name_exact and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    vals = _tail([float(r["Counter_Value"]) for r in rows], last)
    if not vals:
        raise SystemExit(f"no {counter} for {name_exact} under {d}")
    return vals


def counter_table(d, kernel, last=0):
    """{counter: [values per dispatch]} for the dispatches of `kernel` (the
    last `last` of them if last > 0), in dispatch order."""
    rows = [r for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))) if r["Kernel_Name"] == kernel]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    out = {}
    for r in rows:
        out.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: _tail(v, last) for k, v in out.items()}


def copy_factor(d, counter, nbytes):
    """HBM bytes per counter unit, from the largest copy dispatch of the calibration run."""
    best = 0.0
    for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))):
        if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter:
            best = max(best, float(r["Counter_Value"]))
    if best <= 0:
        raise SystemExit(f"no copy dispatch with {counter} under {d}")
    return nbytes / best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--kernel", default="stage_tiled")
    ap.add_argument("--sq", action="append", default=[], help="directory of a --pmc run of SQ counters (repeatable)")
    ap.add_argument("--cells", type=float, default=0.0, help="cells one launch of the kernel updates (per-cell rates)")
    ap.add_argument("--windows", type=int, default=0, help="LAT windows in the run: list every kernel per window")
    ap.add_argument("--alg-bytes", type=float, default=0.0,
                    help="algorithmic HBM bytes of the kernel's launches the figures cover (all, or --last N)")
    ap.add_argument("--cmd", action="append", default=[], help="command that produced the inputs (repeatable)")
    ap.add_argument("--title", default="stage kernel")
    ap.add_argument("--out", required=True)
    ap.add_argument("--json")
    ap.add_argument("--family", help="summarise every kernel whose name contains this (instead of one kernel)")
    ap.add_argument("--units", type=int, default=1, help="units of work in the run (family mode)")
    ap.add_argument("--unit-name", default="units")
    ap.add_argument("--last", type=int, default=0,
                    help="per-launch figures over the kernel's last N dispatches only (a timed pass at the end "
                         "of the run); 0: every dispatch")
    args = ap.parse_args()
    if args.family:
        family_summary(args)
        return

    rows = kernel_stats(args.stats, args.kernel)
    used = rows[0]
    lines = [f"# {args.title}", "", "Commands:", ""]
    lines += [f"    {c}" for c in args.cmd]
    lines += ["", "Kernel statistics (rocprofv3 --kernel-trace --stats):", "",
              "| kernel | calls | average ms | min ms | max ms |", "|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} |")
    lines += ["", f"Variant used after tuning: `{used['Name']}`, average {float(used['AverageNs']) / 1e6:.4f} ms "
                  f"over {used['Calls']} launches.", ""]
    if args.windows > 0:
        allrows = [r for r in csv.DictReader(open(_one(args.stats, "*kernel_stats.csv"))) if "tdh::" in r["Name"]]
        allrows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines += [f"Every library kernel of the run, per window ({args.windows} windows; the network's training "
                  "kernels ran once before them):", "", "| kernel | calls | ms per window |", "|---|---|---|"]
        for r in allrows:
            nm = r["Name"].split("(")[0]
            lines.append(f"| `{nm}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6 / args.windows:.3f} |")
        lines.append("")
    out = {"kernel": used["Name"], "avg_launch_ms": float(used["AverageNs"]) / 1e6, "kernel_hash": kernel_source_hash()}
    if args.last > 0:
        dur = _tail(trace_durations(args.stats, used["Name"]), args.last)
        lines += [f"Timed launches (the last {len(dur)} dispatches of `{used['Name']}`, the run's HIP-event "
                  f"pass): average {statistics.mean(dur):.4f} ms, min {min(dur):.4f}, max {max(dur):.4f}, "
                  f"sum {sum(dur):.2f} ms", ""]
        out["avg_launch_ms_all"] = out["avg_launch_ms"]
        out["avg_launch_ms"] = statistics.mean(dur)
        out["launches"] = len(dur)
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        f_k = copy_factor(args.copy_fetch, "FETCH_SIZE", args.copy_bytes)
        w_k = copy_factor(args.copy_write, "WRITE_SIZE", args.copy_bytes)
        fv = counter_per_dispatch(args.fetch, used["Name"], "FETCH_SIZE", args.last)
        wv = counter_per_dispatch(args.write, used["Name"], "WRITE_SIZE", args.last)
        fb, wb = statistics.mean(fv) * f_k, statistics.mean(wv) * w_k
        lines += ["HBM traffic per launch (counter runs of the same command, copy-calibrated):", "",
                  f"- FETCH_SIZE: mean {statistics.mean(fv):.1f} KiB over {len(fv)} launches; copy factor "
                  f"{f_k:.4f} B per unit -> {fb / 1e6:.2f} MB read",
                  f"- WRITE_SIZE: mean {statistics.mean(wv):.1f} KiB over {len(wv)} launches; copy factor "
                  f"{w_k:.4f} B per unit -> {wb / 1e6:.2f} MB written",
                  f"- total {(fb + wb) / 1e6:.2f} MB per launch", ""]
        out.update({"hbm_read_bytes_per_launch": fb, "hbm_write_bytes_per_launch": wb,
                    "hbm_bytes_per_launch": fb + wb, "fetch_factor": f_k, "write_factor": w_k})
        if args.alg_bytes > 0:
            ratio = (fb + wb) * len(fv) / args.alg_bytes
            lines += [f"- against the algorithmic bytes of those launches ({args.alg_bytes / 1e9:.1f} GB): "
                      f"{ratio:.2f} x", ""]
            out["traffic_over_algorithmic"] = ratio
    for d in args.sq:
        tab = counter_table(d, used["Name"], args.last)
        if not tab:
            continue
        lines += [f"SQ counters per launch ({d.rstrip('/').split('/')[-1]}):", ""]
        for k, v in sorted(tab.items()):
            mean = statistics.mean(v)
            per = f", {mean / args.cells:.1f} per cell" if args.cells > 0 else ""
            lines.append(f"- {k}: mean {mean:.4g} over {len(v)} launches{per}")
            out.setdefault("sq", {})[k] = mean
        lines.append("")
    lines.append(f"Kernel source hash: {out['kernel_hash']}")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
