"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1712_08743_amd.profiling stats TRACE_CSV --command CMD [--out FILE.md]
    python -m paper_1712_08743_amd.profiling traffic --fetch CSV --write CSV \\
        --copy-fetch CSV --copy-write CSV --copy-bytes N --rhs R --command CMD \\
        [--out FILE.md] [--json FILE.json]

    python -m paper_1712_08743_amd.profiling stalls CSV [CSV ...] --command CMD [--out FILE.md]
    python -m paper_1712_08743_amd.profiling gmres-traffic --fetch CSV --write CSV \\
        --copy-fetch CSV --copy-write CSV --copy-bytes N --steps S --report JSON --command CMD \\
        [--out FILE.md] [--json FILE.json]

``stats`` reads a ``--kernel-trace`` CSV and tabulates, per kernel symbol,
the launches, total and average duration; the finest-level kernels are named
by their timing class (``hz_timing_*``). ``traffic`` reads two ``--pmc``
counter-collection CSVs (FETCH_SIZE, WRITE_SIZE, in KiB per dispatch) of a
solve whose every launch carries ``R`` right-hand sides, scales each counter
by what it reads for the library's plain copy kernel of ``N`` bytes read and
``N`` written, and reports bytes per dispatch and per right-hand side. ``stalls`` reads
``--pmc`` runs of the SQ wave counters and tabulates, per kernel, where its
waves spend their cycles and the instructions each wave issues.
``gmres-traffic`` sums the two counters over every dispatch of GMRES's
Gram-Schmidt step kernels and compares the bytes per step with the
algorithmic bytes of the ``bench.py --gmres`` report of the same run
(``--json``: the bytes per step with the kernel source hash, which
``bench.py --gmres`` reports as its roofline's traffic while the hash holds).
"""

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))

# timing class -> kernel symbol(s) (finest level); a class with two symbols
# launches each of them every second iteration
# (the constant-density forms: the last template argument is the density flag)
CLASS_SYMBOL = {
    "presmooth": "hz::k_pre2r_s<4, true, false>",
    "presmooth_s": "hz::k_pre2r_s<5, true, false>",
    "prolong": "hz::k_post2_s<true, false>",
    "apply": "hz::k_bicg_apply_t<0, false>",
    "apply_s": "hz::k_bicg_apply_t<1, false>",
    "update": ("hz::k_bicg_xr_t<0, false>", "hz::k_bicg_xr_t<1, false>"),
    "coarse": "hz::k_coarse",
}


def _code_only(text):
    """C++ source without its comments and with whitespace runs collapsed
    (string literals in these files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the kernel sources' code (comments and layout left out); a
    traffic measurement is valid for it only."""
    h = hashlib.sha256()
    for f in ("hz_kernels.hip", "hz_stream.hip", "hz_krylov.hip", "hz_device.h", "hz_internal.h"):
        with open(os.path.join(HERE, "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def symbol(name):
    """Kernel symbol without the parameter list and the leading 'void '."""
    s = name.split("(")[0].strip()
    return s[5:] if s.startswith("void ") else s


def symbols_of(cls):
    v = CLASS_SYMBOL[cls]
    return v if isinstance(v, tuple) else (v,)


def class_of(sym):
    for k in CLASS_SYMBOL:
        if sym in symbols_of(k):
            return k
    return ""


def window(rows, marker, first, last):
    """Rows that start at or after the first-th launch of kernel `marker` and
    before its last-th (1-based), e.g. the timed steps of a benchmark whose
    every step launches the marker once."""
    starts = sorted(int(r["Start_Timestamp"]) for r in rows if symbol(r["Kernel_Name"]) == marker)
    lo = starts[first - 1] if first - 1 < len(starts) else None
    hi = starts[last - 1] if last - 1 < len(starts) else None
    return [r for r in rows if (lo is None or int(r["Start_Timestamp"]) >= lo)
            and (hi is None or int(r["Start_Timestamp"]) < hi)]


def stats(trace_csv, between=None):
    agg = collections.OrderedDict()
    rows = list(csv.DictReader(open(trace_csv)))
    if between:
        rows = window(rows, *between)
    for r in rows:
        s = symbol(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6  # ms
        a = agg.setdefault(s, [0, 0.0])
        a[0] += 1
        a[1] += d
    return sorted(agg.items(), key=lambda kv: -kv[1][1])


def counters(csv_path, largest=False):
    """kernel symbol -> list of counter values (KiB per dispatch), over the
    dispatches with the symbol's most frequent grid size (a launch-shape
    tuner's trial launches of other shapes are left out), or with its largest
    grid size (largest: the finest level with the whole batch, where a
    kernel also runs on the coarser levels)."""
    by = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(csv_path)):
        by[symbol(r["Kernel_Name"])][int(r["Grid_Size"])].append(float(r["Counter_Value"]))
    out = {}
    for sym, grids in by.items():
        out[sym] = grids[max(grids)] if largest else max(grids.values(), key=len)
    return out


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, rhs, largest=False):
    F, W = counters(fetch_csv, largest), counters(write_csv, largest)
    cF, cW = counters(copy_fetch_csv), counters(copy_write_csv)
    cf = cF["hz::k_copy"]
    cw = cW["hz::k_copy"]
    ffac = copy_bytes / (1024.0 * sum(cf) / len(cf))
    wfac = copy_bytes / (1024.0 * sum(cw) / len(cw))
    rows = {}
    for sym, vals in F.items():
        wv = W.get(sym, [])
        if not wv:
            continue
        fb = 1024.0 * ffac * sum(vals) / len(vals)
        wb = 1024.0 * wfac * sum(wv) / len(wv)
        rows[sym] = {"dispatches": len(vals), "fetch_bytes": fb, "write_bytes": wb,
                     "fetch_bytes_per_rhs": fb / rhs, "write_bytes_per_rhs": wb / rhs}
    return {"fetch_factor": ffac, "write_factor": wfac, "kernels": rows}


GMRES_STEP_KERNELS = ("hz::k_gm_dots2", "hz::k_gm_fin2", "hz::k_gm_update2")


def counter_totals(csv_path, symbols):
    """symbol -> (dispatches, summed counter value in KiB) over every dispatch."""
    out = {s: [0, 0.0] for s in symbols}
    for r in csv.DictReader(open(csv_path)):
        s = symbol(r["Kernel_Name"])
        if s in out:
            out[s][0] += 1
            out[s][1] += float(r["Counter_Value"])
    return out


def gmres_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, steps):
    """HBM bytes per step of GMRES's Gram-Schmidt step kernels: FETCH_SIZE and
    WRITE_SIZE summed over all their dispatches (their grids shrink as the
    right-hand sides converge), scaled by the copy kernel, over `steps`
    identical GMRES solves of the profiled run."""
    cF, cW = counters(copy_fetch_csv), counters(copy_write_csv)
    cf, cw = cF["hz::k_copy"], cW["hz::k_copy"]
    ffac = copy_bytes / (1024.0 * sum(cf) / len(cf))
    wfac = copy_bytes / (1024.0 * sum(cw) / len(cw))
    F = counter_totals(fetch_csv, GMRES_STEP_KERNELS)
    W = counter_totals(write_csv, GMRES_STEP_KERNELS)
    rows = {}
    for s in GMRES_STEP_KERNELS:
        rows[s] = {"dispatches": F[s][0], "fetch_bytes_per_step": 1024.0 * ffac * F[s][1] / steps,
                   "write_bytes_per_step": 1024.0 * wfac * W[s][1] / steps}
    return {"fetch_factor": ffac, "write_factor": wfac, "kernels": rows}


def _gmres_traffic_md(t, command, algorithmic_gb):
    lines = ["# HBM traffic of GMRES(30)'s Gram-Schmidt step kernels (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)",
             "", "Commands:", "", "```", command, "```", "",
             f"Counters summed over every dispatch and scaled by the library's copy kernel (FETCH_SIZE x "
             f"{t['fetch_factor']:.4f}, WRITE_SIZE x {t['write_factor']:.4f}), per GMRES step of the "
             "benchmark batch (256 right-hand sides, all four frequencies).", "",
             "| kernel | dispatches | read GB/step | write GB/step |", "|---|---:|---:|---:|"]
    tot = 0.0
    for s, r in t["kernels"].items():
        lines.append(f"| `{s}` | {r['dispatches']} | {r['fetch_bytes_per_step'] / 1e9:.1f} | "
                     f"{r['write_bytes_per_step'] / 1e9:.1f} |")
        tot += r["fetch_bytes_per_step"] + r["write_bytes_per_step"]
    lines += ["", f"Measured: {tot / 1e9:.1f} GB per step; algorithmic (the dot pass reads j + 2 vectors, the "
              f"update pass reads j + 2 and writes 2, per right-hand side and Arnoldi step j): "
              f"{algorithmic_gb:.1f} GB per step; ratio {tot / 1e9 / algorithmic_gb:.3f}."]
    return "\n".join(lines) + "\n"


def counter_means(csv_paths):
    """kernel symbol -> (grid size, dispatches, {counter: mean per dispatch}) over
    the dispatches with the symbol's most frequent grid size, from one or more
    ``--pmc`` counter-collection CSVs (one row per counter and dispatch)."""
    by = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(list)))
    ids = collections.defaultdict(lambda: collections.defaultdict(set))  # dispatches per run
    for run, path in enumerate(csv_paths):
        for r in csv.DictReader(open(path)):
            sym, g = symbol(r["Kernel_Name"]), int(r["Grid_Size"])
            by[sym][g][r["Counter_Name"]].append(float(r["Counter_Value"]))
            ids[sym][g].add((run, r["Dispatch_Id"]))
    out = {}
    for sym, grids in by.items():
        g, cnt = max(grids.items(), key=lambda kv: max(len(v) for v in kv[1].values()))
        runs = collections.Counter(run for run, _ in ids[sym][g])
        out[sym] = (g, max(runs.values()), {k: sum(v) / len(v) for k, v in cnt.items()})
    return out


def _stalls_md(csv_paths, command, top=12):
    lines = ["# Wave stall counters (rocprofv3 --pmc)", "", "Commands:", "", "```", command, "```", "",
             "Per kernel, the dispatches with its most frequent grid size. Fractions are of `SQ_WAVE_CYCLES` "
             "(the counters count per wave, in the same units): `SQ_WAIT_ANY` = waiting at `s_waitcnt` (for "
             "loads), `SQ_WAIT_INST_ANY` = waiting for an instruction to issue, `SQ_ACTIVE_INST_ANY` / "
             "`_VALU` = issuing. Instructions are per wavefront.", "",
             "| kernel | grid | dispatches | wait (loads) | wait (issue) | active | active VALU | VALU instr. | "
             "VMEM reads | VMEM writes | SALU instr. |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    rows = counter_means(csv_paths)

    def cyc(item):
        g, n, c = item[1]
        return c.get("SQ_WAVE_CYCLES", 0.0) * n

    for sym, (g, n, c) in sorted(rows.items(), key=cyc, reverse=True)[:top]:
        wc, waves = c.get("SQ_WAVE_CYCLES"), c.get("SQ_WAVES")
        if not wc or not waves:
            continue

        def fr(k):
            return f"{c[k] / wc:.2f}" if k in c else ""

        def per_wave(k):
            return f"{c[k] / waves:.0f}" if k in c else ""

        lines.append(f"| `{sym}` | {g} | {n} | {fr('SQ_WAIT_ANY')} | {fr('SQ_WAIT_INST_ANY')} | "
                     f"{fr('SQ_ACTIVE_INST_ANY')} | {fr('SQ_ACTIVE_INST_VALU')} | {per_wave('SQ_INSTS_VALU')} | "
                     f"{per_wave('SQ_INSTS_VMEM_RD')} | {per_wave('SQ_INSTS_VMEM_WR')} | {per_wave('SQ_INSTS_SALU')} |")
    return "\n".join(lines) + "\n"


def _whole_run_md(stats_csv, top=15):
    lines = ["", "Whole run (the `--stats` summary: warm-up, launch-shape trials and every other launch "
             "included):", "", "| kernel | calls | total ms | average us |", "|---|---:|---:|---:|"]
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:top]:
        lines.append(f"| `{symbol(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.1f} | "
                     f"{float(r['AverageNs']) * 1e-3:.1f} |")
    return "\n".join(lines) + "\n"


def _stats_md(trace_csv, command, between=None):
    lines = ["# Kernel durations (rocprofv3 --kernel-trace)", "", "Command:", "", "```", command, "```", ""]
    if between:
        lines += [f"Launches from the {between[1]}-th launch of `{between[0]}` up to (not including) its "
                  f"{between[2]}-th.", ""]
    lines += ["| kernel | timing class | launches | total ms | average us |", "|---|---|---:|---:|---:|"]
    for s, (n, ms) in stats(trace_csv, between):
        lines.append(f"| `{s}` | {class_of(s)} | {n} | {ms:.1f} | {1e3 * ms / n:.1f} |")
    return "\n".join(lines) + "\n"


def _traffic_md(t, command, rhs, largest=False):
    lines = ["# HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)", "",
             "Commands:", "", "```", command, "```", "",
             f"Counters are scaled by the library's copy kernel: FETCH_SIZE x {t['fetch_factor']:.4f}, "
             f"WRITE_SIZE x {t['write_factor']:.4f} (bytes it moves / KiB the counter reads). " +
             (f"Per kernel the dispatches of its largest grid (the finest level), each carrying {rhs} "
              "right-hand sides. " if largest else f"Every dispatch carries {rhs} right-hand sides. ") +
             "Writes are counted when the L2 writes them back, which can be during a later kernel.", "",
             "| kernel | timing class | dispatches | read MB | write MB | read B/RHS/node | write B/RHS/node |",
             "|---|---|---:|---:|---:|---:|---:|"]
    n0 = t.get("nodes", 0)
    for s, r in sorted(t["kernels"].items(), key=lambda kv: -(kv[1]["fetch_bytes"] + kv[1]["write_bytes"])):
        per_node = (f"{r['fetch_bytes_per_rhs'] / n0:.1f} | {r['write_bytes_per_rhs'] / n0:.1f}" if n0 else " | ")
        lines.append(f"| `{s}` | {class_of(s)} | {r['dispatches']} | {r['fetch_bytes'] / 1e6:.1f} | "
                     f"{r['write_bytes'] / 1e6:.1f} | {per_node} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace")
    a.add_argument("--command", required=True)
    a.add_argument("--out")
    a.add_argument("--between", nargs=3, metavar=("KERNEL", "FIRST", "LAST"),
                   help="only launches between the FIRST-th and LAST-th launch of KERNEL")
    a.add_argument("--stats-csv", help="the run's --stats kernel summary, appended as a second table")
    c = sub.add_parser("stalls")
    c.add_argument("csv", nargs="+")
    c.add_argument("--command", required=True)
    c.add_argument("--out")
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        b.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--rhs", type=int, required=True)
    b.add_argument("--nodes", type=int, default=0)
    b.add_argument("--largest-grid", action="store_true",
                   help="per kernel the dispatches with its largest grid (the finest level), not its most frequent")
    b.add_argument("--command", required=True)
    b.add_argument("--out")
    b.add_argument("--json")
    g = sub.add_parser("gmres-traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        g.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    g.add_argument("--copy-bytes", type=float, required=True)
    g.add_argument("--steps", type=int, required=True, help="GMRES solves of the batch in the profiled run")
    g.add_argument("--report", required=True, help="the run's bench.py --gmres JSON line")
    g.add_argument("--command", required=True)
    g.add_argument("--out")
    g.add_argument("--json")
    args = ap.parse_args()
    if args.what == "stalls":
        text = _stalls_md(args.csv, args.command)
    elif args.what == "gmres-traffic":
        t = gmres_traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_bytes, args.steps)
        with open(args.report) as fh:
            rep = json.loads(fh.read().strip().splitlines()[-1])
        text = _gmres_traffic_md(t, args.command, rep["gram_schmidt"]["algorithmic_GB_per_step"])
        if args.json:
            with open(args.json, "w") as fh:
                json.dump({"kernel_source_hash": kernel_source_hash(), "fetch_factor": t["fetch_factor"],
                           "write_factor": t["write_factor"],
                           "workload": rep["config"]["workload"],
                           "bytes_per_step": sum(r["fetch_bytes_per_step"] + r["write_bytes_per_step"]
                                                 for r in t["kernels"].values()),
                           "kernels": t["kernels"]}, fh, indent=1)
    elif args.what == "stats":
        between = (args.between[0], int(args.between[1]), int(args.between[2])) if args.between else None
        text = _stats_md(args.trace, args.command, between)
        if args.stats_csv:
            text += _whole_run_md(args.stats_csv)
    else:
        t = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_bytes, args.rhs,
                    args.largest_grid)
        t["nodes"] = args.nodes
        text = _traffic_md(t, args.command, args.rhs, args.largest_grid)
        if args.json:
            per_class = {}
            for k in CLASS_SYMBOL:
                syms = [s for s in symbols_of(k) if s in t["kernels"]]
                if len(syms) == len(symbols_of(k)):  # mean over the class's symbols (equal launch counts)
                    per_class[k] = {"symbol": " + ".join(syms),
                                    "fetch_bytes_per_rhs": sum(t["kernels"][s]["fetch_bytes_per_rhs"]
                                                               for s in syms) / len(syms),
                                    "write_bytes_per_rhs": sum(t["kernels"][s]["write_bytes_per_rhs"]
                                                               for s in syms) / len(syms)}
            with open(args.json, "w") as fh:
                json.dump({"kernel_source_hash": kernel_source_hash(), "fetch_factor": t["fetch_factor"],
                           "write_factor": t["write_factor"], "rhs_per_dispatch": args.rhs,
                           "classes": per_class}, fh, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
