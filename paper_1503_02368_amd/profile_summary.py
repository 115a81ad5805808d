"""Summarises rocprofv3 CSV output for one kernel into profiles/.

Reads a kernel-trace/stats directory and counter directories written by
``rocprofv3 -f csv``, scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by
what the same counters report for a plain copy of known size, and writes

* a Markdown summary (commands, kernel statistics, counters, traffic), and
* an entry in profiles/traffic.json: HBM bytes per launch of the kernel,
  tagged with the hash of the kernel source so that bench.py drops it once
  the kernel changes.

    python -m paper_1503_02368_amd.profile_summary --workload rmat20_triangles \\
        --kernel k_tri_staged --trace D --fetch D --write D --copy-fetch D \\
        --copy-write D [--counters D ...] --copy-mib 1024 --commands FILE --out profiles/X.md

With --stats-only it writes the kernel statistics table alone (no counters,
no traffic entry), for multi-kernel pipelines such as the GPU trie build:

    python -m paper_1503_02368_amd.profile_summary --stats-only --workload build \\
        --trace D --commands FILE --out profiles/X.md [--note TEXT]
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import hashlib
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SRC = os.path.join(HERE, "csrc", "eh_kernels.hip")
SETS_SRC = os.path.join(HERE, "csrc", "eh_sets.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_sha(src: str = KERNEL_SRC) -> str:
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_entry(name: str, src: str = KERNEL_SRC):
    """The committed counter summary of a workload's launch, or None when the
    kernel source (src) changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        d = json.load(f).get(name)
    if not d or d.get("kernel_sha") != kernel_sha(src):
        return None
    return d


def measured_traffic(name: str, src: str = KERNEL_SRC):
    """L2-to-fabric bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE)
    from the committed rocprofv3 counter runs, or None when the kernel source
    (src) changed since they were taken."""
    d = measured_entry(name, src)
    return d.get("bytes_per_launch") if d else None


def valu_issue(name: str, ms: float, src: str = KERNEL_SRC) -> dict:
    """VALU wave64 instructions per launch (SQ_INSTS_VALU summed over the
    launch's kernels, from the committed counter runs) and the share of the
    chip's VALU issue cycles they fill in ms per launch: a wave64 VALU
    instruction holds one of the 1024 SIMDs (256 CUs x 4) for 4 cycles, at
    2.4 GHz.  Both None when the counters are stale or absent."""
    d = measured_entry(name, src)
    valu = d.get("valu_insts_per_launch") if d else None
    frac = valu * 4 / (256 * 4 * 2.4e9 * ms / 1e3) if valu else None
    return {"valu_insts_per_launch": valu, "valu_issue_frac": frac}


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    rows = []
    for p in files:
        with open(p) as f:
            rows += list(csv.DictReader(f))
    return rows


def counters(d: str, name_part: str):
    """{counter: mean value per dispatch} over dispatches whose kernel name contains name_part."""
    acc = {}
    for r in _csv(d, "counter_collection.csv"):
        if name_part in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: (statistics.fmean(v), len(v)) for k, v in acc.items()}


def counters_by_kernel(d: str, name_part: str):
    """{kernel name: {counter: (mean per dispatch, dispatches)}} for the kernels
    whose name contains name_part (a launch of several kernels, one each)."""
    acc = {}
    for r in _csv(d, "counter_collection.csv"):
        if name_part in r["Kernel_Name"]:
            acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    return {k: {c: (statistics.fmean(v), len(v)) for c, v in m.items()} for k, m in acc.items()}


def kernel_stats(d: str):
    return _csv(d, "kernel_stats.csv")


N_XCD, N_CU, N_SIMD = 8, 256, 1024


def derived(c, avg_us):
    """Issue, residency and busy fractions from the SQ/GRBM counters, when present.

    GRBM_GUI_ACTIVE counts GPU-busy cycles summed over the 8 XCDs, so /8 over the
    kernel's average duration gives the clock.  SQ_ACTIVE_INST_VALU counts the
    VALU issue slots of wave64 instructions (it equals SQ_INSTS_VALU here), each
    of which holds its SIMD for 4 cycles; SQ_WAVE_CYCLES and SQ_WAIT_ANY are in
    the same 4-cycle units; SQ_BUSY_CU_CYCLES counts cycles summed over the CUs."""
    g = {k: v for k, (v, _) in c.items()}
    if "GRBM_GUI_ACTIVE" not in g:
        return []
    cyc = g["GRBM_GUI_ACTIVE"] / N_XCD
    out = ["", "## Derived (per dispatch)", "",
           f"* clock: {cyc / (avg_us * 1e-6) / 1e9:.2f} GHz ({cyc:,.0f} cycles per XCD over "
           f"{avg_us:.1f} us)"]
    if "SQ_ACTIVE_INST_VALU" in g:
        out.append(f"* VALU busy: {4 * g['SQ_ACTIVE_INST_VALU'] / (N_SIMD * cyc) * 100:.1f} % of "
                   f"{N_SIMD} SIMDs x cycles (4 cycles per wave64 VALU instruction)")
    if "SQ_BUSY_CU_CYCLES" in g:
        out.append(f"* CUs busy: {g['SQ_BUSY_CU_CYCLES'] / (N_CU * cyc) * 100:.1f} % of {N_CU} CUs x cycles")
    if "SQ_WAVE_CYCLES" in g:
        res = 4 * g["SQ_WAVE_CYCLES"] / cyc
        waves = g.get("SQ_WAVES", 0)
        out.append(f"* waves resident on average: {res:,.0f} (of {waves:,.0f} launched)")
        if "SQ_WAIT_ANY" in g:
            out.append(f"* share of wave time waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES): "
                       f"{g['SQ_WAIT_ANY'] / g['SQ_WAVE_CYCLES'] * 100:.1f} %")
    if "TCC_HIT_sum" in g and "TCC_MISS_sum" in g:
        out.append(f"* L2 hit rate: {g['TCC_HIT_sum'] / (g['TCC_HIT_sum'] + g['TCC_MISS_sum']) * 100:.1f} %")
    if "SQ_LDS_BANK_CONFLICT" in g and "SQ_ACTIVE_INST_LDS" in g:
        out.append(f"* LDS bank-conflict cycles per LDS issue cycle: "
                   f"{g['SQ_LDS_BANK_CONFLICT'] / g['SQ_ACTIVE_INST_LDS']:.2f}")
    return out


def stats_only(args):
    stats = kernel_stats(args.trace)
    with open(args.commands) as f:
        cmds = f.read().strip()
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    lines = [f"# Kernels of the {args.workload} workload", "",
             "Commands (from the repository root, one MI355X):", "", "```", cmds, "```", ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["## Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | average (us) | total (ms) | share of GPU time |",
              "|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        if "rocprim" in name:
            name = "rocPRIM " + ("radix sort" if "radix" in name else "scan" if "scan" in name
                                 else "select/unique" if ("select" in name or "unique" in name)
                                 else "kernel") + " (" + name[name.find("<") + 1:][:40] + "...)"
        lines.append(f"| {name[:100]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} % |")
    lines += ["", f"Total GPU kernel time: {total / 1e6:.2f} ms.", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print(f"wrote {args.out}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats-only", action="store_true")
    ap.add_argument("--note", default="")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernel", help="substring of the kernel's symbol name")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--counters", action="append", default=[])
    ap.add_argument("--commands", required=True, help="text file with the commands that made the data")
    ap.add_argument("--algorithmic-bytes", type=float, default=0.0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--source", default="eh_kernels.hip",
                    help="file under csrc/ that holds the kernel (its hash tags the entry)")
    args = ap.parse_args()
    if args.stats_only:
        return stats_only(args)
    for need in ("kernel", "fetch", "write", "copy_fetch", "copy_write"):
        if getattr(args, need) is None:
            ap.error(f"--{need.replace('_', '-')} is required without --stats-only")

    stats = kernel_stats(args.trace)
    mine = [r for r in stats if args.kernel in r["Name"]]
    if not mine:
        raise SystemExit(f"kernel {args.kernel} not in {args.trace}")
    # a launch may be several kernels (one dispatch each): traffic is summed
    # over them, durations are each kernel's own (they may overlap)
    avg_us = sum(float(k["AverageNs"]) for k in mine) / 1e3
    known_kib = args.copy_mib * 1024.0
    cf = counters(args.copy_fetch, "copyBuffer")["FETCH_SIZE"][0]
    cw = counters(args.copy_write, "copyBuffer")["WRITE_SIZE"][0]
    f_fac, w_fac = known_kib / cf, known_kib / cw
    fb = counters_by_kernel(args.fetch, args.kernel)
    wb = counters_by_kernel(args.write, args.kernel)
    fk = sum(c["FETCH_SIZE"][0] for c in fb.values())
    wk = sum(c["WRITE_SIZE"][0] for c in wb.values())
    fn = min(c["FETCH_SIZE"][1] for c in fb.values())
    wn = min(c["WRITE_SIZE"][1] for c in wb.values())
    traffic = (fk * f_fac + wk * w_fac) * 1024.0
    per_kernel = {}
    for d in args.counters:
        for kname, m in counters_by_kernel(d, args.kernel).items():
            per_kernel.setdefault(kname, {}).update(m)
    extra = next(iter(per_kernel.values())) if len(per_kernel) == 1 else {}

    with open(args.commands) as f:
        cmds = f.read().strip()
    lines = [f"# {args.kernel} on {args.workload}", "",
             "Commands (from the repository root, one MI355X):", "", "```", cmds, "```", "",
             "## Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.3f} | "
                     f"{float(r['MinNs'])/1e3:.3f} | {float(r['MaxNs'])/1e3:.3f} | {float(r['Percentage']):.2f} % |")
    several = len(mine) > 1
    lines += ["", "## Memory traffic (per launch: " +
              (f"the {len(mine)} kernels matching `{args.kernel}`, one dispatch each, summed)"
               if several else "one dispatch of the kernel)"), "",
              f"* FETCH_SIZE: {fk:,.0f} KiB (mean of {fn} dispatches) x {f_fac:.3f} = "
              f"{fk * f_fac * 1024 / 1e9:.3f} GB",
              f"* WRITE_SIZE: {wk:,.0f} KiB (mean of {wn} dispatches) x {w_fac:.3f} = "
              f"{wk * w_fac * 1024 / 1e6:.3f} MB",
              f"* Calibration: a copy of {args.copy_mib} MiB reads {cf:,.0f} KiB by FETCH_SIZE and "
              f"writes {cw:,.0f} KiB by WRITE_SIZE per dispatch (factors {f_fac:.3f}, {w_fac:.3f}).",
              f"* L2-to-fabric traffic per launch (reads the 256 MB last-level cache serves are "
              f"included): {traffic / 1e9:.3f} GB; over the " +
              ("summed average durations" if several else "average duration") +
              f" {avg_us:.1f} us that is {traffic / (avg_us * 1e-6) / 1e9:.0f} GB/s "
              f"({traffic / (avg_us * 1e-6) / 8e12 * 100:.1f} % of 8 TB/s)."]
    if args.algorithmic_bytes:
        lines.append(f"* Algorithmic bytes per launch: {args.algorithmic_bytes / 1e9:.3f} GB "
                     f"({args.algorithmic_bytes / (avg_us * 1e-6) / 1e9:.0f} GB/s).")
    if extra:
        lines += ["", "## Other counters (mean per dispatch)", "", "| counter | value | dispatches |",
                  "|---|---|---|"]
        for name in sorted(extra):
            v, n = extra[name]
            lines.append(f"| {name} | {v:,.0f} | {n} |")
    lines += derived(extra, avg_us)
    if several:
        # the kernels of one launch run side by side in the trace; a counter
        # run serialises the dispatches, so each kernel's derived figures use
        # its own duration there
        by_name = {}
        if args.counters:
            for r in _csv(args.counters[0], "kernel_trace.csv"):
                if args.kernel in r["Kernel_Name"]:
                    by_name.setdefault(r["Kernel_Name"], []).append(
                        (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        by_name = {k: statistics.median(v) for k, v in by_name.items()}
        lines += ["", "The kernels run side by side on forked streams, so the trace's durations "
                  "overlap; the counter runs serialise the dispatches, and each kernel's section "
                  "gives its duration there."]
        for kname in sorted(per_kernel, key=lambda k: -by_name.get(k, 0.0)):
            m = per_kernel[kname]
            us = by_name.get(kname, 0.0)
            lines += ["", f"## {kname[:100]} ({us:.1f} us alone)", "",
                      "| counter | value | dispatches |", "|---|---|---|"]
            for name in sorted(m):
                v, n = m[name]
                lines.append(f"| {name} | {v:,.0f} | {n} |")
            lines += derived(m, us)[1:] if us else []
    src = os.path.join(ROOT, "paper_1503_02368_amd", "csrc", args.source)
    sha = kernel_sha(src)
    lines += ["", f"Kernel source hash ({args.source}, sha256 prefix): {sha}", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))

    tj = {}
    if os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tj = json.load(f)
    valu = sum(m["SQ_INSTS_VALU"][0] for m in per_kernel.values() if "SQ_INSTS_VALU" in m)
    tj[args.workload] = {"kernel": args.kernel, "kernel_sha": sha, "source": args.source,
                         "bytes_per_launch": traffic, "avg_us": avg_us,
                         "valu_insts_per_launch": valu or None,
                         "fetch_kib": fk, "write_kib": wk, "fetch_factor": f_fac,
                         "write_factor": w_fac, "summary": os.path.relpath(args.out, ROOT)}
    with open(args.traffic, "w") as f:
        json.dump(tj, f, indent=1, sort_keys=True)
    print(f"{args.workload}: {avg_us:.1f} us, traffic {traffic / 1e9:.3f} GB per launch")


if __name__ == "__main__":
    main()
