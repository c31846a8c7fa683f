"""Short text summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1411_0436_amd.prof_summary stats KERNEL_STATS_CSV OUT --command "..."
        per-kernel calls / average / total time of a --kernel-trace --stats run;

    python -m paper_1411_0436_amd.prof_summary sq OUT DIR [DIR ...] --match NAME
        --workload W --precision P --command "..."
        SQ instruction / wait counters per dispatch and per wave;

    python -m paper_1411_0436_amd.prof_summary compare OUT --match NAME --set LABEL=DIR[,DIR...]
        --set LABEL=DIR[,DIR...] [--per-launch-units U] --command "..."
        counters of the kernels whose name contains NAME under two or more
        settings (each from one or more counter runs), side by side with their
        ratio to the first, and per unit of work when U is given;

    python -m paper_1411_0436_amd.prof_summary traffic --fetch DIR --write DIR
        --copy-fetch DIR --copy-write DIR --match NAME --kind KIND
        --workload W --precision P OUT --command "..."
        HBM bytes per dispatch of the kernels whose name contains NAME, from a
        FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled by
        what the same counter reads for a plain device copy of known size
        (bytes moved / counter bytes).  The summary records the digest of the
        kernel sources so that a later change of the kernels retires it.

Only rocprofv3's CSV files are read; nothing here touches the GPU.
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["fft_common.h", "fft_bodies.h", "k_single.hip", "k_fourstep.hip", "k_rows.h",
                  "k_rows_f32.hip", "k_rows_mfma.hip", "pfbs_internal.h"]


def kernel_digest() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter, match):
    """Average over dispatches of the summed counter (over its instances) for
    kernels whose name contains `match`; also returns the dispatch count."""
    per = collections.defaultdict(float)
    names = {}
    for r in rows:
        if r["Counter_Name"] != counter or match not in r["Kernel_Name"]:
            continue
        per[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = r["Kernel_Name"]
    if not per:
        raise SystemExit("no %s rows for kernels matching %r" % (counter, match))
    return sum(per.values()) / len(per), len(per), sorted(set(names.values()))


def _copy_factor(rows, counter, copy_bytes):
    # the largest dispatch of the calibration run is the device copy
    best = 0.0
    for r in rows:
        if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
            best = max(best, float(r["Counter_Value"]))
    if best <= 0:
        raise SystemExit("no copy dispatch with %s in the calibration run" % counter)
    return copy_bytes / (best * 1024.0), best


def cmd_stats(a):
    with open(a.csv) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["# rocprofv3 --kernel-trace --stats summary", "# command: %s" % a.command,
           "# kernel sources sha1: %s" % kernel_digest(), "",
           "%-64s %7s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_ms", "share")]
    for r in rows[: a.top]:
        name = r["Name"].replace("void ", "").split("(")[0]
        out.append("%-64s %7s %12.2f %12.3f %6.1f%%" % (name[:64], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       100.0 * float(r["TotalDurationNs"]) / tot))
    _write(a.out, out)


def cmd_traffic(a):
    fr, wr = _counter_rows(a.fetch), _counter_rows(a.write)
    cf, cw = _counter_rows(a.copy_fetch), _counter_rows(a.copy_write)
    copy_bytes = a.copy_mib * 1048576.0
    kf, cf_raw = _copy_factor(cf, "FETCH_SIZE", copy_bytes)
    kw, cw_raw = _copy_factor(cw, "WRITE_SIZE", copy_bytes)
    f_kib, nf, names = _per_dispatch(fr, "FETCH_SIZE", a.match)
    w_kib, nw, _ = _per_dispatch(wr, "WRITE_SIZE", a.match)
    out = ["# HBM traffic per dispatch from rocprofv3 counters", "# commands: %s" % a.command,
           "# kernels: %s" % "; ".join(n.replace("void ", "").split("(")[0] for n in names),
           "# copy calibration: %.0f MiB device copy reads FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB"
           % (a.copy_mib, cf_raw, cw_raw),
           "kernel: %s" % a.kind, "workload: %s" % a.workload, "precision: %s" % a.precision,
           "kernel_sources_sha1: %s" % kernel_digest(),
           "dispatches: %d fetch, %d write" % (nf, nw),
           "fetch_kib_per_dispatch: %.1f" % f_kib, "write_kib_per_dispatch: %.1f" % w_kib,
           "fetch_scale: %.4f" % kf, "write_scale: %.4f" % kw,
           "fetch_bytes_per_launch: %.0f" % (f_kib * 1024.0 * kf),
           "write_bytes_per_launch: %.0f" % (w_kib * 1024.0 * kw)]
    _write(a.out, out)


def cmd_sq(a):
    """Per-dispatch SQ counters of the kernels whose name contains MATCH,
    from one or more counter runs, with per-wave instruction counts."""
    vals = collections.OrderedDict()
    names = set()
    for d in a.dirs:
        for r in _counter_rows(d):
            if a.match not in r["Kernel_Name"]:
                continue
            names.add(r["Kernel_Name"].replace("void ", "").split("(")[0])
            key = r["Counter_Name"]
            vals.setdefault(key, collections.defaultdict(float))[r.get("Dispatch_Id", r.get("Correlation_Id", "0"))] += \
                float(r["Counter_Value"])
    out = ["# rocprofv3 SQ counters per dispatch (summed over the counter's instances, averaged over dispatches)",
           "# commands: %s" % a.command, "# workload: %s, precision: %s" % (a.workload, a.precision),
           "# kernel sources sha1: %s" % kernel_digest(), "", "kernel: %s" % "; ".join(sorted(names))]
    avg = {k: sum(v.values()) / max(1, len(v)) for k, v in vals.items()}
    for k in sorted(avg):
        out.append("  %-24s %.4g" % (k, avg[k]))
    waves = avg.get("SQ_WAVES", 0.0)
    if waves:
        per = ", ".join("%s %.1f" % (lab, avg[c] / waves) for lab, c in
                        (("VALU", "SQ_INSTS_VALU"), ("LDS", "SQ_INSTS_LDS"), ("VMEM read", "SQ_INSTS_VMEM_RD"),
                         ("VMEM write", "SQ_INSTS_VMEM_WR"), ("SALU", "SQ_INSTS_SALU")) if c in avg)
        out.append("  per wave: %s instructions" % per)
    if "SQ_WAIT_INST_ANY" in avg and "SQ_WAVE_CYCLES" in avg and avg["SQ_WAVE_CYCLES"]:
        out.append("  waiting on counters: %.0f %% of wave cycles" % (100.0 * avg["SQ_WAIT_INST_ANY"] / avg["SQ_WAVE_CYCLES"]))
    if "SQ_LDS_BANK_CONFLICT" in avg and avg.get("SQ_ACTIVE_INST_LDS"):
        out.append("  LDS bank-conflict cycles / LDS active cycles: %.2f"
                   % (avg["SQ_LDS_BANK_CONFLICT"] / avg["SQ_ACTIVE_INST_LDS"]))
    _write(a.out, out)


def cmd_compare(a):
    """Per-dispatch counters of the kernels whose name contains MATCH under
    several labelled settings, with the ratio of each to the first setting."""
    sets = []
    for spec in a.set:
        label, dirs = spec.split("=", 1)
        vals, names = collections.OrderedDict(), set()
        for d in dirs.split(","):
            for r in _counter_rows(d):
                if a.match not in r["Kernel_Name"]:
                    continue
                names.add(r["Kernel_Name"].replace("void ", "").split("(")[0])
                vals.setdefault(r["Counter_Name"], collections.defaultdict(float))[r["Dispatch_Id"]] += \
                    float(r["Counter_Value"])
        sets.append((label, {k: sum(v.values()) / max(1, len(v)) for k, v in vals.items()}, sorted(names)))
    out = ["# rocprofv3 counters per dispatch under several settings (summed over the counter's instances,",
           "# averaged over dispatches)", "# commands: %s" % a.command, "# kernel sources sha1: %s" % kernel_digest(), ""]
    for label, _, names in sets:
        out.append("%s: %s" % (label, "; ".join(names)))
    counters = sorted(set().union(*[set(v) for _, v, _ in sets]))
    head = "%-30s" % "counter" + "".join("%16s" % lab for lab, _, _ in sets) + "".join(
        "%14s" % ("%s/%s" % (lab[:6], sets[0][0][:6])) for lab, _, _ in sets[1:])
    out += ["", head]
    for c in counters:
        v0 = sets[0][1].get(c)
        row = "%-30s" % c + "".join("%16.4g" % v.get(c, float("nan")) for _, v, _ in sets)
        row += "".join("%14.3f" % (v.get(c, float("nan")) / v0 if v0 else float("nan")) for _, v, _ in sets[1:])
        out.append(row)
    if a.per_launch_units:
        out += ["", "per unit of work (%g units per launch):" % a.per_launch_units]
        for c in counters:
            out.append("%-30s" % c + "".join("%16.4g" % (v.get(c, float("nan")) / a.per_launch_units)
                                              for _, v, _ in sets))
    _write(a.out, out)


def _write(path, lines):
    text = "\n".join(lines) + "\n"
    if path == "-":
        sys.stdout.write(text)
    else:
        with open(path, "w") as fh:
            fh.write(text)
        sys.stdout.write(text)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-mib", type=float, default=1024.0)
    t.add_argument("--match", required=True)
    t.add_argument("--kind", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--precision", default="fp32")
    t.add_argument("--command", required=True)
    t.add_argument("out")
    q = sub.add_parser("sq", help="SQ counters per dispatch")
    q.add_argument("out")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--match", required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--precision", default="fp32")
    q.add_argument("--command", required=True)
    c = sub.add_parser("compare", help="counters under several settings")
    c.add_argument("out")
    c.add_argument("--match", required=True)
    c.add_argument("--set", action="append", required=True, help="LABEL=DIR[,DIR...]")
    c.add_argument("--per-launch-units", type=float, default=0.0)
    c.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "sq": cmd_sq, "compare": cmd_compare}[a.cmd](a)


if __name__ == "__main__":
    main()
