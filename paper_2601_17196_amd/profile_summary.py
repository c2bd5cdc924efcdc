"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

  python -m paper_2601_17196_amd.profile_summary stats KERNEL_STATS_CSV --title T --command C --out FILE.md
        [--trace KERNEL_TRACE_CSV --kernel PATTERN --min-frac F]
  python -m paper_2601_17196_amd.profile_summary pmc FETCH_CSV WRITE_CSV --out FILE.json --command C ...
        [--min-frac F]

With --trace, the stats summary also lists the durations of the named
kernel's dispatches that take at least F of the longest one (a persistent
kernel's full launches, apart from its short autotuning launches), and their
average.  In pmc mode, --min-frac keeps only the dispatches whose fetched
bytes are at least F of the largest.

The pmc mode reads two counter-collection runs (FETCH_SIZE, then WRITE_SIZE,
KiB per dispatch), averages them per kernel, and scales them by the factor
that makes a plain device copy of known size read and write exactly its
bytes.  It records a hash of the kernel sources, so that a consumer can tell
whether the counters still describe the current kernels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/pot_kernels.hip", "csrc/pot_device.h", "csrc/pot_internal.h"]
BATCHED_SOURCES = ["csrc/pot_batched.hip", "csrc/pot_device.h", "csrc/pot_internal.h"]
SHARED_SOURCES = ["csrc/pot_shared.hip", "csrc/pot_device.h", "csrc/pot_internal.h"]


def kernel_source_hash(files=None) -> str:
    """Hash of the sources a kernel is built from (default: the
    single-instance kernels) and of the compiler flags of each HIP source."""
    from . import build as hipbuild
    h = hashlib.sha256()
    for f in (files or KERNEL_SOURCES):
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
        name = os.path.basename(f)
        if name in hipbuild.SOURCES:
            h.update(" ".join(hipbuild.HIPCC_FLAGS + hipbuild.SOURCE_FLAGS.get(name, [])).encode())
    return h.hexdigest()[:16]


def stats_table(path, title, command):
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (repository root, one MI355X):", "", "    export TMPDIR=/tmp"]
    out += ["    " + line for line in command.split("\n")]
    out += ["", "| kernel | calls | total ms | average us | min us | max us |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{r['Name'][:72]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    return "\n".join(out) + "\n"


def trace_section(path, pattern, min_frac, note="the others are short autotuning launches"):
    """Durations (us) of the dispatches of the kernel matching pattern that
    take at least min_frac of its longest one."""
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            for r in csv.DictReader(open(path)) if pattern in r["Kernel_Name"]]
    if not durs:
        return ""
    top = max(durs)
    keep = [d for d in durs if d >= min_frac * top]
    out = ["", f"Dispatches of `{pattern}` taking at least {min_frac:g} of the longest ({len(keep)} of {len(durs)};"
                f" {note}):", ""]
    shown = ", ".join(f"{d / 1e3:.2f} ms" if d >= 1e4 else f"{d:.2f} us" for d in keep[:40])
    out.append("    " + shown + (f", ... ({len(keep) - 40} more)" if len(keep) > 40 else ""))
    avg = sum(keep) / len(keep)
    out += ["", f"Average of these: {avg / 1e3:.3f} ms" if avg >= 1e4 else f"Average of these: {avg:.2f} us"]
    return "\n".join(out) + "\n"


def per_kernel(path, counter):
    """{kernel name: [value per dispatch]} for one counter (values summed over
    the rows of a dispatch)."""
    acc = collections.defaultdict(float)
    name = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        key = r["Dispatch_Id"]
        acc[key] += float(r["Counter_Value"])
        name[key] = r["Kernel_Name"]
    out = collections.defaultdict(list)
    for key in sorted(acc, key=int):          # in dispatch order
        out[name[key]].append(acc[key])
    return out


def pmc_summary(fetch_csv, write_csv, copy_bytes, copy_pattern, kernel_pattern, command, sources=None,
                min_frac=0.0, copy_count=3):
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    if min_frac > 0.0:
        # full launches only: the write pass's dispatches follow the fetch pass's selection by rank of size
        for d in (f, w):
            for k in d:
                if kernel_pattern in k:
                    top = max(d[k])
                    d[k] = [v for v in d[k] if v >= min_frac * top]

    def pick(d, pat):
        vals = [v for k, lst in d.items() if pat in k for v in lst]
        return sum(vals) / len(vals) if vals else None, len(vals)
    # the probe's copies of the known size are the run's first copy_count copy
    # dispatches (uploads of the workload, which also copy, come after them)
    def first_copies(d):
        vals = [v for k, lst in d.items() if copy_pattern in k for v in lst][:copy_count]
        return sum(vals) / len(vals) if vals else None
    cf = first_copies(f)
    cw = first_copies(w)
    kf, nf = pick(f, kernel_pattern)
    kw, nw = pick(w, kernel_pattern)
    sf = copy_bytes / (cf * 1024.0) if cf else None
    sw = copy_bytes / (cw * 1024.0) if cw else None
    out = {"kernel": kernel_pattern, "dispatches": [nf, nw],
           "fetch_kib_raw": kf, "write_kib_raw": kw,
           "copy_bytes": copy_bytes, "copy_dispatches": copy_count, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
           "scale_fetch": sf, "scale_write": sw,
           "fetch_bytes": kf * 1024.0 * sf if kf and sf else None,
           "write_bytes": kw * 1024.0 * sw if kw and sw else None,
           "kernel_sources": sources or KERNEL_SOURCES,
           "kernel_source_hash": kernel_source_hash(sources), "command": command}
    if min_frac > 0.0:
        out["min_frac"] = min_frac
    if out["fetch_bytes"] is not None and out["write_bytes"] is not None:
        out["traffic_bytes"] = out["fetch_bytes"] + out["write_bytes"]
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--trace", help="kernel-trace CSV of the same run")
    s.add_argument("--kernel", help="kernel name pattern for the per-dispatch list")
    s.add_argument("--min-frac", type=float, default=0.5)
    s.add_argument("--note", default="the others are short autotuning launches",
                   help="what the shorter dispatches are")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--copy-bytes", type=float, required=True)
    p.add_argument("--copy-pattern", default="copy")
    p.add_argument("--kernel-pattern", required=True)
    p.add_argument("--command", required=True)
    p.add_argument("--out", required=True)
    p.add_argument("--batched", action="store_true", help="the kernel is the batched one (its own sources)")
    p.add_argument("--shared", action="store_true", help="the kernel is the shared-cost product (its own sources)")
    p.add_argument("--min-frac", type=float, default=0.0,
                   help="keep the kernel's dispatches of at least this fraction of its largest")
    a = ap.parse_args()
    if a.mode == "stats":
        text = stats_table(a.csv, a.title, a.command)
        if a.trace and a.kernel:
            text += trace_section(a.trace, a.kernel, a.min_frac, a.note)
        open(a.out, "w").write(text)
    else:
        res = pmc_summary(a.fetch_csv, a.write_csv, a.copy_bytes, a.copy_pattern, a.kernel_pattern, a.command,
                          BATCHED_SOURCES if a.batched else SHARED_SOURCES if a.shared else None, a.min_frac)
        json.dump(res, open(a.out, "w"), indent=1)
    print(open(a.out).read())


if __name__ == "__main__":
    main()
