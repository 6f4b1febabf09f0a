"""Summaries of rocprofv3 output for the benchmark (no GPU work here).

Kernel statistics (``--kernel-trace --stats``) become a short markdown table;
two counter passes (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, each a
run of its own) become HBM bytes per launch of one kernel, scaled by what the
same counters read for a plain device-to-device copy of known size run in
the same process (``bench.py --copy-probe MIB``).  The result is written as a
``traffic:`` line that ``bench.py`` reads back; it carries the SHA-256 of the
kernel's source file, so a figure measured on an older kernel is not reused.

    python -m paper_2501_01676_amd.profiling stats STATS_CSV --steps N --out FILE --cmd "..."
    python -m paper_2501_01676_amd.profiling traffic FETCH_CSV WRITE_CSV --kernel NAME
        --source FILE --workload NAME --probe-bytes B --out FILE --cmd "..."
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short_name(name):
    """Kernel name without namespaces and argument list."""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("(anonymous namespace)::", "").replace("abddc::", "")
    return n.split("(")[0]


def source_sha256(path):
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stats_table(stats_csv, steps, top=15):
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["| kernel | calls/step | ms/step | avg us | share |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{short_name(r['Name'])}` | {int(r['Calls']) / steps:.1f} | "
                     f"{float(r['TotalDurationNs']) / steps / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f} % |")
    lines.append(f"| all kernels | | {tot / steps / 1e6:.3f} | | 100 % |")
    return "\n".join(lines)


def _per_dispatch(counter_csv):
    """(kernel, counter value) per dispatch, in dispatch order."""
    rows = list(csv.DictReader(open(counter_csv)))
    if rows and "Dispatch_Id" in rows[0]:
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(short_name(r["Kernel_Name"]), float(r["Counter_Value"])) for r in rows]


def calibration(values, probe_bytes):
    """bytes per counter unit from the three probe copies: the last three
    copyBuffer dispatches (bench.py --copy-probe runs them after every
    solve), which must agree with each other."""
    probe = [v for k, v in values if "copyBuffer" in k][-3:]
    if len(probe) < 3:
        raise SystemExit("copy probe dispatches not found")
    if max(probe) > 1.05 * min(probe):
        raise SystemExit(f"the last three copies disagree ({probe}): not the probe")
    return probe_bytes / statistics.mean(probe)


def traffic(fetch_csv, write_csv, kernel, probe_bytes, names=None):
    """Mean counter bytes per launch of `kernel`, or of every kernel in
    `names` taken together (template instances the benchmark tracks as one
    class)."""
    match = set(names) if names else {kernel}
    f = _per_dispatch(fetch_csv)
    w = _per_dispatch(write_csv)
    cf, cw = calibration(f, probe_bytes), calibration(w, probe_bytes)
    kf = [v for k, v in f if k in match]
    kw = [v for k, v in w if k in match]
    if not kf or not kw:
        raise SystemExit(f"kernel {kernel} not in counter output")
    fetch = statistics.mean(kf) * cf
    write = statistics.mean(kw) * cw
    return {"fetch_bytes": fetch, "write_bytes": write, "bytes": fetch + write, "launches": len(kf),
            "fetch_scale": cf, "write_scale": cw}


def read_traffic(kernel, workload, search_dir=None):
    """HBM bytes per launch recorded for (kernel, workload) under profiles/,
    or None when absent or measured on a different kernel source."""
    d = search_dir or os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    for fn in sorted(os.listdir(d)):
        if not fn.endswith(".md"):
            continue
        for line in open(os.path.join(d, fn)):
            if not line.startswith("traffic:"):
                continue
            kv = dict(x.split("=", 1) for x in line[len("traffic:"):].split())
            if kv.get("kernel") != kernel or kv.get("workload") != workload:
                continue
            try:
                if source_sha256(kv["source"]) != kv["sha256"]:
                    return None
            except OSError:
                return None
            return float(kv["bytes_per_launch"])
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("stats_csv")
    a.add_argument("--steps", type=float, required=True, help="solves in the profiled run (warmup included)")
    a.add_argument("--out", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="Kernel time")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", required=True)
    b.add_argument("--source", required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--probe-bytes", type=float, required=True)
    b.add_argument("--algorithmic-bytes", type=float, default=None)
    b.add_argument("--names", nargs="*", default=None,
                   help="kernel instances counted together under --kernel (default: --kernel alone)")
    b.add_argument("--out", required=True)
    b.add_argument("--cmd", required=True)
    args = ap.parse_args()
    if args.cmd_name == "stats":
        text = (f"# {args.title}\n\nCommand:\n\n```\n{args.cmd}\n```\n\n"
                f"Per solve: the totals divided by {args.steps:g}, every solve the run made (bench.py: the "
                f"warmup solves, the timed ones and the two untimed solves that time the other kernel "
                f"classes):\n\n"
                f"{stats_table(args.stats_csv, args.steps)}\n")
    else:
        t = traffic(args.fetch_csv, args.write_csv, args.kernel, args.probe_bytes, args.names)
        sha = source_sha256(args.source)
        extra = ""
        if args.algorithmic_bytes:
            extra = f"\nAlgorithmic bytes per launch (the benchmark's model): {args.algorithmic_bytes:.4g}; " \
                    f"measured / algorithmic = {t['bytes'] / args.algorithmic_bytes:.2f}\n"
        text = (f"# HBM traffic of `{args.kernel}` ({args.workload})\n\nCommands (one counter per run):\n\n"
                f"```\n{args.cmd}\n```\n\n"
                f"Copy-probe scale (bytes per counter unit): FETCH_SIZE {t['fetch_scale']:.4g}, "
                f"WRITE_SIZE {t['write_scale']:.4g}.\n\n"
                + (f"Instances counted together: {', '.join(args.names)}.\n\n" if args.names else "")
                + f"Per launch, mean over {t['launches']} launches: fetched {t['fetch_bytes'] / 1e6:.2f} MB, "
                f"written {t['write_bytes'] / 1e6:.2f} MB, total {t['bytes'] / 1e6:.2f} MB.\n{extra}\n"
                f"traffic: kernel={args.kernel} workload={args.workload} bytes_per_launch={t['bytes']:.6g} "
                f"source={args.source} sha256={sha}\n")
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
