"""Summaries of rocprofv3 output (kernel statistics and HBM traffic counters).

Usage (after the rocprofv3 runs, with their CSV output directories):

  python -m paper_2407_07463_amd.profiling stats DIR --out FILE.md --command "..."
      per-kernel calls / total / average duration from a `--kernel-trace
      --stats -f csv` run.

  python -m paper_2407_07463_amd.profiling traffic --fetch DIR1 --write DIR2 \\
      --kernel REGEX --copy REGEX --copy-bytes B --out FILE.txt --command "..."
      HBM bytes per dispatch of the kernels matching REGEX from a FETCH_SIZE
      run and a WRITE_SIZE run (KiB per dispatch), each scaled by what the
      same counter reads for a plain copy kernel that reads and writes B bytes.
      The summary records the SHA-256 of the advection sources, so that a
      reader can tell whether the kernel changed since.

  python -m paper_2407_07463_amd.profiling counters DIR [DIR...] --kernel REGEX \
      --counters NAME... --out FILE.txt --command "..." [--command "..."] [--sources ...]
      per-kernel mean of each counter per dispatch from a `--pmc` run
      (derived metrics such as MfmaUtil as rocprofv3 reduces them).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
ADVECT_SOURCES = ["csrc/advect_kernels.hpp", "csrc/plic.hpp", "csrc/advect.hip",
                  "csrc/common.hpp"]


def advect_source_sha(sources=None) -> str:
    """SHA-256 over the given sources (paths relative to the package;
    default: the advection kernels)."""
    h = hashlib.sha256()
    for rel in sources or ADVECT_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _find(directory: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return hits[-1]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def short_name(name: str) -> str:
    """Kernel name without namespaces and parameter list."""
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"^void ", "", name)
    depth, out = 0, []
    for ch in name:  # drop the parameter list, keep template arguments
        if ch == "(" and depth == 0 and out:
            break
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        out.append(ch)
    return "".join(out).strip()


def kernel_stats(directory: str):
    """[(name, calls, total_ns, avg_ns)] sorted by total time."""
    rows = _rows(_find(directory, "kernel_stats.csv"))
    out = []
    for r in rows:
        out.append((short_name(_col(r, "Name", "KernelName")), int(float(_col(r, "Calls"))),
                    float(_col(r, "TotalDurationNs")), float(_col(r, "AverageNs"))))
    out.sort(key=lambda t: -t[2])
    return out


def counter_means(directory: str, counter: str):
    """{kernel name: (dispatches, mean counter value per dispatch)}."""
    rows = _rows(_find(directory, "counter_collection.csv"))
    acc = defaultdict(lambda: [0, 0.0])
    for r in rows:
        if _col(r, "Counter_Name") != counter:
            continue
        k = short_name(_col(r, "Kernel_Name"))
        acc[k][0] += 1
        acc[k][1] += float(_col(r, "Counter_Value"))
    return {k: (n, v / n) for k, (n, v) in acc.items()}


def write_stats(directory, out, command, title):
    st = kernel_stats(directory)
    tot = sum(t for _, _, t, _ in st) or 1.0
    lines = [f"# {title}", "", "Command:", "", f"    {command}", "",
             "| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for name, calls, t, avg in st:
        lines.append(f"| `{name}` | {calls} | {t / 1e6:.3f} | {avg / 1e3:.2f} | {100 * t / tot:.1f}% |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return st


def write_traffic(fetch_dir, write_dir, kernel_re, copy_re, copy_bytes, out, command_fetch, command_write,
                  sources=None):
    fe = counter_means(fetch_dir, "FETCH_SIZE")
    wr = counter_means(write_dir, "WRITE_SIZE")
    kre, cre = re.compile(kernel_re), re.compile(copy_re)
    copies_f = [v for k, v in fe.items() if cre.search(k)]
    copies_w = [v for k, v in wr.items() if cre.search(k)]
    if not copies_f or not copies_w:
        raise RuntimeError("copy kernel not found in the counter output")
    if len(copies_f) > 1 or len(copies_w) > 1:
        names = sorted(k for k in set(fe) | set(wr) if cre.search(k))
        raise RuntimeError(f"copy pattern {copy_re!r} matches several kernels: {names}")
    kib = copy_bytes / 1024.0
    f_factor = copies_f[0][1] / kib  # counter KiB per true KiB read
    w_factor = copies_w[0][1] / kib
    lines = ["# HBM traffic per dispatch from rocprofv3 counters", "",
             f"FETCH_SIZE run: {command_fetch}", f"WRITE_SIZE run: {command_write}", "",
             f"copy kernel: the dispatches whose name matches '{copy_re}'; it reads and writes "
             f"{copy_bytes} B per dispatch",
             f"copy_fetch_factor = {f_factor:.6f}   (FETCH_SIZE KiB / true KiB read)",
             f"copy_write_factor = {w_factor:.6f}   (WRITE_SIZE KiB / true KiB written)",
             (f"advect_source_sha256 = {advect_source_sha()}" if not sources else
              f"source_sha256 = {advect_source_sha(sources)}   ({', '.join(sources)})"), ""]
    for k in sorted(set(fe) | set(wr)):
        if not kre.search(k):
            continue
        nf, f = fe.get(k, (0, float("nan")))
        nw, w = wr.get(k, (0, float("nan")))
        fb = f / f_factor * 1024.0
        wb = w / w_factor * 1024.0
        lines.append(f"kernel = {k} | dispatches {nf}/{nw} | FETCH_SIZE {f:.1f} KiB | WRITE_SIZE {w:.1f} KiB | "
                     f"read_bytes = {fb:.0f} | write_bytes = {wb:.0f} | traffic_bytes = {fb + wb:.0f}")
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def write_counters(directories, kernel_re, counters, out, commands, title, sources=None):
    """Per-kernel mean of each counter per dispatch (derived metrics included, as rocprofv3
    reduces them), one line per kernel matching kernel_re. Counters may come from several
    runs (one directory and command each): a counter is read from the first run that has it."""
    if isinstance(directories, str):
        directories = [directories]
    if isinstance(commands, str):
        commands = [commands]
    kre = re.compile(kernel_re)
    means = {}
    for cn in counters:
        for d in directories:
            m = counter_means(d, cn)
            if m:
                means[cn] = m
                break
        else:
            means[cn] = {}
    names = sorted({k for m in means.values() for k in m if kre.search(k)})
    lines = [f"# {title}", ""] + [f"Command: {c}" for c in commands] + [
        "", f"source_sha256 = {advect_source_sha(sources)}   ({', '.join(sources or ADVECT_SOURCES)})", ""]
    for k in names:
        parts = [f"kernel = {k}"]
        nd = max(means[cn].get(k, (0, 0.0))[0] for cn in counters)
        parts.append(f"dispatches = {nd}")
        for cn in counters:
            n, v = means[cn].get(k, (0, float("nan")))
            parts.append(f"{cn} = {v:.6g}")
        lines.append(" | ".join(parts))
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")


def read_traffic(path):
    """{kernel: traffic bytes per dispatch} and the recorded source hash, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    sha, out = None, {}
    with open(path) as f:
        for line in f:
            if line.startswith("advect_source_sha256 = "):
                sha = line.split("=", 1)[1].strip()
            m = re.match(r"kernel = (.*?) \|.*traffic_bytes = ([0-9.]+)", line)
            if m:
                out[m.group(1)] = float(m.group(2))
    return out, sha


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--out", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    b.add_argument("--sources", nargs="*", default=None,
                   help="sources of the counted kernel (relative to the package) whose hash the summary records; "
                        "default: the advection kernels")
    c = sub.add_parser("counters")
    c.add_argument("dir", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--counters", nargs="+", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True, action="append", help="the command of each run, in order")
    c.add_argument("--title", default="rocprofv3 counters per dispatch")
    c.add_argument("--sources", nargs="*", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "counters":
        write_counters(args.dir, args.kernel, args.counters, args.out, args.command, args.title, args.sources)
        print(open(args.out).read())
        return
    if args.cmd == "stats":
        for name, calls, t, avg in write_stats(args.dir, args.out, args.command, args.title)[:12]:
            print(f"{name:60s} {calls:6d} {t / 1e6:10.3f} ms {avg / 1e3:10.2f} us")
    else:
        write_traffic(args.fetch, args.write, args.kernel, args.copy, args.copy_bytes, args.out,
                      args.command_fetch, args.command_write, args.sources)
        print(open(args.out).read())


if __name__ == "__main__":
    main()
