"""Summaries of rocprofv3 output for the committed profile notes.

  python -m paper_2206_14662_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
  python -m paper_2206_14662_amd.profiling traffic <kernel-regex> <fetch_dir> <write_dir> \
      <copy_fetch_dir> <copy_write_dir> <out.txt> "<command>"

`stats` condenses a `--kernel-trace --stats` CSV into a table (one line per
kernel, template variants kept apart, plus the launch-weighted average of each
kernel family).  `traffic` turns two `--pmc` runs (FETCH_SIZE, WRITE_SIZE, KiB
per dispatch) into HBM bytes per launch of the named kernel, scaling each
counter by what it reads for a plain device copy of known size.
"""
import csv
import glob
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("fp32.hip", "fp32.h", "pic_internal.h")


def kernel_source_hash():
    """Hash of the sources the batched FP32 particle kernel is built from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    m = re.search(r"([A-Za-z_][A-Za-z0-9_]*(?:<[0-9, ]+>)?)\(", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:48]


def family(name):
    return re.sub(r"<[0-9, ]+>$", "", name)


def stats(csv_path, out_path, command):
    rows = list(csv.DictReader(open(csv_path)))
    per = []
    fam = {}
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    for r in rows:
        n = short_name(r["Name"])
        calls = int(r["Calls"])
        t = float(r["TotalDurationNs"])
        per.append((n, calls, t, float(r["MinNs"]), float(r["MaxNs"])))
        f = fam.setdefault(family(n), [0, 0.0])
        f[0] += calls
        f[1] += t
    per.sort(key=lambda x: -x[2])
    lines = [f"command: {command}", "", "| kernel | calls | avg us | min us | max us | % time |",
             "|---|---|---|---|---|---|"]
    for n, c, t, lo, hi in per:
        lines.append(f"| {n} | {c} | {t / c / 1e3:.2f} | {lo / 1e3:.2f} | {hi / 1e3:.2f} | {100 * t / tot:.2f} |")
    lines += ["", "launch-weighted averages of kernel families:", ""]
    for n, (c, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        if c > 1 or "<" in n:
            lines.append(f"- {n}: {c} launches, average {t / c / 1e3:.2f} us")
    open(out_path, "w").write("\n".join(lines) + "\n")


def _counter(dirname, regex, counter):
    files = glob.glob(os.path.join(dirname, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {dirname}")
    vals = []
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] == counter and re.search(regex, r["Kernel_Name"]):
                vals.append(float(r["Counter_Value"]))
    return vals


def traffic(regex, fetch_dir, write_dir, cfetch_dir, cwrite_dir, out_path, command):
    copy_bytes = 2 << 30
    f = _counter(fetch_dir, regex, "FETCH_SIZE")
    w = _counter(write_dir, regex, "WRITE_SIZE")
    cf = _counter(cfetch_dir, "copyBuffer", "FETCH_SIZE")
    cw = _counter(cwrite_dir, "copyBuffer", "WRITE_SIZE")
    if not (f and w and cf and cw):
        raise SystemExit("missing counter rows")
    kf = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    kw = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    fb = sum(f) / len(f) * 1024.0 * kf
    wb = sum(w) / len(w) * 1024.0 * kw
    lines = [
        f"command: {command}",
        f"kernel regex: {regex}",
        f"dispatches: fetch {len(f)}, write {len(w)}",
        f"FETCH_SIZE per dispatch: {sum(f) / len(f):.1f} KiB (copy calibration x{kf:.3f})",
        f"WRITE_SIZE per dispatch: {sum(w) / len(w):.1f} KiB (copy calibration x{kw:.3f})",
        f"read_bytes_per_launch: {fb:.6g}",
        f"write_bytes_per_launch: {wb:.6g}",
        f"bytes_per_launch: {fb + wb:.6g}",
        f"source_hash: {kernel_source_hash()}",
    ]
    open(out_path, "w").write("\n".join(lines) + "\n")


def read_traffic(path):
    """bytes_per_launch from a traffic summary if it was taken on the current
    kernel sources, else None."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    else:
        raise SystemExit(__doc__)
