"""Summaries of rocprofv3 output (kernel traces and PMC counters).

Usage (on the results directory a rocprofv3 run wrote with `-d DIR -o run`):

    python3 -m paper_1903_10977_amd.profiling kernels DIR [--match SUBSTR]
    python3 -m paper_1903_10977_amd.profiling traffic FETCH_DIR WRITE_DIR --kernel SUBSTR --grid G \
        --copy-mib M [--command TEXT]
    python3 -m paper_1903_10977_amd.profiling counters DIR [DIR ...] --kernel SUBSTR

`kernels` prints per-kernel launch counts and durations; `counters` prints the
mean of every counter collected in the given runs per dispatch of the matching
kernels (one row per kernel name and grid); `traffic` turns the
FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of one kernel into bytes
per launch, each scaled by what the same counter reads for a plain device
copy of M MiB (an elementwise kernel that reads M MiB and writes M MiB), and
records the hash of the stencil-kernel sources so that a reader can tell
whether the figure still describes the current kernel.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import os
import sqlite3
import sys

from . import PACKAGE_DIR

# sources that define the fused smoothing-step kernel
KERNEL_SOURCES = ("csrc/op_row.h", "csrc/level_kernels.hip", "csrc/imsmg_internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PACKAGE_DIR, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _db(path):
    dbs = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return sqlite3.connect(dbs[0])


def kernel_rows(path, match=None):
    """[(name, grid, launches, avg_us, total_ms)] sorted by total time."""
    c = _db(path)
    q = """select name, grid_x, count(*), avg(duration) / 1000.0, sum(duration) / 1e6
           from kernels group by name, grid_x order by sum(duration) desc"""
    rows = [r for r in c.execute(q) if match is None or match in r[0]]
    return rows


def pmc_rows(path, counter):
    """{(kernel name, grid size): (dispatches, mean counter value)}"""
    c = _db(path)
    q = """select kernel_name, grid_size, count(*), avg(value) from counters_collection
           where counter_name = ? group by kernel_name, grid_size"""
    return {(r[0], r[1]): (r[2], r[3]) for r in c.execute(q, (counter,))}


def counter_table(paths, kernel):
    """{(kernel name, grid size): {counter: (dispatches, mean value, mean
    duration in us)}} over every counter found in the runs under paths, for
    kernels containing kernel (a counter's value is summed over the hardware
    instances of one dispatch; durations are those of the counter runs)."""
    out = {}
    for path in paths:
        c = _db(path)
        q = """select kernel_name, grid_size, counter_name, count(*), avg(value), avg(duration) / 1000.0
               from counters_collection group by kernel_name, grid_size, counter_name"""
        for name, grid, counter, n, mean, dur in c.execute(q):
            if kernel in name:
                out.setdefault((name, grid), {})[counter] = (n, mean, dur)
    return out


def _pick(rows, kernel, grid):
    hits = [(k, v) for k, v in rows.items() if kernel in k[0] and (grid is None or k[1] == grid)]
    if not hits:
        raise KeyError(f"no dispatch of {kernel} (grid {grid})")
    n = sum(v[0] for _, v in hits)
    mean = sum(v[0] * v[1] for _, v in hits) / n
    return hits[0][0][0], n, mean


def copy_reference(rows, copy_bytes):
    """Counter value (KiB) of the calibration copy: the elementwise kernel whose
    grid moves copy_bytes (largest dispatch of the vectorized elementwise
    negation the bench runs for it; any elementwise kernel if none is named)."""
    hits = [(k, v) for k, v in rows.items() if "elementwise" in k[0] and "neg" in k[0].lower()]
    if not hits:
        hits = [(k, v) for k, v in rows.items() if "elementwise" in k[0]]
    if not hits:
        raise KeyError("no calibration copy kernel in the trace")
    k, v = max(hits, key=lambda kv: kv[0][1])
    return k[0], v[1]


def traffic_summary(fetch_dir, write_dir, kernel, grid, copy_mib, command=""):
    fetch = pmc_rows(fetch_dir, "FETCH_SIZE")
    write = pmc_rows(write_dir, "WRITE_SIZE")
    copy_bytes = copy_mib * (1 << 20)
    _, cf = copy_reference(fetch, copy_bytes)
    _, cw = copy_reference(write, copy_bytes)
    f_fetch = copy_bytes / (cf * 1024.0)
    f_write = copy_bytes / (cw * 1024.0)
    name, nf, kf = _pick(fetch, kernel, grid)
    _, nw, kw = _pick(write, kernel, grid)
    fetch_b = kf * 1024.0 * f_fetch
    write_b = kw * 1024.0 * f_write
    lines = [
        f"# HBM traffic of {name.split('(')[0]} (grid {grid}) from rocprofv3 PMC counters",
        "# commands (repository root = $R, run from /tmp with TMPDIR=/tmp):",
    ]
    lines += [f"#   {c}" for c in command.split(" ;; ") if c]
    lines += [
        f"kernel: {name}",
        f"kernel_source_sha256: {kernel_source_hash()}",
        f"copy_calibration_mib: {copy_mib}",
        f"copy_fetch_kib: {cf:.1f}   (expected {copy_bytes / 1024:.0f}; scale {f_fetch:.4f})",
        f"copy_write_kib: {cw:.1f}   (expected {copy_bytes / 1024:.0f}; scale {f_write:.4f})",
        f"dispatches: fetch {nf}, write {nw}",
        f"fetch_kib_per_dispatch: {kf:.1f}",
        f"write_kib_per_dispatch: {kw:.1f}",
        f"fetch_bytes_per_launch_scaled: {fetch_b:.0f}",
        f"write_bytes_per_launch_scaled: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    return "\n".join(lines) + "\n"


def read_traffic(path):
    """traffic_bytes_per_launch from a summary written by traffic_summary, or
    None when the file is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("--match", default=None)
    k.add_argument("--top", type=int, default=60)
    pc = sub.add_parser("counters")
    pc.add_argument("dirs", nargs="+")
    pc.add_argument("--kernel", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int, default=None)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        rows = kernel_rows(a.dir, a.match)
        print(f"{'kernel':72s} {'grid':>9s} {'launches':>8s} {'avg_us':>9s} {'total_ms':>9s}")
        for name, grid, cnt, avg, tot in rows[: a.top]:
            print(f"{name[:72]:72s} {grid:9d} {cnt:8d} {avg:9.2f} {tot:9.3f}")
    elif a.cmd == "counters":
        for (name, grid), cs in sorted(counter_table(a.dirs, a.kernel).items()):
            print(f"kernel: {name[:100]}  grid {grid}")
            for counter, (n, mean, dur) in sorted(cs.items()):
                print(f"  {counter:36s} dispatches {n:6d}  mean per dispatch {mean:.6g}  (duration {dur:.2f} us)")
    else:
        sys.stdout.write(traffic_summary(a.fetch_dir, a.write_dir, a.kernel, a.grid, a.copy_mib, a.command))


if __name__ == "__main__":
    main()
