"""Summaries of rocprofv3 runs of bench.py for the ``profiles/`` folder.

    python -m paper_1804_10120_amd.profsum --trace DIR [--fetch DIR --write DIR]
        --cmd "the profiled command" --out profiles/

Reads the CSV output of ``rocprofv3 --kernel-trace --stats --output-format
csv`` (kernel_stats) and of two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
runs (counter_collection).  Writes ``kernel_stats_<workload>.md`` with the
per-kernel durations, and for each of the fused kernels a
``pmc_<kernel>.md`` with its HBM traffic per launch.  Counter readings are
scaled by what the same counter reads for the library's streaming copy of
known size (so the scale factor absorbs how many memory channels a counter
sees); the file records a hash of the kernel sources, and the benchmark
reports the traffic only while the sources still match.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OPS = {"dtg_chain": "tl::OpChain,", "dtg_chain_bwd": "tl::OpChainBwd,"}
DOUBLES_READ = {"dtg_chain": 43, "dtg_chain_bwd": 40}
DOUBLES_WRITTEN = {"dtg_chain": 6, "dtg_chain_bwd": 43}


def sources_sha256(root=None):
    """Hash of everything the library's machine code is built from: every
    file under the package's ``csrc/`` (kernels, device bodies, the ABI and
    the generated kernels), the public headers ``include/*.h`` and the
    compiler flags of the build (with the repository path taken out).  A
    counter figure taken from other code than this hash describes is stale."""
    from . import build as tlbuild
    root = os.path.dirname(PKG) if root is None else root
    csrc = os.path.join(root, os.path.basename(PKG), "csrc")
    inc = os.path.join(root, "include")
    files = []
    for d, _, names in os.walk(csrc):
        files += [os.path.join(d, x) for x in names if not x.endswith((".pyc", ".o", ".so"))]
    files += [os.path.join(inc, x) for x in os.listdir(inc) if x.endswith(".h")]
    h = hashlib.sha256()
    for fn in sorted(files, key=lambda x: os.path.relpath(x, root)):
        with open(fn, "rb") as f:
            h.update(os.path.relpath(fn, root).encode() + b"\0" + f.read())
    flags = [x.replace(tlbuild.ROOT, "$ROOT") for x in tlbuild.COMMON]
    h.update(b"\0flags\0" + " ".join(flags).encode())
    return h.hexdigest()


def _csv(folder, suffix):
    files = sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {folder}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def short(name, width=90):
    return name if len(name) <= width else name[:width - 3] + "..."


def kernel_stats(folder):
    rows = _csv(folder, "kernel_stats.csv")
    out = []
    for r in rows:
        out.append({"name": r["Name"], "calls": int(r["Calls"]),
                    "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                    "pct": float(r.get("Percentage", 0.0))})
    return sorted(out, key=lambda r: -r["total_ns"])


def launch_shapes(folder):
    """Per (kernel, grid size): dispatches, average duration (ns), VGPRs."""
    rows = _csv(folder, "kernel_trace.csv")
    agg = defaultdict(list)
    vgpr = {}
    for r in rows:
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]))
        agg[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        vgpr[key] = int(r["VGPR_Count"]) + int(r.get("Accum_VGPR_Count", 0) or 0)
    out = [{"name": k[0], "grid": k[1], "calls": len(v), "avg_ns": sum(v) / len(v),
            "min_ns": min(v), "max_ns": max(v), "total_ns": sum(v), "vgpr": vgpr[k]}
           for k, v in agg.items()]
    return sorted(out, key=lambda r: -r["total_ns"])


# Algorithmic bytes per grid point of each kernel named in a dispatch label
# (8 B per stored element read or written).
LABEL_BYTES = {"sym_inverse": 96, "christoffel": 336, "cov_deriv": 312, "dtg": 176,
               "dtg_chain": 392, "dtg_chain_bwd": 664, "dtg_chain_fwd_bwd": 784,
               "dtg_chain_batched": 392, "dtg_chain_bwd_batched": 664}
LABEL = re.compile(r"^c(\d+) (\w+) n=(\d+)(?: (.*))?$")
HBM_PEAK_GBS = 8000.0


SPLIT = re.compile(r"\b(\d+) launches\b")


def labelled_dispatches(folder):
    """Per dispatch label ``c<config> <kernel> n=<points> [variant]`` (the names
    bench.py --label-kernels gives its calls, which the profiler's kernel
    renaming puts in place of the kernel name): calls, average, min and max
    duration (ns), and the algorithmic GB/s and fraction of the HBM peak of
    the average.  A variant "<K> launches" marks n points split over K
    launches, whose rate is taken over K average durations."""
    rows = _csv(folder, "kernel_trace.csv")
    agg = defaultdict(list)
    for r in rows:
        if LABEL.match(r["Kernel_Name"].strip()):
            agg[r["Kernel_Name"].strip()].append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = []
    for name, v in agg.items():
        m = LABEL.match(name)
        cfg, kernel, n, variant = int(m.group(1)), m.group(2), int(m.group(3)), m.group(4) or ""
        avg = sum(v) / len(v)
        k = SPLIT.search(variant)
        per = avg * (int(k.group(1)) if k else 1)
        gbs = LABEL_BYTES[kernel] * n / per if kernel in LABEL_BYTES else None
        out.append({"label": name, "config": cfg, "kernel": kernel, "points": n,
                    "variant": variant, "calls": len(v), "avg_ns": avg, "min_ns": min(v),
                    "max_ns": max(v), "GB_s": gbs,
                    "frac": gbs / HBM_PEAK_GBS if gbs is not None else None})
    return sorted(out, key=lambda r: (r["config"], r["points"], r["kernel"], r["variant"]))


def bench_lines(specs):
    """[(label, JSON record)] of the benchmark lines in the files ``LABEL=PATH``."""
    out = []
    for spec in specs:
        label, _, fn = spec.rpartition("=")
        with open(fn) as f:
            for line in f:
                if line.startswith('{"metric"'):
                    out.append((label or os.path.basename(fn), json.loads(line)))
    return out


def counters(folder, counter):
    """{kernel name: {grid size: [values]}} of one counter (KiB per dispatch)."""
    rows = _csv(folder, "counter_collection.csv")
    agg = defaultdict(lambda: defaultdict(list))
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        agg[r["Kernel_Name"]][int(r["Grid_Size"])].append(float(r["Counter_Value"]))
    return agg


def _largest(agg, needle):
    best = None
    for name, by_grid in agg.items():
        if needle in name:
            for grid, vals in by_grid.items():
                if best is None or grid > best[1]:
                    best = (name, grid, vals)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--labels", help="kernel trace of a run with labelled dispatches "
                    "(bench.py --label-kernels under --kernel-rename); default: --trace")
    ap.add_argument("--labels-cmd", default="", help="the labelled run's command")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cmd", required=True, help="the profiled command, for the record")
    ap.add_argument("--pmc-cmd", default="", help="the counter runs' command")
    ap.add_argument("--points", type=int, required=True, help="grid points per launch")
    ap.add_argument("--copy-doubles", type=int, default=64 * 1024 * 1024)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--bench", nargs="*", default=[],
                    help="LABEL=FILE of bench.py's JSON line (the profiled run's output, and "
                         "the same workload's unprofiled run)")
    ap.add_argument("--out", default="profiles")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)

    st = kernel_stats(a.trace)
    path = os.path.join(a.out, f"kernel_stats_{a.workload}.md")
    with open(path, "w") as f:
        f.write(f"# rocprofv3 kernel statistics: {a.workload}\n\n")
        f.write(f"Command ($REPO is the repository root, $OUT the directory the results went to; "
                f"run from /tmp with TMPDIR=/tmp):\n\n"
                f"    {a.cmd}\n\n")
        f.write("| kernel | calls | average (us) | total (us) | % |\n|---|---|---|---|---|\n")
        for r in st[:20]:
            f.write(f"| `{short(r['name'])}` | {r['calls']} | {r['avg_ns'] / 1e3:.2f} | "
                    f"{r['total_ns'] / 1e3:.1f} | {r['pct']:.1f} |\n")
        f.write("\nThe same dispatches split by launch size (from the kernel trace), the ten "
                "largest by total time:\n\n"
                "| kernel | grid (work-items) | calls | average (us) | VGPRs |\n"
                "|---|---|---|---|---|\n")
        for r in launch_shapes(a.trace)[:10]:
            f.write(f"| `{short(r['name'])}` | {r['grid']} | {r['calls']} | "
                    f"{r['avg_ns'] / 1e3:.2f} | {r['vgpr']} |\n")
        shapes = launch_shapes(a.trace)
        f.write(f"\nThe kernels of the benchmark step (one launch each over {a.points} points; "
                "every dispatch of that kernel at that size in the run, the step's and the "
                "other rows' alike):\n\n"
                "| kernel | grid (work-items) | calls | average (us) | min (us) | max (us) |\n"
                "|---|---|---|---|---|---|\n")
        for kernel, needle in OPS.items():
            for r in shapes:
                if r["name"].startswith("void tl::k_points<" + needle) and r["grid"] == a.points:
                    f.write(f"| `{short(r['name'])}` ({kernel}) | {r['grid']} | {r['calls']} | "
                            f"{r['avg_ns'] / 1e3:.2f} | {r['min_ns'] / 1e3:.2f} | "
                            f"{r['max_ns'] / 1e3:.2f} |\n")
        lab = labelled_dispatches(a.labels or a.trace)
        if lab:
            f.write("\nEvery labelled dispatch of the run by configuration (bench.py "
                    "--label-kernels; kernel durations from the trace; GB/s = algorithmic "
                    "bytes of the launch / average duration)"
                    + (f", from\n\n    {a.labels_cmd}\n\n" if a.labels_cmd else ":\n\n")
                    + "| configuration | kernel | points | variant | calls | average (us) | "
                    "min (us) | max (us) | GB/s | of 8 TB/s |\n"
                    "|---|---|---|---|---|---|---|---|---|---|\n")
            for r in lab:
                g = "" if r["GB_s"] is None else f"{r['GB_s']:.0f}"
                fr = "" if r["frac"] is None else f"{100 * r['frac']:.1f} %"
                f.write(f"| {r['config']} | {r['kernel']} | {r['points']} | {r['variant']} | "
                        f"{r['calls']} | {r['avg_ns'] / 1e3:.2f} | {r['min_ns'] / 1e3:.2f} | "
                        f"{r['max_ns'] / 1e3:.2f} | {g} | {fr} |\n")
        lines = bench_lines(a.bench)
        if lines:
            f.write("\nbench.py's own timing of its dominant kernel (HIP events on the kernel's "
                    "stream, averaged over the timed region):\n\n"
                    "| run | kernel | average (us) | achieved (GB/s) | fraction of peak |\n"
                    "|---|---|---|---|---|\n")
            for label, d in lines:
                r = d["roofline"]
                f.write(f"| {label} | {r['kernel']} | {r['duration_us']:.2f} | "
                        f"{r['achieved']:.1f} | {r['frac']:.4f} |\n")
    print("wrote", path)

    if not (a.fetch and a.write):
        return
    fetch = counters(a.fetch, "FETCH_SIZE")
    write = counters(a.write, "WRITE_SIZE")
    copy_bytes = 8 * a.copy_doubles
    cf = _largest(fetch, "k_copy")
    cw = _largest(write, "k_copy")
    f_scale = copy_bytes / (1024 * sum(cf[2]) / len(cf[2]))
    w_scale = copy_bytes / (1024 * sum(cw[2]) / len(cw[2]))
    sha = sources_sha256()
    for kernel, needle in OPS.items():
        kf = _largest(fetch, needle)
        kw = _largest(write, needle)
        if kf is None or kw is None:
            continue
        fk = sum(kf[2]) / len(kf[2])
        wk = sum(kw[2]) / len(kw[2])
        fetch_b = fk * 1024 * f_scale
        write_b = wk * 1024 * w_scale
        alg_r = 8 * DOUBLES_READ[kernel] * a.points
        alg_w = 8 * DOUBLES_WRITTEN[kernel] * a.points
        path = os.path.join(a.out, f"pmc_{kernel}.md")
        with open(path, "w") as f:
            f.write(f"# HBM traffic of {kernel}: {a.workload}\n\n"
                    f"Two counter runs, one counter each ($REPO is the repository root, $OUT the "
                    f"directory the results went to; run "
                    f"from /tmp with TMPDIR=/tmp):\n\n"
                    f"    {a.pmc_cmd.replace('COUNTER', 'FETCH_SIZE')}\n"
                    f"    {a.pmc_cmd.replace('COUNTER', 'WRITE_SIZE')}\n\n"
                    f"Kernel: `{short(kf[0], 120)}`, grid {kf[1]} work-items, "
                    f"{len(kf[2])} dispatches averaged.\n\n"
                    "Calibration: the library's streaming copy of "
                    f"{copy_bytes} B read and written per launch reads FETCH_SIZE "
                    f"{sum(cf[2]) / len(cf[2]):.1f} KiB and WRITE_SIZE "
                    f"{sum(cw[2]) / len(cw[2]):.1f} KiB, so the scale factors are "
                    f"{f_scale:.4f} (fetch) and {w_scale:.4f} (write).\n\n"
                    "| | counter (KiB/dispatch) | scaled bytes | algorithmic bytes | ratio |\n"
                    "|---|---|---|---|---|\n"
                    f"| read | {fk:.1f} | {fetch_b:.0f} | {alg_r} | {fetch_b / alg_r:.4f} |\n"
                    f"| write | {wk:.1f} | {write_b:.0f} | {alg_w} | {write_b / alg_w:.4f} |\n\n"
                    "Machine-readable record (read by bench.py):\n\n")
            f.write(f"kernel: {kernel}\n")
            f.write(f"points: {a.points}\n")
            f.write(f"sources_sha256: {sha}\n")
            f.write(f"fetch_bytes_per_launch: {fetch_b:.0f}\n")
            f.write(f"write_bytes_per_launch: {write_b:.0f}\n")
            f.write(f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}\n")
            f.write(f"algorithmic_bytes_per_launch: {alg_r + alg_w}\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
