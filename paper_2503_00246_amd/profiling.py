"""Summaries of rocprofv3 output for the benchmark's kernels.

    python -m paper_2503_00246_amd.profiling trace DIR                # kernel-trace --stats directory
    python -m paper_2503_00246_amd.profiling bytes FETCH_DIR WRITE_DIR KEY [--out profiles/traffic.json]

`bytes` scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of the ghost kernel by what the
same counters read for the plain device copy that `bench.py --calibrate` runs on a buffer of known size
(n_lattice * 8 bytes read and written), and records bytes per launch with the hash of the kernel source.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2503_00246_amd", "csrc", "ghost_kernels.hip")


def _csv(directory, suffix):
    files = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def short_name(name):
    base = name.replace("ghost::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
    return base[:90]


def trace_summary(directory):
    """Per-kernel calls, average and total duration from a --kernel-trace --stats run."""
    rows = _csv(directory, "kernel_stats.csv")
    out = []
    for r in rows:
        out.append({"kernel": short_name(r["Name"]), "calls": int(r["Calls"]),
                    "avg_us": float(r["AverageNs"]) / 1e3, "total_ms": float(r["TotalDurationNs"]) / 1e6,
                    "pct": float(r["Percentage"])})
    return out


def counter_per_kernel(directory, counter):
    rows = _csv(directory, "counter_collection.csv")
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return per


def scaled_bytes(fetch_dir, write_dir, kernel_key, copy_key="copyBuffer", copy_bytes=None):
    """(fetch bytes, write bytes) per launch of the kernel whose name contains kernel_key.

    The calibration copy is the largest dispatch of the copy kernel (small uploads use it too).
    """
    fetch = counter_per_kernel(fetch_dir, "FETCH_SIZE")
    write = counter_per_kernel(write_dir, "WRITE_SIZE")

    def pick(per, key, agg=statistics.median):
        vals = [v for k, vs in per.items() if key in k for v in vs]
        if not vals:
            raise KeyError(f"no kernel matching {key!r}")
        return agg(vals)

    f_k, w_k = pick(fetch, kernel_key), pick(write, kernel_key)
    f_c, w_c = pick(fetch, copy_key, max), pick(write, copy_key, max)
    fs = ws = 1024.0  # counters are KiB per dispatch
    if copy_bytes:
        fs, ws = copy_bytes / f_c, copy_bytes / w_c
    return f_k * fs, w_k * ws, {"fetch_scale_bytes_per_unit": fs, "write_scale_bytes_per_unit": ws,
                                "copy_fetch_units": f_c, "copy_write_units": w_c}


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    b = sub.add_parser("bytes")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("key", help="workload/scatter/precision key for the traffic file")
    b.add_argument("--kernel", default="box_kernel<double")
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "trace":
        for r in trace_summary(a.dir):
            print(f"| {r['kernel']} | {r['calls']} | {r['avg_us']:.2f} | {r['total_ms']:.3f} | {r['pct']:.1f} |")
    else:
        fb, wb, scale = scaled_bytes(a.fetch_dir, a.write_dir, a.kernel, copy_bytes=a.copy_bytes)
        rec = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb, "kernel_sha": kernel_sha(),
               **scale}
        print(json.dumps({a.key: rec}, indent=1))
        if a.out:
            data = {}
            if os.path.exists(a.out):
                with open(a.out) as f:
                    data = json.load(f)
            data[a.key] = rec
            with open(a.out, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
