"""Summaries of rocprofv3 outputs (CSV) for the committed profile notes.

    python -m paper_2508_20735_amd.profiling stats <kernel_stats.csv>
    python -m paper_2508_20735_amd.profiling traffic <fetch_dir> <write_dir> \
        --copy-bytes N [--out profiles/traffic.json]

``stats`` prints a markdown table of the per-kernel totals of a
``rocprofv3 --kernel-trace --stats`` run.  ``traffic`` reads the counter
collections of two ``rocprofv3 --pmc`` runs (FETCH_SIZE, then WRITE_SIZE, in
KiB per dispatch) and converts them into HBM bytes per launch of every round
kernel, scaling each counter by what it reads for a plain device copy of
known size (``--copy-bytes``; the run must contain exactly such a copy, e.g.
``bench.py --copy-calibration-mib 512``).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROUND_KERNELS = ("k_mark", "k_signature", "k_insert", "k_insert_lds", "k_insert_lds2",
                 "k_round_end", "k_pattern_round", "k_packed_round", "k_pb_gather",
                 "k_signature_pb", "k_pb_count", "k_pb_scatter", "k_pb_gather8",
                 "k_packed_pb", "k_count_labels")
# The library's per-kernel timing names a launch of the grouping step
# "k_insert": one dispatch of an LDS-staged variant and one of the plain
# kernel, of which exactly one does the round's work.  "k_packed_pb" is the
# packed label round through slices: the byte gather, the round, and the
# count of the labels it marked.
LIBRARY_GROUPS = {"k_insert": ("k_insert_lds2", "k_insert_lds", "k_insert"),
                  "k_packed_pb": ("k_pb_gather8", "k_packed_pb", "k_count_labels")}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def short_name(name: str) -> str:
    """'void dfamin::(anonymous namespace)::k_signature<4>(...)' -> 'k_signature<4>'."""
    name = re.sub(r"^void ", "", name).replace("(anonymous namespace)::", "")
    name = name.split("(")[0]
    return name.split("::")[-1].strip()


def base_name(name: str) -> str:
    return re.sub(r"<.*>$", "", short_name(name))


def kernel_stats_table(path: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append("| {} | {} | {:.3f} | {:.2f} | {:.2f} | {:.2f} | {} |".format(
            short_name(r["Name"]), r["Calls"], int(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, int(r["MinNs"]) / 1e3, int(r["MaxNs"]) / 1e3,
            r["Percentage"]))
    return "\n".join(lines)


def _counter_rows(run_dir: str):
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection CSV under {run_dir}")
    for path in files:
        yield from csv.DictReader(open(path))


def per_dispatch(run_dir: str, counter: str) -> dict:
    """{dispatch id: (kernel name, counter value summed over its instances)}."""
    out = {}
    for r in _counter_rows(run_dir):
        if r.get("Counter_Name") != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r.get("Kernel_Name", "")
        val = float(r.get("Counter_Value", 0) or 0)
        prev = out.get(did)
        out[did] = (name, (prev[1] if prev else 0.0) + val)
    return out


def kernel_source_digest(root: str) -> str:
    h = hashlib.sha1()
    for f in ("refine_kernels.hip", "dfamin_internal.h", "device_common.h"):
        with open(os.path.join(root, "paper_2508_20735_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    fetch = per_dispatch(fetch_dir, "FETCH_SIZE")
    write = per_dispatch(write_dir, "WRITE_SIZE")

    def kib_by_kernel(d):
        acc = defaultdict(list)
        for name, val in d.values():
            acc[name].append(val * 1024.0)
        return acc

    fk, wk = kib_by_kernel(fetch), kib_by_kernel(write)
    copy_f = [v for n, vs in fk.items() if COPY_KERNEL in n for v in vs]
    copy_w = [v for n, vs in wk.items() if COPY_KERNEL in n for v in vs]
    big_f = max(copy_f) if copy_f else 0.0
    big_w = max(copy_w) if copy_w else 0.0
    if big_f <= 0 or big_w <= 0:
        raise RuntimeError("the runs contain no calibration copy")
    sf, sw = copy_bytes / big_f, copy_bytes / big_w
    out = {"copy_bytes": copy_bytes, "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    names = {base_name(n) for n in fk} | {base_name(n) for n in wk}
    for b in sorted(names):
        if b not in ROUND_KERNELS:
            continue
        fv = [v for n, vs in fk.items() if base_name(n) == b for v in vs]
        wv = [v for n, vs in wk.items() if base_name(n) == b for v in vs]
        if not fv or not wv:
            continue
        f_avg = sum(fv) / len(fv) * sf
        w_avg = sum(wv) / len(wv) * sw
        out["kernels"][b] = {"launches": len(fv), "fetch_bytes_per_launch": f_avg,
                             "write_bytes_per_launch": w_avg,
                             "hbm_bytes_per_launch": f_avg + w_avg}
    # per launch under the library's timing names (bench.py's "kernel")
    lib = {}
    for b, e in out["kernels"].items():
        if not any(b in members for members in LIBRARY_GROUPS.values()):
            lib[b] = dict(e)
    for name, members in LIBRARY_GROUPS.items():
        parts = [out["kernels"][m] for m in members if m in out["kernels"]]
        if not parts:
            continue
        launches = max(p["launches"] for p in parts)
        f_tot = sum(p["fetch_bytes_per_launch"] * p["launches"] for p in parts)
        w_tot = sum(p["write_bytes_per_launch"] * p["launches"] for p in parts)
        lib[name] = {"launches": launches, "fetch_bytes_per_launch": f_tot / launches,
                     "write_bytes_per_launch": w_tot / launches,
                     "hbm_bytes_per_launch": (f_tot + w_tot) / launches,
                     "dispatches": {m: out["kernels"][m]["launches"]
                                    for m in members if m in out["kernels"]}}
    out["library_kernels"] = lib
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--out")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(kernel_stats_table(args.csv, args.top))
        return 0
    res = traffic(args.fetch_dir, args.write_dir, args.copy_bytes)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res["kernel_source_sha1"] = kernel_source_digest(root)
    text = json.dumps(res, indent=2)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
