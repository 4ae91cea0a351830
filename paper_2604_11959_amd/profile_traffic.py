"""HBM traffic of the regular-region kernel from rocprofv3 counter runs.

    python -m paper_2604_11959_amd.profile_traffic PMC_DIR OUT_JSON --command "..."

PMC_DIR holds the CSV output of four ``rocprofv3 --pmc`` runs (one counter
each, as the hardware allows): ``fetch`` and ``write`` of the benchmark (one
RK step, no graph, so every stage is its own dispatch) and ``cfetch`` /
``cwrite`` of a plain 1 GiB device copy (``bench.py --calib-copy``).  The copy
reads and writes exactly 2^30 bytes, which fixes the scale factor of each
counter (FETCH_SIZE counts some request sizes at half width).  The summary
records the mean calibrated bytes per regular-region launch, a SHA-256 of
the kernel source and the algorithmic bytes of one launch (which fix the
regular region it covered), so that a later change of either invalidates it.
It also records the calibrated bytes per stage of each pass over the general
range and the redistribution, with a SHA-256 of their sources.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", n) for n in ("bulk.hip", "stage_common.h")]
GENERAL_SOURCES = [os.path.join(HERE, "csrc", n) for n in ("stage.hip", "wsrd.hip", "stage_common.h", "xcd.h")]
COPY_BYTES = 1 << 30
# the kernels of a stage besides the regular-region one
GENERAL_PASSES = ("k_gen_prims", "k_gen_fhat", "k_gen_cut", "k_gen_update", "k_qhat", "k_grad", "k_final")


def source_sha256(paths=None) -> str:
    """SHA-256 over the given sources (default: the regular-region kernel's)."""
    h = hashlib.sha256()
    for path in paths or KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _per_dispatch(path: str, counter: str):
    """{dispatch id: (kernel name, summed value in KiB)} for one counter."""
    out = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, val = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, val + float(r["Counter_Value"]))
    return out


def _copy_kib(path: str, counter: str) -> float:
    vals = [v for n, v in _per_dispatch(path, counter).values() if "copyBuffer" in n]
    if not vals:
        raise SystemExit(f"no copy dispatch in {path}")
    return max(vals)


def summarize(pmc_dir: str, kernel_prefix: str = "k_bulk"):
    f = lambda name: os.path.join(pmc_dir, f"{name}_counter_collection.csv")
    fetch = _per_dispatch(f("fetch"), "FETCH_SIZE")
    write = _per_dispatch(f("write"), "WRITE_SIZE")
    fscale = COPY_BYTES / (_copy_kib(f("cfetch"), "FETCH_SIZE") * 1024.0)
    wscale = COPY_BYTES / (_copy_kib(f("cwrite"), "WRITE_SIZE") * 1024.0)
    pick = lambda d: [v for _, (n, v) in sorted(d.items()) if kernel_prefix in n]
    fk, wk = pick(fetch), pick(write)
    if not fk or len(fk) != len(wk):
        raise SystemExit("fetch / write runs do not hold the same regular-region dispatches")
    per_launch = [fv * 1024.0 * fscale + wv * 1024.0 * wscale for fv, wv in zip(fk, wk)]
    # the passes over the general range and the redistribution: calibrated
    # bytes per stage of each of their kernels, averaged over the stages of
    # the run (dispatches from the first regular-region launch on)
    ids = sorted(fetch)
    first = next(d for d in ids if kernel_prefix in fetch[d][0])
    other = {}
    for d in ids:
        if d <= first or d not in write:
            continue
        name = fetch[d][0].replace("void ", "").replace("ebs::(anonymous namespace)::", "").strip()
        name = name.split("<")[0].split("(")[0]
        if name not in GENERAL_PASSES:
            continue
        b = fetch[d][1] * 1024.0 * fscale + write[d][1] * 1024.0 * wscale
        other.setdefault(name, []).append(b)
    stage_bytes = {n: sum(v) / len(per_launch) for n, v in other.items()}
    return {
        "kernel": kernel_prefix,
        "launches": len(per_launch),
        "fetch_kib_per_launch": fk,
        "write_kib_per_launch": wk,
        "fetch_scale": fscale,
        "write_scale": wscale,
        "traffic_bytes_per_launch": sum(per_launch) / len(per_launch),
        "general_range_bytes_per_stage": stage_bytes,
        "kernel_source_sha256": source_sha256(),
        "general_source_sha256": source_sha256(GENERAL_SOURCES),
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("pmc_dir")
    ap.add_argument("out_json")
    ap.add_argument("--command", default="", help="the profiling command, recorded verbatim")
    ap.add_argument("--workload", default="")
    ap.add_argument("--tile", default="")
    ap.add_argument("--bench-log", default="",
                    help="output of the profiled bench run; its algorithmic bytes per launch are recorded")
    args = ap.parse_args(argv)
    s = summarize(args.pmc_dir)
    s["alg_bytes_per_launch"] = None
    if args.bench_log:
        with open(args.bench_log) as f:
            for line in f:
                if line.startswith("{") and '"roofline"' in line:
                    s["alg_bytes_per_launch"] = json.loads(line)["roofline"]["alg_bytes_per_launch"]
    s["command"] = args.command
    s["workload"] = args.workload
    s["tile"] = [int(v) for v in args.tile.split("x")] if args.tile else None
    with open(args.out_json, "w") as fo:
        json.dump(s, fo, indent=1)
        fo.write("\n")
    print(json.dumps(s))
    return 0


if __name__ == "__main__":
    sys.exit(main())
