"""HBM traffic of the renderer's kernels from rocprofv3 counter runs.

Two ``rocprofv3 --pmc`` runs of the same command (one with FETCH_SIZE, one
with WRITE_SIZE; both report KiB per dispatch) are reduced to bytes per
launch for each kernel (each entry keeps the workload and command it was
measured with; ``--merge`` adds the kernels of another schedule to an
existing record). Each counter is scaled by the factor that makes a
plain elementwise copy of known size (run inside the same command) read and
write exactly its size. The record carries a digest of the kernel sources
it was measured on, so a reader can tell when the kernels have changed
since.

    python -m paper_2410_08129_amd.pmc --fetch F.csv --write W.csv \\
        --copy-bytes 268435456 --workload "..." --command "..." --out traffic.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# kernel name prefix -> source files that define it
KERNEL_SOURCES = {
    "k_raster_fwd": ("raster.hip", "common.h"),
    "k_raster_bwd": ("raster.hip", "common.h"),
    "k_preprocess": ("preprocess.hip", "common.h"),
    "k_preprocess_bwd": ("preprocess.hip", "common.h"),
    "k_sort_pass": ("sort.hip", "common.h"),
    "k_ranges": ("sort.hip", "common.h"),
    "k_fill_zero": ("preprocess.hip", "common.h"),
}


def short_name(full: str) -> str:
    n = full.replace("void ", "").replace("htgs::", "").split("(")[0]
    return n.split("<")[0].strip()


def source_digest(kernel: str) -> str:
    """sha256 over the source files of ``kernel`` (short name)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _per_kernel(path):
    d = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d


def summarize(fetch_csv, write_csv, copy_bytes):
    fetch, write = _per_kernel(fetch_csv), _per_kernel(write_csv)
    # the calibration copy: the elementwise kernel whose FETCH_SIZE is
    # closest to its known size
    best = None
    for k, vals in fetch.items():
        if "elementwise" not in k:
            continue
        for i, v in enumerate(vals):
            ratio = copy_bytes / max(v * 1024.0, 1.0)
            if 0.25 < ratio < 4.0 and (best is None or abs(ratio - 1.0) < abs(best[0] - 1.0)):
                best = (ratio, k, i)
    if best is None:
        raise SystemExit("no calibration copy found in the counter runs")
    _, ck, ci = best
    sf = copy_bytes / (fetch[ck][ci] * 1024.0)
    sw = copy_bytes / (write[ck][ci] * 1024.0)
    kernels = {}
    for k, vals in fetch.items():
        name = short_name(k)
        if name not in KERNEL_SOURCES:
            continue
        wv = write.get(k, [0.0])
        key = k.replace("void ", "").replace("htgs::", "").split("(")[0]
        kernels[key] = dict(
            kernel=name, launches=len(vals),
            fetch_kib=sum(vals) / len(vals), write_kib=sum(wv) / len(wv),
            read_bytes=sum(vals) / len(vals) * 1024.0 * sf,
            write_bytes=sum(wv) / len(wv) * 1024.0 * sw,
            source_sha256=source_digest(name))
    return dict(scale_fetch=sf, scale_write=sw, copy_bytes=copy_bytes, kernels=kernels)


def traffic_for(record_path, kernel_key):
    """Scaled HBM bytes per launch (read + write) of ``kernel_key`` from a
    stored record, or None if absent or measured on other sources."""
    if not os.path.exists(record_path):
        return None
    with open(record_path) as fh:
        rec = json.load(fh)
    k = rec.get("kernels", {}).get(kernel_key)
    if k is None or k["source_sha256"] != source_digest(k["kernel"]):
        return None
    return dict(read=k["read_bytes"], write=k["write_bytes"],
                total=k["read_bytes"] + k["write_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--workload", default="")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--merge", action="store_true",
                    help="keep the kernels of an existing record that this run did not launch")
    a = ap.parse_args()
    rec = summarize(a.fetch, a.write, a.copy_bytes)
    for k in rec["kernels"].values():
        k["workload"] = a.workload
        k["command"] = a.command
    if a.merge and os.path.exists(a.out):
        with open(a.out) as fh:
            old = json.load(fh)
        for key, k in old.get("kernels", {}).items():
            rec["kernels"].setdefault(key, k)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    for k, v in rec["kernels"].items():
        print(f"{k:40s} read {v['read_bytes'] / 1e6:9.1f} MB  write {v['write_bytes'] / 1e6:9.1f} MB")


if __name__ == "__main__":
    main()
