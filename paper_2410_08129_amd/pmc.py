"""HBM traffic of the renderer's kernels from rocprofv3 counter runs.

Two ``rocprofv3 --pmc`` runs of the same command are reduced to bytes per
launch for each kernel (each entry keeps the workload and command it was
measured with; ``--merge`` adds the kernels of another schedule to an
existing record):

* reads: the L2-to-memory read requests by size, TCC_EA0_RDREQ_32B_sum,
  TCC_EA0_RDREQ_64B_sum and TCC_EA0_RDREQ_128B_sum (with TCC_EA0_RDREQ_sum,
  which they should add up to); bytes = 32 n32 + 64 n64 + 128 n128. (The
  derived FETCH_SIZE of this ROCm counts a 128-byte request as 64 bytes
  unless the memory reported it as a bubble, so it reads half of a
  streaming copy's bytes and the right amount of a gather of small
  requests: no single scale factor fits every kernel.)
* writes: TCC_EA0_WRREQ_sum and TCC_EA0_WRREQ_64B_sum; bytes = 32 (n - n64)
  + 64 n64 (the derived WRITE_SIZE).

A plain elementwise copy of known size, run inside the same command, checks
the byte counts (its ratio is reported; nothing is scaled). The record
carries a digest of the kernel sources it was measured on, so a reader can
tell when the kernels have changed since.

    python -m paper_2410_08129_amd.pmc --fetch R.csv --write W.csv \\
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
    "k_preprocess_scan": ("preprocess.hip", "common.h"),
    "k_emit": ("preprocess.hip", "common.h"),
    "k_sort_count": ("sort.hip", "common.h"),
    "k_sort_scan": ("sort.hip", "common.h"),
    "k_sort_scatter": ("sort.hip", "common.h"),
    "k_ranges": ("sort.hip", "common.h"),
    "k_tile_order_count": ("sort.hip", "common.h"),
    "k_tile_order_place": ("sort.hip", "common.h"),
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
    """{kernel: {counter: [value per dispatch]}}"""
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(path) as fh:
        for r in csv.DictReader(fh):
            d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return d


def _read_bytes(c):
    n = [c.get(f"TCC_EA0_RDREQ_{b}B_sum") for b in (32, 64, 128)]
    if any(v is None for v in n):
        raise SystemExit("read run lacks TCC_EA0_RDREQ_{32,64,128}B_sum")
    return [32 * a + 64 * b + 128 * q for a, b, q in zip(*n)]


def _write_bytes(c):
    n, n64 = c.get("TCC_EA0_WRREQ_sum"), c.get("TCC_EA0_WRREQ_64B_sum")
    if n is None or n64 is None:
        raise SystemExit("write run lacks TCC_EA0_WRREQ_sum / TCC_EA0_WRREQ_64B_sum")
    return [32 * (a - b) + 64 * b for a, b in zip(n, n64)]


def summarize(read_csv, write_csv, copy_bytes):
    rd, wr = _per_kernel(read_csv), _per_kernel(write_csv)
    # the check copy: the elementwise kernel whose read bytes are closest
    # to its known size
    best = None
    for k, c in rd.items():
        if "elementwise" not in k:
            continue
        for i, v in enumerate(_read_bytes(c)):
            ratio = v / copy_bytes
            if 0.25 < ratio < 4.0 and (best is None or abs(ratio - 1.0) < abs(best[0] - 1.0)):
                best = (ratio, k, i)
    if best is None:
        raise SystemExit("no check copy found in the counter runs")
    _, ck, ci = best
    copy_read = _read_bytes(rd[ck])[ci] / copy_bytes
    copy_write = _write_bytes(wr[ck])[ci] / copy_bytes if ck in wr else None
    kernels = {}
    for k, c in rd.items():
        name = short_name(k)
        if name not in KERNEL_SOURCES:
            continue
        rb = _read_bytes(c)
        wb = _write_bytes(wr[k]) if k in wr else [0.0]
        req = c.get("TCC_EA0_RDREQ_sum", [0.0])
        sizes = {f"rdreq_{b}B": sum(c[f"TCC_EA0_RDREQ_{b}B_sum"]) / len(rb) for b in (32, 64, 128)}
        key = k.replace("void ", "").replace("htgs::", "").split("(")[0]
        kernels[key] = dict(
            kernel=name, launches=len(rb), rdreq=sum(req) / len(req), **sizes,
            read_bytes=sum(rb) / len(rb), write_bytes=sum(wb) / len(wb),
            source_sha256=source_digest(name))
    return dict(copy_check=dict(bytes=copy_bytes, read_ratio=copy_read, write_ratio=copy_write),
                kernels=kernels)


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
