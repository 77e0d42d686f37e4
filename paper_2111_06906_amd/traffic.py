"""Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) into HBM bytes per
verification call (the sum over its kernels), scaled by what the same counters read for a plain
device-to-device copy of known size, and store them with the hash of the kernel
sources they were taken on.

    python -m paper_2111_06906_amd.traffic <fetch_dir> <write_dir> <copy_MiB> [out.json]

Both runs profile ``bench.py --calib-copy-mib <copy_MiB>``, which enqueues one
copy of that size before the timed frames.  Per kernel the first launch of a
run is a warm-up and is dropped.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources whose change invalidates stored counter readings
VERIFY_SOURCES = ("paper_2111_06906_amd/csrc/pv_device.h", "paper_2111_06906_amd/csrc/pv_kernels.hip")


def _code_only(text: str) -> str:
    """The source without comments and blank runs: editing a comment does not
    change the kernels the counters were read on.  (No string literal in these
    sources contains a comment marker.)"""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sources_sha1(root: str = ROOT) -> str:
    h = hashlib.sha1()
    for rel in VERIFY_SOURCES:
        with open(os.path.join(root, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_kernel(rows, counter):
    out = {}
    for r in rows:
        if r.get("Counter_Name") == counter:
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _pick(d, key):
    for k, v in d.items():
        if key in k:
            return v
    raise SystemExit("kernel %r not in counter output" % key)


# kernels launched once per verification call (the shared scan kernels that
# also serve queue building and photon compaction are not attributed)
VERIFY_KERNELS = ("k_verify_scan", "k_verify_gather", "k_verify_trace", "k_verify_finish", "k_verify_stats")


def _per_call(d):
    """Mean over launches (the first, a warm-up, dropped) summed over the
    kernels of one verification call."""
    tot, n = 0.0, 0
    for k, v in d.items():
        if any(name in k for name in VERIFY_KERNELS):
            v = v[1:] or v
            tot += sum(v) / len(v)
            n = max(n, len(v))
    if not n:
        raise SystemExit("no verification kernels in counter output")
    return tot, n


def summarize(fetch_dir, write_dir, copy_mib):
    fetch = _per_kernel(_rows(fetch_dir), "FETCH_SIZE")
    write = _per_kernel(_rows(write_dir), "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    # the largest copy dispatch is the calibration copy
    sf = max(_pick(fetch, "copyBuffer")) / copy_kib
    sw = max(_pick(write, "copyBuffer")) / copy_kib
    vf, nf = _per_call(fetch)
    vw, nw = _per_call(write)
    fb = vf * 1024.0 / sf
    wb = vw * 1024.0 / sw
    return {"kernel": "verification call: " + " + ".join(VERIFY_KERNELS), "fetch_bytes_per_launch": fb,
            "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb, "copy_scale_fetch": sf,
            "copy_scale_write": sw, "launches": [nf, nw], "calibration": "%g MiB device-to-device copy" % copy_mib,
            "sources_sha1": sources_sha1()}


def main(argv):
    if len(argv) < 3:
        raise SystemExit(__doc__)
    rec = summarize(argv[0], argv[1], float(argv[2]))
    out = argv[3] if len(argv) > 3 else os.path.join(ROOT, "profiles", "verify_traffic.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:])
