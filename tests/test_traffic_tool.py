"""Host logic of the HBM-traffic summary: counter rows to bytes per
verification call, scaled by the calibration copy; the source hash ignores
comments."""
import csv
import os

import pytest

from paper_2111_06906_amd import traffic as T

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_bytes_per_call_scaled_by_the_copy(tmp_path):
    mib = 1024
    kib = mib * 1024.0
    # the copy reads half its size in FETCH_SIZE units and writes all of it
    fetch = [("__amd_rocclr_copyBuffer", 0.5 * kib), ("__amd_rocclr_copyBuffer", 10.0),
             ("void pv::k_verify_scan(...)", 9999.0), ("void pv::k_verify_scan(...)", 100.0),
             ("void pv::k_verify_scan(...)", 300.0),
             ("void pv::k_verify_trace<true>(...)", 7777.0), ("void pv::k_verify_trace<true>(...)", 50.0),
             ("void pv::k_verify_trace<true>(...)", 50.0),
             ("void pv::k_retrace<true, 4>(...)", 123456.0)]   # not part of the call
    write = [("__amd_rocclr_copyBuffer", kib), ("void pv::k_verify_scan(...)", 5.0),
             ("void pv::k_verify_scan(...)", 20.0), ("void pv::k_verify_scan(...)", 40.0)]
    _write(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "w"), "WRITE_SIZE", write)
    rec = T.summarize(str(tmp_path / "f"), str(tmp_path / "w"), mib)
    assert rec["copy_scale_fetch"] == pytest.approx(0.5)
    assert rec["copy_scale_write"] == pytest.approx(1.0)
    # first launch of each kernel dropped: scan (100 + 300) / 2, trace 50 KiB
    assert rec["fetch_bytes_per_launch"] == pytest.approx((200.0 + 50.0) * 1024 / 0.5)
    assert rec["write_bytes_per_launch"] == pytest.approx(30.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
    assert rec["sources_sha1"] == T.sources_sha1()


def test_source_hash_ignores_comments():
    code = "int f(int x) { return x + 1; }\n"
    commented = "// adds one\nint f(int x) { /* the argument */ return x + 1; }  // done\n\n"
    assert T._code_only(code) == T._code_only(commented)
    assert T._code_only(code) != T._code_only(code.replace("+ 1", "+ 2"))
