"""Host logic of bench.py, on the CPU: the one-GPU guard, the HBM traffic
figure built from two counter runs scaled by a copy of known size, and the
source hash that keeps a stored figure from outliving the kernel it measured."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _counters(d, counter, rows):
    """rows: (dispatch, kernel name, KiB); one dispatch may have several rows
    (one per counter instance), which the reader adds up."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, kib in rows:
            w.writerow(dict(Dispatch_Id=disp, Kernel_Name=name, Counter_Name=counter,
                            Counter_Value=kib))


@pytest.fixture(scope="module")
def bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_is_scaled_by_the_copy_probe(bench, tmp_path):
    kern = "void bdfx::k_integrate<21, float, 4, 1, 1, true, false, 0, false>(bdfx::Params)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy of 1 MiB reads as 512 KiB (factor 2) and writes as 1024 KiB (factor 1)
    _counters(tmp_path / "F", "FETCH_SIZE",
              [(1, "fill", 3.0), (2, copy, 512.0), (7, kern, 600.0), (7, kern, 400.0)])
    _counters(tmp_path / "W", "WRITE_SIZE", [(2, copy, 1024.0), (7, kern, 300.0)])
    out = tmp_path / "traffic.json"
    doc = bench.traffic_from(str(tmp_path / "F"), str(tmp_path / "W"), 1.0, "wl", "form",
                             out=str(out))
    assert doc["fetch"]["scale"] == 2.0 and doc["write"]["scale"] == 1.0
    assert doc["fetch"]["bytes"] == 1000.0 * 2.0 * 1024.0
    assert doc["traffic_bytes"] == (2000.0 + 300.0) * 1024.0
    assert json.loads(out.read_text()) == doc
    assert doc["source_hash"] == bench.kernel_source_hash()


def test_stored_traffic_needs_the_same_sources(bench, tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    doc = dict(workload="wl", form="form", source_hash=bench.kernel_source_hash(),
               traffic_bytes=123.0)
    f.write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("wl", "form") == 123.0
    assert bench.stored_traffic("other", "form") is None
    assert bench.stored_traffic("wl", "other") is None
    f.write_text(json.dumps(dict(doc, source_hash="0" * 16)))
    assert bench.stored_traffic("wl", "form") is None
    f.write_text("not json")
    assert bench.stored_traffic("wl", "form") is None
