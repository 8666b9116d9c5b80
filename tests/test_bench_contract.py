"""Host-side parts of bench.py that need no GPU: the refusal of several GPUs,
and the hardware-counter record it reads for the roofline's traffic figure
(the record is used only while the kernel sources are the ones it was
measured on)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)


def test_traffic_record_is_well_formed():
    rec = {}
    with open(os.path.join(ROOT, bench.TRAFFIC_RECORD)) as f:
        for line in f:
            k, _, v = line.strip().partition(": ")
            rec[k] = v
    assert len(rec["kernel_source_sha256"]) == 64
    traffic = int(rec["traffic_bytes_per_launch"])
    # each distribution read once and written once: 2 x 19 x 4 B x 256 x 128 x 128
    algorithmic = 2 * 19 * 4 * 256 * 128 * 128
    assert algorithmic <= traffic < 1.1 * algorithmic


def test_traffic_follows_the_kernel_sources(monkeypatch):
    t = bench.measured_traffic()
    assert t is None or isinstance(t, int)
    # a different source hash disables the record
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic() is None
