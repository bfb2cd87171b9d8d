"""Host-side checks of bench.py (no GPU): the one-GPU guard, the argument defaults of the legs,
and the counter record that feeds the roofline's traffic field."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_record_applies_only_to_its_kernel_and_sources():
    assert bench.counter_record("k_hops_fx<64, 1, 0, 16>") is None
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    for key in ("kernel", "kernel_hash", "bytes_per_launch", "read_bytes", "write_bytes", "valu_insts_per_hop",
                "lds_insts_per_hop"):
        assert key in rec, key
    assert rec["bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    # a record taken on other sources is not used
    if rec["kernel_hash"] == bench.kernel_hash():
        assert bench.measured_traffic(rec["kernel"].replace("void cg::", "")) == rec["bytes_per_launch"]
    else:
        assert bench.measured_traffic(rec["kernel"].replace("void cg::", "")) is None


def test_kernel_hash_covers_the_hop_kernel_sources():
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert all(os.path.exists(p) for p in bench.KERNEL_SRCS)
