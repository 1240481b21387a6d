"""CPU checks of the benchmark's host-side contract: a multi-GPU request is
refused with a message, the byte model matches the per-site record sizes, and
the committed traffic record parses."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_model_matches_record_sizes():
    V = 48 * 48 * 48 * 96
    # F16S: a 12-component column is 48 B of halves + a 4 B scale, a link 36 + 4 B
    assert bench.pass_bytes(V, "F16S", True) == V * (18 * 52 + 3 * 40)
    assert bench.pass_bytes(V, "F32", False) == V * (24 * 96 + 3 * 72)
    # per site-update: the strict checkerboard pass minimum per updated site and column
    assert bench.pass_bytes(V, "F16S", True) / (12 * V / 2) == pytest.approx(176.0)
    assert bench.pass_bytes(V, "F32", False) / (12 * V) == pytest.approx(210.0)
    assert bench.MODEL_BYTES_PER_SITE_UPDATE[("F16S", True)] == 124
    assert bench.MODEL_BYTES_PER_SITE_UPDATE[("F16S", False)] == 114


def test_traffic_record_parses_and_is_keyed_to_the_kernel():
    path = os.path.join(ROOT, "profiles", "smear_f16s_48c96_traffic.txt")
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    assert float(rec["traffic_bytes_per_launch"]) > float(rec["write_size_bytes_per_launch"]) > 0
    assert len(rec["kernel_source_sha256"]) == 64
    mode = rec.get("launch_mode", "even_odd")
    assert mode in ("full", "even_odd")
    # the record is reported only while it matches the kernel sources
    stale = rec["kernel_source_sha256"] != bench.kernel_source_digest()
    assert (bench.measured_traffic(mode=mode) is None) == stale
    # and only for the launch shape and mode it was measured with
    shape = tuple(int(x) for x in rec["launch_shape_tuple"].split(","))
    assert len(shape) == 7
    assert (bench.measured_traffic(shape, mode) is None) == stale
    other = (shape[0] % 4 + 1,) + shape[1:]
    assert bench.measured_traffic(other, mode) is None
    assert bench.measured_traffic(shape, "even_odd" if mode == "full" else "full") is None
