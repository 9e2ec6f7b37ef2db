"""Host-side parts of bench.py: the one-GPU contract, the roofline's
operation counts and the committed traffic record's parser (no GPU)."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_unit_counts(bench):
    # 940 operations per neighbour entry with the limiter, 690 without
    assert bench.flux_flops_unit(2_500_000, 59_963_063, 1) == 940 * 59_963_063
    assert bench.flux_flops_unit(1000, 24_000, 0) == 690 * 24_000


def test_itemised_count_by_hand(bench):
    # three points: interior 0 (entries in s+ and n-, and in s- only),
    # wall 1 (its n+ membership dropped), outer 2 (no residual)
    kind = np.array([0, 1, 2], np.uint8)
    ptr = np.array([0, 2, 3, 4])
    flags = np.array([1 | 8, 2, 4, 1 | 4], np.uint8)
    common = bench.FLOPS_ENTRY_COMMON + bench.FLOPS_ENTRY_LIMITER
    # entries used: 0 (2 stencils), 1 (1), 2 (wall: n+ dropped, none) -> 2 entries, 3 stencils
    want = 2 * common + 3 * bench.FLOPS_PER_STENCIL
    assert bench.flux_flops_per_launch(flags, kind, ptr, 1) == want


def test_traffic_record_parser(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    sha = hashlib.sha256(b"kernel source").hexdigest()
    rec = tmp_path / "rec.md"
    line = {"kernel": "k", "fetch_kib": 10.0, "write_kib": 4.0, "fetch_scale": 2.0,
            "write_scale": 1.0, "sources_sha256": sha}
    rec.write_text("# summary\n\nrecord: " + json.dumps(line) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", {"w": str(rec)})
    assert bench.committed_traffic("w") == 10.0 * 1024 * 2.0 + 4.0 * 1024
    # another source text: the counters no longer describe the kernel
    src.write_text("changed")
    assert bench.committed_traffic("w") is None
    assert bench.committed_traffic("missing") is None
