"""Host logic of the benchmark script, on the CPU: the algorithmic byte
count per site, the lookup of the committed counter traffic (taken only when
the kernel sources are the profiled ones), and the refusal of more than one
GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    import bench
    return bench


def test_bytes_per_site(bench):
    # two lattices: 19 populations read and written, 18 int32 pull indices
    assert bench.bytes_per_site("f64") == 2 * 19 * 8 + 18 * 4 == 376
    assert bench.bytes_per_site("f32") == 224
    assert bench.bytes_per_site("f16") == 148
    # in place: half the index reads on average over an even and an odd sweep
    assert bench.bytes_per_site("f16", aa=True) == 2 * 19 * 2 + 9 * 4 == 112
    # int16 deltas halve the index bytes of the near fraction
    assert bench.bytes_per_site("f32", near=1.0) == 2 * 19 * 4 + 18 * 2
    assert bench.bytes_per_site("f32", near=0.8119) == pytest.approx(152 + 18 * (0.8119 * 2 + 0.1881 * 4))
    assert bench.bytes_per_site("f16sr", aa=True, near=0.5) == 76 + 9 * 3


def test_source_hash_ignores_comments_only(bench):
    def reader(extra):
        def read(name):
            with open(os.path.join(ROOT, "paper_2010_04144_amd", "csrc", name)) as fh:
                return fh.read() + extra
        return read
    base = bench.kernel_source_hash()
    assert bench.kernel_source_hash(reader("\n// a note\n/* block\n note */\n\n")) == base
    assert bench.kernel_source_hash(reader("\nstatic int unused_marker;\n")) != base


def test_traffic_lookup(bench, monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic_branching_artery.json")) as fh:
        summary = json.load(fh)
    entry = summary["entries"][0]
    key = (entry["prec"], entry["layout_flags"], entry["block"], entry["sched_flags"])
    # taken from the committed summary when it was made from these kernel sources
    monkeypatch.setattr(bench, "kernel_source_hash", lambda read=None: summary["kernel_source_sha256_16"])
    assert bench.traffic_from_profile(*key) == entry["bytes_per_launch"]
    assert bench.traffic_from_profile(key[0], key[1], key[2], 12345) is None
    # and never once the kernels have changed
    monkeypatch.setattr(bench, "kernel_source_hash", lambda read=None: "0000000000000000")
    assert bench.traffic_from_profile(*key) is None


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_relative_error_and_its_record(bench):
    """The parity metric: the largest deviation over the largest signal, or
    over the floor when the signal is smaller; the record keeps the absolute
    deviation and the signal size, so a ratio held up by the floor shows."""
    import numpy as np
    a = np.array([1.0, 2.0, 3.0])
    b = np.array([1.0, 2.5, 3.0])
    rec = {}
    assert bench.rel_err(a, b, b, 0.0, rec, "x") == pytest.approx(0.5 / 3.0)
    assert rec["x"] == {"abs": 0.5, "signal": 3.0, "floor": 0.0}
    small = np.array([1e-9, -2e-9])
    assert bench.rel_err(small, small + 1e-18, small, 1e-4, rec, "y") == pytest.approx(1e-14)
    assert rec["y"]["signal"] == pytest.approx(2e-9) and rec["y"]["floor"] == 1e-4
    assert bench.rel_err(np.zeros(2), np.full(2, 3e-17), np.zeros(2)) == pytest.approx(3e-17)
