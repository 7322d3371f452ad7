"""Host logic of bench.py: the key that ties the committed HBM traffic counters to the kernel
code, the scaling of those counters to a run's sample count, and the one-GPU guard."""

import json
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ("kernels.hip", "device_common.h", "hb_internal.h")


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the hashed kernel sources under a temporary root that bench.py reads."""
    src = tmp_path / "paper_1504_02687_amd" / "csrc"
    src.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_1504_02687_amd", "csrc", f), src / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def _edit(path, fn):
    text = path.read_text(encoding="utf-8")
    path.write_text(fn(text), encoding="utf-8")


def test_source_hash_ignores_comments_and_layout(tree):
    h0 = bench.kernel_source_hash()
    assert h0 == bench.kernel_source_hash() and len(h0) == 16
    k = tree / "paper_1504_02687_amd" / "csrc" / "kernels.hip"
    _edit(k, lambda t: "// a new comment line\n/* and a block\n   comment */\n" + t.replace("\n", "\n\n", 5))
    assert bench.kernel_source_hash() == h0
    _edit(k, lambda t: t.replace("constexpr int kBinChunks = 8;", "constexpr int kBinChunks = 4;"))
    assert bench.kernel_source_hash() != h0


def test_source_hash_keeps_string_literals(tree):
    h0 = bench.kernel_source_hash()
    h = tree / "paper_1504_02687_amd" / "csrc" / "hb_internal.h"
    # a comment marker inside a string literal is code, not a comment
    _edit(h, lambda t: t + '\nstatic const char *kProbe = "a // b";\n')
    h1 = bench.kernel_source_hash()
    _edit(h, lambda t: t.replace('"a // b"', '"a // c"'))
    assert len({h0, h1, bench.kernel_source_hash()}) == 3


def test_traffic_scales_with_samples_and_needs_the_same_code(tree):
    path = tree / "profiles" / "hbm_traffic.json"
    path.write_text(json.dumps({
        "kernel_source_hash": bench.kernel_source_hash(),
        "points_per_launch": 2.0e9,
        "kernels": {"k_advect_smooth": {"bytes_per_launch": 40.0e9}},
    }))
    names = {"advect_smooth": "k_advect_smooth"}
    assert bench.traffic_for("advect_smooth", names, [1.0e9, 3.0e9]) == pytest.approx(40.0e9)
    assert bench.traffic_for("advect_smooth", names, [1.0e9]) == pytest.approx(20.0e9)
    assert bench.traffic_for("resample_splat", {"resample_splat": "k_resample_count"}, [1.0e9]) is None
    _edit(tree / "paper_1504_02687_amd" / "csrc" / "kernels.hip", lambda t: t + "\nint kChanged;\n")
    assert bench.traffic_for("advect_smooth", names, [1.0e9]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
