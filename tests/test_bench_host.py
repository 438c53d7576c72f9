"""Host logic of bench.py: the stored counter figures (HBM bytes, VALU
instructions per particle-kernel launch) are reported only while the
particle-kernel sources they were measured on are unchanged, and the
`--gpus` contract (one GPU only)."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_figures_follow_the_source_hash(tmp_path, monkeypatch):
    rec = {"push_kernel": {"workload": "lwfa2048x256", "source_sha": bench.kernel_source_hash(),
                           "bytes_per_launch": 2.0e8, "valu_insts_per_launch": 3.0e7}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(rec))
    (tmp_path / "paper_1912_04064_amd").symlink_to(os.path.join(ROOT, "paper_1912_04064_amd"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.push_traffic("lwfa") == 2.0e8
    assert bench.push_valu("lwfa") == 3.0e7
    # another workload, or sources changed since the counters: no figure
    assert bench.push_traffic("thermal2k") is None
    assert bench.push_valu("cyl3d") is None
    rec["push_kernel"]["source_sha"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.push_traffic("lwfa") is None
    assert bench.push_valu("lwfa") is None


def test_valu_line():
    assert bench.valu_line(None, 0.08) is None
    v = bench.valu_line(6.144e7, 0.1)   # 6.144e7 instructions in 100 us
    assert v["achieved"] == pytest.approx(6.144e11)
    assert v["frac"] == pytest.approx(1.0)
    assert v["peak"] == pytest.approx(256 * 2.4e9)


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1912_04064_amd", "csrc")
    dst = tmp_path / "paper_1912_04064_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("k_push.hip", "part.h", "sdmd_dev.h"):
        (dst / f).write_text(open(os.path.join(src, f)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    p = dst / "k_push.hip"
    p.write_text(p.read_text() + "\n// a comment\n/* another */\n")
    assert bench.kernel_source_hash() == h0
    p.write_text(p.read_text() + "\nstatic int changed_code;\n")
    assert bench.kernel_source_hash() != h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
