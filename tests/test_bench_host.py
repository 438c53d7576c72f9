"""Host logic of bench.py: the stored counter figures (HBM bytes, VALU
instructions per particle-kernel launch) are reported only for the step
window they were averaged over and while the particle-kernel sources they
were measured on are unchanged; the `--gpus` contract (one GPU only); the
two CPU-baseline legs."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_figures_follow_the_window_and_the_source_hash(tmp_path, monkeypatch):
    """Counter figures are reported for the exact step window they were
    averaged over, and only while the kernel sources are unchanged."""
    fig = {"bytes_per_launch": 2.0e8, "valu_insts_per_launch": 3.0e7}
    rec = {"push_kernel": {"workload": "lwfa2048x256", "source_sha": bench.kernel_source_hash(),
                           "windows": {"5-25": fig}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(rec))
    (tmp_path / "paper_1912_04064_amd").symlink_to(os.path.join(ROOT, "paper_1912_04064_amd"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.push_counters("lwfa", 5, 25) == fig
    # another window, another workload, or sources changed since: no figure
    assert bench.push_counters("lwfa", 0, 1000) is None
    assert bench.push_counters("lwfa", 20, 40) is None
    assert bench.push_counters("thermal2k", 5, 25) is None
    rec["push_kernel"]["source_sha"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.push_counters("lwfa", 5, 25) is None


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


def test_cpu_model_and_baseline_fields(monkeypatch):
    """The CPU baseline reports both legs, the threads it used, nproc and the
    CPU model (a tiny workload stands in for the LWFA band here)."""
    from paper_1912_04064_amd import workloads as WL
    small = WL.thermal_2d(n=(32, 32), ppc=2, patch=(8, 8), nreg=(2, 1))
    monkeypatch.setattr(bench, "workload", lambda name: small)
    monkeypatch.setenv("OMP_NUM_THREADS", "2")
    out = bench.cpu_baseline("thermal_small", budget_s=0.2)
    assert out["cores"] == 2 and out["single_core"]["cores"] == 1
    assert out["value"] > 0 and out["single_core"]["value"] > 0
    assert out["nproc"] >= 1 and isinstance(out["cpu_model"], str) and out["kind"] == "oracle"
