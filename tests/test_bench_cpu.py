"""Host logic of bench.py (no GPU): the --gpus guard and the lookup of the
dominant kernel's measured HBM traffic, which is reported only for the
workload the counters were taken on and while the kernel sources still hash
to the recorded value."""
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ("solver_kernels.hip", "internal.h")


K = "k_cg_spmv_sym"


def _fake_root(tmp_path, workload, sha=None, bytes_=123456789):
    csrc = tmp_path / "paper_2107_11541_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for name in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2107_11541_amd", "csrc", name), csrc / name)
        h.update((csrc / name).read_bytes())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / f"{K}_{workload}.md").write_text(
        f"# summary\n\n    traffic_kernel: {K}\n"
        f"    traffic_workload: {workload}\n    traffic_bytes_per_launch: {bytes_}\n"
        f"    source_sha256: {sha or h.hexdigest()}\n")
    return tmp_path


def test_traffic_read_for_its_workload(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(_fake_root(tmp_path, "hex128")))
    assert bench.measured_traffic("hex128", K) == 123456789.0
    assert bench.measured_traffic("hybrid128", K) is None     # no summary for it
    assert bench.measured_traffic("hex128", "k_cg_spmv_pq") is None     # nor for the other kernel


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    root = _fake_root(tmp_path, "hybrid128")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("hybrid128", K) == 123456789.0
    with open(root / "paper_2107_11541_amd" / "csrc" / "internal.h", "a") as fh:
        fh.write("\n// edited\n")
    assert bench.measured_traffic("hybrid128", K) is None


def test_traffic_dropped_for_another_workload_or_hash(tmp_path, monkeypatch):
    root = _fake_root(tmp_path, "hex128", sha="0" * 64)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("hex128", K) is None
    (root / "profiles" / f"{K}_tet128.md").write_text((root / "profiles" / f"{K}_hex128.md").read_text())
    assert bench.measured_traffic("tet128", K) is None     # records another workload


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_committed_traffic_summaries_name_their_workload():
    # each committed SpMV summary records the workload in its file name, a
    # positive byte count and a full hash
    import glob
    import re
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_cg_spmv_*_*.md")))
    assert paths
    for p in paths:
        kern, wl = re.match(r"(k_cg_spmv_(?:sym|pq))_(.+)\.md$", os.path.basename(p)).groups()
        kv = dict(ln.strip().split(": ", 1) for ln in open(p) if re.match(r"\s+(traffic_\w+|source_sha256): ", ln))
        assert kv["traffic_workload"] == wl and kv["traffic_kernel"] == kern
        assert float(kv["traffic_bytes_per_launch"]) > 0
        assert re.fullmatch(r"[0-9a-f]{64}", kv["source_sha256"])
