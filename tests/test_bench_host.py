"""Host-side logic of bench.py (no GPU): the traffic figures it reads from profiles/ and their
gating on the kernel source, the HBM fraction, and the refusal of more than one GPU."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(tmp_path, src_text, sha=None, value="1.25e+09"):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "src").mkdir(exist_ok=True)
    (tmp_path / "src" / "k.hip").write_text(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    (tmp_path / "profiles" / "k_traffic.md").write_text(
        f"# summary\n\ntraffic_bytes_per_launch: {value}\nsource: src/k.hip\n"
        f"source_sha256: {digest}\n")


def test_traffic_read_while_the_source_is_unchanged(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "kernel text\n")
    assert bench.read_traffic("k_traffic.md") == pytest.approx(1.25e9)


def test_traffic_dropped_once_the_source_changes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "kernel text\n", sha=hashlib.sha256(b"older kernel text\n").hexdigest())
    assert bench.read_traffic("k_traffic.md") is None


def test_traffic_missing_summary_or_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("absent.md") is None
    _summary(tmp_path, "kernel text\n")
    os.remove(tmp_path / "src" / "k.hip")
    assert bench.read_traffic("k_traffic.md") is None


def test_committed_summaries_match_their_sources():
    # the summaries the bench line reads name their kernel source and its hash
    for name in ("k_nt_xtg_cfg4_traffic.md", "k_nt_xv_cfg4_traffic.md",
                 "k_nt3_xtg_cfg4_traffic.md", "k_nt3_xv_cfg4_traffic.md"):
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        assert "traffic_bytes_per_launch:" in txt and "source_sha256:" in txt, name


def test_hbm_fraction():
    # 8 GB in 4 ms is 2 TB/s, a quarter of the 8 TB/s peak
    assert bench.hbm_frac(8.0e9, 4000.0) == pytest.approx(0.25)
    assert bench.hbm_frac(None, 4000.0) is None
    assert bench.hbm_frac(8.0e9, 0.0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
