"""bench.py's command-line contract on the host (no GPU needed): a run on
more than one GPU is refused with a message before anything touches a GPU,
and the committed counter summaries are read only while they describe the
current kernel sources."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_stale_counter_summary_is_ignored(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    (tmp_path / "profiles").mkdir()
    stem = "k_probe_counters"
    (tmp_path / "profiles" / (stem + ".txt")).write_text(
        "kernel_source_sha256 = 0000\nhbm_bytes_per_launch = 123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0000")
    assert bench.profile_values(stem)["hbm_bytes_per_launch"] == "123"
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "1111")
    assert bench.profile_values(stem) == {}
    assert bench.profile_values("absent") == {}
