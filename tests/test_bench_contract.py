"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

import pytest


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_figures_follow_the_kernel_source(tmp_path, monkeypatch):
    """Traffic and counter figures are reported only while the forward
    kernel source is the one they were measured on."""
    sys.path.insert(0, ROOT)
    import bench
    fig = bench.profile_figures()
    if not fig:  # allowed: bench.py then reports traffic as null
        pytest.skip("the committed counters predate the current kernel source")
    assert fig["traffic"] > 0 and fig["counter_flop"] > 0
    # a copy of the tree whose kernel source differs: no figures
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1201_2450_amd" / "csrc").mkdir(parents=True)
    with open(os.path.join(ROOT, "profiles", "jacobi_enh256_traffic.txt")) as fh:
        (tmp_path / "profiles" / "jacobi_enh256_traffic.txt").write_text(fh.read())
    with open(os.path.join(ROOT, "paper_1201_2450_amd", "csrc", "tiled_fwd.hip")) as fh:
        (tmp_path / "paper_1201_2450_amd" / "csrc" / "tiled_fwd.hip").write_text(fh.read() + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_figures() == {}
