"""Host logic of bench.py (no GPU): the one-GPU guard and the gating of the
roofline object's HBM traffic on the kernel sources the counters were taken
from."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def _fake_tree(root, src: str):
    csrc = os.path.join(root, "paper_2512_11800_amd", "csrc")
    os.makedirs(csrc, exist_ok=True)
    with open(os.path.join(csrc, "render.hip"), "w") as f:
        f.write(src)
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)


def test_traffic_is_read_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    root = str(tmp_path)
    monkeypatch.setattr(bench, "ROOT", root)
    _fake_tree(root, "// kernel version 1\n")
    sha = bench._kernel_source_sha()
    with open(os.path.join(root, "profiles", "render_w2_k4_counters.md"), "w") as f:
        f.write("# counters\n\n"
                f"    source_sha256: {sha}\n"
                "    traffic_bytes[mb::k_render_fwd<4, 4, 0>]: 1174119554\n"
                "    traffic_bytes[mb::k_render_bwd<4, 4, 0>]: 1746778569\n")
    assert bench._measured_traffic("mb::k_render_fwd<4, 4, 0>") == 1174119554.0
    assert bench._measured_traffic("mb::k_render_bwd<4, 4, 0>") == 1746778569.0
    assert bench._measured_traffic("mb::k_render_bwd<6, 4, 0>") is None  # not measured
    # a kernel edited after the counters were taken: the figures no longer apply
    _fake_tree(root, "// kernel version 2\n")
    assert bench._kernel_source_sha() != sha
    assert bench._measured_traffic("mb::k_render_fwd<4, 4, 0>") is None


def test_traffic_without_a_profile_is_null(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_tree(str(tmp_path), "// kernel\n")
    assert bench._measured_traffic("mb::k_render_fwd<4, 4, 0>") is None
