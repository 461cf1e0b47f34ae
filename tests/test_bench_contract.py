"""The benchmark's contract that holds without a GPU: more than one GPU is
refused with a message and exit status 2, before any device work; the
committed counter-traffic figure is used only for the run it was taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_traffic_is_tied_to_sources_interval_and_tile(tmp_path, monkeypatch):
    """The committed counter figure is reported only for the run it was taken
    on: the same kernel and sort sources, sort interval and tile."""
    sys.path.insert(0, ROOT)
    import bench
    digest = bench.kernel_sources_digest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    text = ("- traffic_bytes_per_launch: `123`\n- texture_addresser_busy: `0.5`\n"
            "- valu_busy: `0.25`\n- sort_every: `4`\n- tile: `16,4,4`\n"
            f"- sources_sha256: `{digest}`\n")
    (prof / "push_emit_cX_traffic.md").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_sources_digest reads the sources under ROOT: keep it on the repository
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: digest)
    assert bench.counter_traffic("cX", 4, (16, 4, 4)) == 123.0
    busy = bench.counter_busy("cX", 4, (16, 4, 4))
    assert busy["texture_addresser_busy"] == 0.5 and busy["valu_busy"] == 0.25
    assert bench.counter_traffic("cX", 10, (16, 4, 4)) is None
    assert bench.counter_busy("cX", 10, (16, 4, 4)) is None
    assert bench.counter_traffic("cX", 4, (32, 2, 2)) is None
    assert bench.counter_traffic("cY", 4, (16, 4, 4)) is None
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: "0" * 64)
    assert bench.counter_traffic("cX", 4, (16, 4, 4)) is None
