"""Host-side behaviour of bench.py (CPU only): more than one GPU is refused
with a message, and the measured-traffic figure is reported only for the
stage-kernel sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    import hashlib
    got = bench.measured_traffic()
    h = hashlib.sha256()
    for s in bench.STAGE_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    text = open(bench.TRAFFIC_SUMMARY).read()
    # a figure exactly when the summary was taken on these sources
    assert (got is not None and got > 0) == (h.hexdigest() in text)
    # a summary taken on other sources gives no figure
    at = text.index("`", text.index("sha256 over")) + 1
    other = tmp_path / "summary.md"
    other.write_text(text[:at] + "0" * 64 + text[at + 64:])
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(other))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
