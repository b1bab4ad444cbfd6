"""Host-side checks of bench.py's bookkeeping (no GPU): the HBM traffic it
reports comes from the committed counter summary only while the integration
kernel's source is the one those counters were taken on, and a run on more
than one GPU is refused with a message."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def summary():
    return open(os.path.join(ROOT, "profiles", "rollout_fp64_1M_hbm_traffic.md")).read()


def test_traffic_follows_the_committed_kernel_source():
    """The summary's figure while the source hash matches, else none."""
    txt = summary()
    src = txt.split("kernel_source: ")[1].split()[0]
    sha = txt.split("source_sha1: ")[1].split()[0]
    now = hashlib.sha1(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    want = int(txt.split("traffic_bytes_per_launch: ")[1].split()[0])
    # a plausible size: above the algorithmic bytes (93 B per sample), within HBM reach
    assert 93 * 1_048_576 < want < 2_000_000_000
    assert bench.measured_traffic() == (want if now == sha else None)


def test_traffic_is_dropped_when_the_source_differs(tmp_path, monkeypatch):
    root = tmp_path / "r"
    (root / "profiles").mkdir(parents=True)
    txt = summary()
    src = txt.split("kernel_source: ")[1].split()[0]
    (root / "profiles" / "rollout_fp64_1M_hbm_traffic.md").write_text(txt)
    (root / os.path.dirname(src)).mkdir(parents=True)
    (root / src).write_text(open(os.path.join(ROOT, src)).read() + "\n// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0
    assert "GPU" in (r.stdout + r.stderr)
