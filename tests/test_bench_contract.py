"""bench.py's host side, on the CPU: the one-GPU rule and the algorithmic
byte counts its bandwidth figures divide by."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_ee_step_bytes_counts_each_vector_once():
    """A step of Krylov dimension j = 2 (m_max = 30) at N points, FP32 basis
    (w = 4), written out vector by vector: matvec 0 reads u_0, y32 and writes
    w; matvec 1 reads u_1, y32, q_0, writes w; matvec 2 reads u_2, y32, q_0,
    q_1, writes w; update 0 reads u_0, w, writes q_0, u_1; update 1 reads q_0,
    u_1, w, writes q_1, u_2; the solution update reads y (8) and 2 columns and
    writes y (8); the estimate reads 3 FP64 fields, writes f (8) and v_1 (4)
    and the FP32 copy of y (4)."""
    N, w = 1000, 4
    matvecs = (3 + 4 + 5) * w
    updates = (4 + 5) * w
    solution = 8 + 2 * w + 8
    estimate = 3 * 8 + 8 + w + 4
    assert bench.ee_step_bytes(2, 30, w, N, True) == N * (matvecs + updates + solution + estimate)
    # at j = m_max the last matvec stores no w
    assert bench.ee_step_bytes(30, 30, w, N, True) - bench.ee_step_bytes(29, 30, w, N, True) == N * (
        (30 + 2) * w + (29 + 4) * w + w)


def test_traffic_is_used_only_for_the_same_replay(tmp_path, monkeypatch):
    """The counter-measured traffic is attached to the roofline only when it
    was taken on the current kernel sources and on a replay of the same
    algorithmic bytes per launch."""
    f = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    sha = bench.kernel_source_sha()
    f.write_text(f"source_sha: {sha}\nreplay_bytes_per_launch: 1000000\ntraffic_bytes_per_launch: 1013000\n")
    assert bench.measured_traffic(1000000.0) == 1013000.0
    assert bench.measured_traffic(1000500.0) == 1013000.0
    assert bench.measured_traffic(1002000.0) is None
    f.write_text("source_sha: 0000\nreplay_bytes_per_launch: 1000000\ntraffic_bytes_per_launch: 1013000\n")
    assert bench.measured_traffic(1000000.0) is None
