"""Host-side parts of the benchmark script: the one-GPU limit, the
algorithmic byte counts the roofline is computed from, and when the stored
counter summary may supply its measured traffic."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_cell():
    """Phase V at 32 levels, FP64: 14 words read (M 3, theta_L, Gamma, rho,
    rho theta, W, p*, S_W, H_rho, H_rth, rho[t], p[t]) and 5 written (rho,
    rho theta, W, p*, D) = 152 B, plus 6 ids and 21 coefficients per column
    over 32 levels = 6 B.  Phase M: 11 words (M in and out, S_M, p*, D) = 88
    B plus 720 B of geometry per column = 22.5 B.  In the mixed form the
    horizontal words are 4 B."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.vert_bytes_per_cell(32, False) == 158.0
    assert bench.hmom_bytes_per_cell(32, False) == 110.5
    # mixed: 8-byte rho, rho theta, W, S_W, rho[t], p[t]; 4-byte M, theta_L,
    # Gamma, p*, H_rho, H_rth; writes 3 x 8 + 2 x 4; geometry in 4 bytes
    assert bench.vert_bytes_per_cell(32, True) == 6 * 8 + 8 * 4 + 3 * 8 + 2 * 4 + (6 * 4 + 21 * 4) / 32
    assert bench.hmom_bytes_per_cell(32, True) == 11 * 4 + (6 * 4 + 21 * 4 + 3 * 4 + 18 * 4 + 54 * 4) / 32


def test_counter_traffic_only_for_the_kernels_it_was_taken_on(tmp_path, monkeypatch):
    """The roofline's measured HBM bytes come from a stored counter summary
    that names the SHA-256 of the kernel source; any other source gives
    null, and so does a missing or unreadable summary."""
    import hashlib
    import json
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "paper_1607_05535_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src / "kernels.hip").write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(b"// kernel source\n").hexdigest()
    summary = tmp_path / "profiles" / "vert_g6L32_counters.json"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic() is None
    summary.write_text(json.dumps({"hbm_bytes_per_launch": 123.0, "kernels_hip_sha256": sha}))
    assert bench.counter_traffic() == 123.0
    (src / "kernels.hip").write_bytes(b"// changed\n")
    assert bench.counter_traffic() is None
    summary.write_text("not json")
    assert bench.counter_traffic() is None
