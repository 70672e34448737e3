"""Host-side pieces of bench.py: the one-GPU guard and the algorithmic byte
model of each pass (the figures behind the roofline fraction)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_alg_bytes_per_pass():
    import bench
    # one 1024^2 image: row pass 32 B per half-spectrum entry (in + out) and
    # 20 B per pixel (ytilde, d in, d out), plus z out on unobserved pixels;
    # column pass 40 B per half-spectrum entry
    probs = [dict(M=1024, N=1024)]
    row, col = bench.alg_bytes(probs, 0.25)
    nh = 513
    assert row == 1024 * nh * 32 + 1024 * 1024 * 20 + 4 * 0.25 * 1024 * 1024
    assert col == 1024 * nh * 40
    # additive over images; odd half widths
    row2, col2 = bench.alg_bytes(probs + [dict(M=96, N=72)], 0.0)
    assert col2 == col + 96 * 37 * 40
    assert row2 == 1024 * nh * 32 + 1024 * 1024 * 20 + 96 * 37 * 32 + 96 * 72 * 20


def test_src_hash_covers_the_kernel_sources():
    import bench
    h = bench.src_hash()
    assert len(h) == 16 and h == bench.src_hash()
