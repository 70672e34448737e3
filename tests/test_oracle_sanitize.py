"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: an
instrumented build of oracle.c runs a cross-section of the CPU pins (FFTs of
power-of-two and Bluestein lengths, the PSF embedding, convolutions, the
initial state, the iteration with every option, the colour variant, the
objective and the reverse mode) in a child process; any out-of-bounds access,
use after free or undefined operation aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import numpy as np
import oracle
from paper_1602_01410_amd import synth
rng = np.random.default_rng(0)
for n in (1, 2, 3, 8, 12, 18, 72, 96, 100):
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.allclose(oracle.fft1(x), np.fft.fft(x))
for M, N in ((8, 12), (9, 6)):
    x = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    assert np.allclose(oracle.fft2(x), np.fft.fft2(x))
    assert np.allclose(oracle.dft2_direct(x), np.fft.fft2(x))
for kind, kw in ((synth.MASK_BOUNDARY, {}), (synth.MASK_EXPLICIT, dict(missing=0.3)),
                 (synth.MASK_DECIMATE, dict(decim=3))):
    p = synth.problem(18, 24, 5, "rect", "random", mask_kind=kind, bsnr=40.0, lam=1e-2, mu=0.05, seed=3,
                      nrect=4, **kw)
    y, m, h = p["y"].astype(float), p["mask"].astype(np.uint8), p["h"].astype(float)
    oracle.psf_spectrum(18, 24, h)
    a = oracle.conv_direct(h, y)
    b = oracle.conv_fft(h, y)
    assert np.allclose(a, b)
    oracle.conv_fft(h, y, adjoint=True)
    oracle.gradT(*oracle.grad(y))
    for kw2 in (dict(), dict(alpha=1.0, phi="quad"), dict(passes=3, adapt_t=3.0, warm_iters=5)):
        r = oracle.admm_run(y, m, h, 1e-2, 0.05, 6, **kw2)
        assert np.isfinite(r["x"]).all()
    oracle.objective(h, r["yt"], r["x"], 1e-2)
    gy, gl, gh = oracle.admm_backward(y, m, h, 1e-2, 0.05, 5, rng.standard_normal(y.shape))
    assert np.isfinite(gy).all() and np.isfinite(gh).all()
q = synth.rgb_problem(16, 24, 5, seed=4, bsnr=40.0, lam=1e-3, mu=0.05)
r = oracle.admm_run_vec(q["ys"].astype(float), q["masks"], q["h"].astype(float), 1e-3, 0.05, 5, passes=2,
                        adapt_t=3.0, warm_iters=3)
assert np.isfinite(r["x"]).all()
print("SANITIZED_OK")
'''


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    import oracle
    lib = oracle.build(out=str(tmp_path / "oracle_san.so"), sanitize=True)
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
