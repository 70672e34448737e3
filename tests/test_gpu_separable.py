"""Blur spectrum setup and separable blurs in the column pass.  A blur
kernel that is the outer product of two 1-D kernels enters the x-step of eq.
(dual_x_iter_resolved_boundaries) through the product of its 1-D spectra
instead of the stored 2-D spectrum: the images that take that path, and the
results of both paths against the FP64 oracle and against each other.
Kernels wider than 65 taps get their spectrum from FFTs rather than direct
sums."""
import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, gpu_run, log, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _batch(seed=71):
    """Box, Gaussian, even box on an odd support (all separable), motion and
    a Gaussian with one tap nudged by 1e-4 of its peak (not separable)."""
    probs = [synth.problem(72, 96, 9, "rect", "box", bsnr=50.0, lam=1e-3, mu=0.05, seed=seed),
             synth.problem(128, 128, 11, "rect", "gauss", sigma=2.0, mask_kind=synth.MASK_DECIMATE, decim=2,
                           bsnr=45.0, lam=1e-3, mu=0.05, seed=seed + 1),
             synth.problem(96, 72, 15, "rect", "motion", mask_kind=synth.MASK_EXPLICIT, missing=0.3,
                           bsnr=40.0, lam=2e-3, mu=0.05, seed=seed + 2),
             synth.problem(64, 64, 7, "rect", "gauss", sigma=1.5, bsnr=50.0, lam=1e-3, mu=0.05, seed=seed + 3)]
    h = probs[3]["h"].astype(np.float64)
    h[1, 2] += 1e-4 * h.max()
    probs[3]["h"] = (h / h.sum()).astype(np.float32)
    even = synth.problem(64, 96, 5, "rect", "box", bsnr=50.0, lam=1e-3, mu=0.05, seed=seed + 4)
    he = np.zeros((5, 5))
    he[:4, :4] = 1.0 / 16.0
    even["h"] = he.astype(np.float32)
    probs.append(even)
    return probs


def test_separable_flags_and_oracle_parity():
    probs = _batch()
    iters = 60
    g = gpu_run(probs, iters)
    flags = g["plan"].separable()
    log("separable flags: %s" % (flags,))
    assert flags == (1, 1, 0, 0, 1)
    for b, p in enumerate(probs):
        r = oracle_run(p, iters)
        assert_parity(g["x"][b], r["x"], what="img%d x" % b)
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_separable_matches_stored_spectrum(use_graph):
    """Both paths on the same inputs: flags (1, 1, 0, 0, 1) against all 0;
    the results differ by rounding only, and not at all for the images that
    take the stored spectrum either way."""
    probs = _batch(seed=81)
    iters = 40
    # launch shapes and tiles fixed, so that both runs execute the same code
    kw = dict(use_graph=use_graph, check_every=10, schedule=1, row_tiles=1)
    a = gpu_run(probs, iters, **kw)
    b = gpu_run(probs, iters, separable_blur=0, **kw)
    assert b["plan"].separable() == (0, 0, 0, 0, 0)
    for k, p in enumerate(probs):
        r = rel_l2(a["x"][k], b["x"][k])
        log("img%d separable vs stored: rel_l2 %.3e" % (k, r))
        if k in (2, 3):
            assert np.array_equal(a["x"][k], b["x"][k])
        else:
            assert r <= 1e-5


def test_wide_kernel_takes_fft_setup():
    """Kernels wider than 65 taps get their spectrum from 2-D FFTs instead of
    the direct sums (and never the separable path): the spectrum against the
    oracle, then a run against the oracle."""
    import torch
    import oracle
    from paper_1602_01410_amd import binding
    kernels = [synth.gaussian_kernel(67, 9.0), synth.box_kernel(5)]
    plan = binding.Plan([dict(height=192, width=256, ksize=k.shape[0]) for k in kernels])
    h = torch.from_numpy(np.concatenate([k.astype(np.float32).ravel() for k in kernels])).cuda()
    spec = plan.blur_spectrum(h).cpu().numpy().view(np.complex64).reshape(len(kernels), 192, 256)
    for k, s in zip(kernels, spec):
        ref = oracle.psf_spectrum(192, 256, k.astype(np.float32).astype(np.float64))
        r = rel_l2(s, ref)
        log("ksize %d spectrum rel_l2 %.3e" % (k.shape[0], r))
        assert r <= 1e-6
    p = synth.problem(192, 256, 67, "rect", "gauss", sigma=9.0, bsnr=50.0, lam=1e-3, mu=0.05, seed=91)
    g = gpu_run([p], 30)
    assert g["plan"].separable() == (0,)
    r = oracle_run(p, 30)
    assert_parity(g["x"][0], r["x"], what="ksize 67 x")
    assert_parity(g["yt"][0], r["yt"], what="ksize 67 ytilde")
