"""deconv_admm_run_static (no device allocation: its workspace is the
library's static device array) against deconv_admm_run on a plan with its own
workspace: two calls in a row, the second with a smaller batch, must give the
same x, ytilde and statistics bit for bit (same kernels, same tiles); a batch
too large for the array is refused."""
import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import desc, device_inputs, log

pytestmark = pytest.mark.gpu

OPTS = dict(schedule=3, check_every=10)


def _compare(probs, iters, **extra):
    import torch
    from paper_1602_01410_amd import binding
    opts = dict(OPTS, **extra)
    images = [desc(p) for p in probs]
    y, mask, h, lam, mu = device_inputs(probs)
    plan = binding.Plan(images, **opts)
    yt_ref = torch.empty_like(y)
    x_ref, st_ref = plan.run(y, mask, h, lam, mu, iters, ytilde_out=yt_ref, stats=True)
    torch.cuda.synchronize()
    plan.close()
    x = torch.full_like(y, float("nan"))
    yt = torch.full_like(y, float("nan"))
    x, st = binding.run_static(images, y, mask, h, lam, mu, iters, x_out=x, ytilde_out=yt, stats=True, **opts)
    torch.cuda.synchronize()
    log("  %d images, %d px: max |dx| %.3e" % (len(probs), y.numel(), float((x - x_ref).abs().max())))
    assert torch.equal(x, x_ref)
    assert torch.equal(yt, yt_ref)
    for a, b in zip(st, st_ref):
        assert a == b, (a, b)


def test_static_run_matches_plan_run_twice():
    big = [synth.problem(256, 256, 9, "rect", "gauss", sigma=1.5, mask_kind=synth.MASK_DECIMATE, decim=4,
                         bsnr=40.0, lam=1e-3, mu=0.05, seed=71),
           synth.problem(192, 288, 7, "rect", "box", mask_kind=synth.MASK_EXPLICIT, missing=0.3, bsnr=45.0,
                         lam=2e-3, mu=0.1, seed=72),
           synth.problem(512, 512, 11, "grf", "gauss", sigma=2.0, bsnr=50.0, lam=5e-4, mu=0.02, seed=73)]
    small = [synth.config_plain_72()]
    log("first call: 3 images")
    _compare(big, 30)
    log("second call: one 72^2 image (whole-image-in-LDS path)")
    _compare(small, 25)
    log("third call: the same on the two-pass kernels")
    _compare(small, 25, small_images=0)


def test_static_run_refuses_a_batch_beyond_the_array():
    import torch
    from paper_1602_01410_amd import binding
    images = [dict(height=2048, width=2048, ksize=9)]
    assert binding.workspace_size(images) > 64 << 20
    n = 2048 * 2048
    y = torch.zeros(n, device="cuda")
    h = torch.full((81,), 1.0 / 81, device="cuda")
    lam = torch.full((1,), 1e-3, device="cuda")
    mu = torch.full((1,), 0.05, device="cuda")
    with pytest.raises(binding.DeconvError) as e:
        binding.run_static(images, y, None, h, lam, mu, 5, torch.empty_like(y))
    assert e.value.code == 7
    # with checkpoints (a reverse pass needs a plan that outlives the call)
    with pytest.raises(binding.DeconvError) as e:
        binding.run_static([dict(height=64, width=64, ksize=5)], y[:4096], None, h[:25], lam, mu, 5,
                           torch.empty_like(y[:4096]), ckpt_every=5, max_iters=5)
    assert e.value.code == 1
