"""Failure paths and workspace hygiene on the GPU:
* NaN in one image's observed data reaches that image's residuals and is
  reported as DECONV_ERR_NONFINITE for it alone at the next check; the
  other images of the batch are bit-identical to a clean run, and a NaN at
  an unobserved pixel (whose value the method never reads) changes nothing;
* a caller workspace filled with NaN before plan creation gives outputs
  bit-identical to one filled with zeros (no kernel reads workspace memory
  it has not written in the same call), for plain runs, Proposed-AD passes
  with the adaptive penalty and warm start, and the reverse pass."""
import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import desc, device_inputs, log

pytestmark = pytest.mark.gpu


def _batch():
    return [synth.problem(96, 128, 7, "rect", "gauss", sigma=1.5, bsnr=40.0, lam=2e-3, mu=0.05, seed=901),
            synth.problem(128, 128, 9, "rect", "box", mask_kind=synth.MASK_EXPLICIT, missing=0.3, bsnr=45.0,
                          lam=1e-3, mu=0.05, seed=902),
            synth.problem(72, 72, 5, "rect", "gauss", sigma=1.0, mask_kind=synth.MASK_DECIMATE, decim=3,
                          bsnr=40.0, lam=3e-3, mu=0.1, seed=903)]


def test_nan_in_one_image_is_reported_for_it_alone():
    import torch
    from paper_1602_01410_amd import binding
    probs = _batch()
    iters, K = 20, 5
    plan = binding.Plan([desc(p) for p in probs], check_every=K)
    y, mask, h, lam, mu = device_inputs(probs)
    x_clean, st_clean = plan.run(y, mask, h, lam, mu, iters, stats=True)
    x_clean = x_clean.clone()
    assert all(s["status"] == 0 for s in st_clean)
    off = [0]
    for p in probs:
        off.append(off[-1] + p["M"] * p["N"])
    # NaN at an observed pixel of image 1, at an unobserved (band) pixel of image 2
    yb = y.clone()
    obs1 = np.flatnonzero(probs[1]["mask"].ravel())
    yb[off[1] + int(obs1[len(obs1) // 2])] = float("nan")
    yb[off[2] + 0] = float("nan")
    assert probs[2]["mask"].ravel()[0] == 0
    with pytest.raises(binding.DeconvError) as e:
        plan.run(yb, mask, h, lam, mu, iters, stats=True)
    assert e.value.code == 4
    st = e.value.stats
    log("statuses: %s" % [s["status"] for s in st])
    assert [s["status"] for s in st] == [0, 4, 0]
    # the first check after the NaN entered already saw it
    x_bad = torch.empty_like(y)
    with pytest.raises(binding.DeconvError) as e:
        plan.run(yb, mask, h, lam, mu, K, x_out=x_bad, stats=True)
    assert [s["status"] for s in e.value.stats] == [0, 4, 0]
    # a run with no check does not synchronise on it; the others are clean
    x2, _ = plan.run(yb, mask, h, lam, mu, iters)
    torch.cuda.synchronize()
    for b in (0, 2):
        assert torch.equal(x2[off[b]:off[b + 1]], x_clean[off[b]:off[b + 1]]), b
    assert not torch.isfinite(x2[off[1]:off[2]]).all()


def _poisoned_pair(images, opts, run):
    """Run `run(plan)` on a plan whose caller workspace was filled with NaN
    and on one filled with zeros; returns both results."""
    import torch
    from paper_1602_01410_amd import binding
    nbytes = binding.workspace_size(images, **opts)
    out = []
    for fill in (float("nan"), 0.0):
        ws = torch.full(((nbytes + 3) // 4,), fill, dtype=torch.float32, device="cuda")
        plan = binding.Plan(images, workspace=ws, **opts)
        out.append(run(plan))
        torch.cuda.synchronize()
        plan.close()
    return out


# schedule 3 (no autotuning): the autotuner would clear the state buffers
@pytest.mark.parametrize("opts", [dict(check_every=10, schedule=3),
                                  dict(check_every=5, bgs_passes=2, adapt_t=3.0, warm_iters=10, schedule=3),
                                  dict(check_every=4, use_graph=0, batched=0)])
def test_poisoned_workspace_forward(opts):
    import torch
    probs = _batch()
    images = [desc(p) for p in probs]
    y, mask, h, lam, mu = device_inputs(probs)

    def run(plan):
        yt = torch.empty_like(y)
        x, st = plan.run(y, mask, h, lam, mu, 23, ytilde_out=yt, stats=True)
        x2, st2 = plan.run(y, mask, h, lam, mu, 7, stats=True)
        return x.clone(), yt, st, x2.clone(), st2

    a, b = _poisoned_pair(images, opts, run)
    assert torch.isfinite(a[0]).all()
    for u, v in zip(a, b):
        if isinstance(u, torch.Tensor):
            assert torch.equal(u, v)
        else:
            assert u == v


def test_poisoned_workspace_backward():
    import torch
    probs = _batch()
    images = [desc(p) for p in probs]
    y, mask, h, lam, mu = device_inputs(probs)
    g = torch.Generator(device="cpu").manual_seed(5)
    gx = torch.randn(y.numel(), generator=g).cuda()

    def run(plan):
        x, _ = plan.run(y, mask, h, lam, mu, 12)
        gy, gl, gh = plan.backward(y, mask, h, lam, mu, gx)
        return x.clone(), gy, gl, gh

    a, b = _poisoned_pair(images, dict(ckpt_every=4, max_iters=12, schedule=3), run)
    assert torch.isfinite(a[1]).all()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
