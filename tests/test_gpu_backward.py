"""Adjoint kernels vs the FP64 hand-written oracle adjoint (which is itself
pinned by central finite differences in the CPU tests)."""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth

from .gpu_util import desc, device_inputs, explicit_mask, log, rel_l2

pytestmark = pytest.mark.gpu


def _problems():
    return [synth.problem(24, 18, 5, "rect", "random", mask_kind=synth.MASK_EXPLICIT, missing=0.2, bsnr=40.0,
                          lam=3e-3, mu=0.05, seed=71, nrect=5),
            synth.problem(48, 64, 7, "rect", "random", mask_kind=synth.MASK_DECIMATE, decim=2, bsnr=40.0,
                          lam=5e-3, mu=0.08, seed=72, nrect=5),
            synth.problem(72, 72, 9, "rect", "gauss", sigma=2.0, bsnr=45.0, lam=1e-3, mu=0.05, seed=73)]


@pytest.mark.parametrize("iters,ck", [(6, 2), (7, 3), (5, 5)])
def test_backward_matches_oracle(iters, ck):
    import torch
    from paper_1602_01410_amd import binding
    probs = _problems()
    plan = binding.Plan([desc(p) for p in probs], ckpt_every=ck, max_iters=iters)
    y, mask, h, lam, mu = device_inputs(probs)
    x, _ = plan.run(y, mask, h, lam, mu, iters)
    rng = np.random.default_rng(iters * 10 + ck)
    gxs = [rng.standard_normal((p["M"], p["N"])).astype(np.float32) for p in probs]
    gx = torch.from_numpy(np.concatenate([g.ravel() for g in gxs])).cuda()
    gy, gl, gh = plan.backward(y, mask, h, lam, mu, gx)
    torch.cuda.synchronize()
    gys = [a.cpu().numpy().astype(np.float64) for a in plan.split(gy)]
    ghs, o = [], 0
    for p in probs:
        k = p["K"] * p["K"]
        ghs.append(gh[o:o + k].cpu().numpy().reshape(p["K"], p["K"]).astype(np.float64))
        o += k
    gls = gl.cpu().numpy()
    for b, p in enumerate(probs):
        ry, rl, rh = oracle.admm_backward(p["y"].astype(np.float64), explicit_mask(p), p["h"].astype(np.float64),
                                          float(np.float32(p["lam"])), float(np.float32(p["mu"])), iters,
                                          gxs[b].astype(np.float64))
        ey, eh = rel_l2(gys[b], ry), rel_l2(ghs[b], rh)
        el = abs(float(gls[b]) - rl) / max(abs(rl), 1e-12)
        log("img%d grad_y %.2e grad_h %.2e grad_lambda %.2e (ref %.4e)" % (b, ey, eh, el, rl))
        assert ey <= 1e-3 and eh <= 1e-3, (b, ey, eh)
        assert el <= 1e-3 or abs(float(gls[b]) - rl) <= 1e-6 * np.abs(ry).max(), (b, el)


def test_autograd_function():
    import torch
    from paper_1602_01410_amd import binding
    p = _problems()[2]
    plan = binding.Plan([desc(p)], ckpt_every=4, max_iters=8)
    y, mask, h, lam, mu = device_inputs([p])
    y.requires_grad_(True)
    h.requires_grad_(True)
    lam.requires_grad_(True)
    x = binding.admm(y, h, lam, plan, mask, mu, 8)
    target = torch.from_numpy(p["x_true"].reshape(-1)).cuda()
    loss = 0.5 * ((x - target) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ry, rl, rh = oracle.admm_backward(p["y"].astype(np.float64), explicit_mask(p), p["h"].astype(np.float64),
                                      float(np.float32(p["lam"])), float(np.float32(p["mu"])), 8,
                                      (x.detach().cpu().numpy() - p["x_true"].reshape(-1)).reshape(p["M"], p["N"]))
    assert rel_l2(y.grad.cpu().numpy().reshape(p["M"], p["N"]), ry) <= 1e-3
    assert rel_l2(h.grad.cpu().numpy().reshape(p["K"], p["K"]), rh) <= 1e-3


def test_backward_few_tiles_matches_batch():
    """A lone 512^2 image takes the launch choices of plans with few tiles
    (512-thread column tiles, non-temporal spectra) in its forward recompute;
    its gradients equal those of the same image inside a batch of eight,
    which takes the ordinary ones."""
    import torch
    from paper_1602_01410_amd import binding
    p = synth.problem(512, 512, 9, "rect", "gauss", sigma=1.5, bsnr=45.0, lam=1e-3, mu=0.05, seed=512, nrect=12)
    iters, ck = 10, 5
    out = []
    for B in (1, 8):
        probs = [p] * B
        plan = binding.Plan([desc(q) for q in probs], ckpt_every=ck, max_iters=iters)
        y, mask, h, lam, mu = device_inputs(probs)
        plan.run(y, mask, h, lam, mu, iters)
        n = 512 * 512
        # the same dL/dx on every image
        gx = torch.sin((torch.arange(y.numel(), device=y.device) % n).float() * 1e-3).contiguous()
        gy, gl, gh = plan.backward(y, mask, h, lam, mu, gx)
        torch.cuda.synchronize()
        out.append((gy[:n].cpu().numpy().astype(np.float64), float(gl[0]), gh[:81].cpu().numpy().astype(np.float64)))
        plan.close()
    (y1, l1, h1), (y8, l8, h8) = out
    log("grad_y %.2e grad_h %.2e grad_lambda %.2e" % (rel_l2(y8, y1), rel_l2(h8, h1), abs(l8 - l1) / abs(l1)))
    assert rel_l2(y8, y1) <= 1e-6 and rel_l2(h8, h1) <= 1e-6 and abs(l8 - l1) <= 1e-6 * abs(l1)


def test_backward_names_its_run():
    """The reverse pass replays the checkpoints of the run it names: after a
    second forward on the plan, the autograd function of the first refuses
    (status 8) instead of returning the second run's gradient; a blur
    spectrum query in between changes nothing; the same reverse pass asked
    for twice gives the same gradients."""
    import torch
    from paper_1602_01410_amd import binding
    probs = _problems()
    plan = binding.Plan([desc(p) for p in probs], ckpt_every=3, max_iters=9)
    y, mask, h, lam, mu = device_inputs(probs)
    g = torch.Generator(device="cpu").manual_seed(3)
    gx = torch.randn(y.numel(), generator=g).cuda()
    x1, _ = plan.run(y, mask, h, lam, mu, 9)
    rid = plan.run_id()
    assert rid != 0
    gy1, gl1, gh1 = plan.backward(y, mask, h, lam, mu, gx, run_id=rid)
    gy2, gl2, gh2 = plan.backward(y, mask, h, lam, mu, gx, run_id=rid)
    assert plan.run_id() == 0      # the forward state was used as scratch
    plan.blur_spectrum(h * 0.5)
    gy3, gl3, gh3 = plan.backward(y, mask, h, lam, mu, gx, run_id=rid)
    torch.cuda.synchronize()
    for a, b in ((gy1, gy2), (gl1, gl2), (gh1, gh2), (gy1, gy3), (gl1, gl3), (gh1, gh3)):
        assert torch.equal(a, b)
    plan.run(y * 1.1, mask, h, lam, mu, 9)
    assert plan.run_id() not in (0, rid)
    with pytest.raises(binding.DeconvError) as e:
        plan.backward(y, mask, h, lam, mu, gx, run_id=rid)
    assert e.value.code == 8
    # the autograd function: two forwards on one plan, then the first's backward
    yy = y.clone().requires_grad_(True)
    xa = binding.admm(yy, h, lam, plan, mask, mu, 9)
    xb = binding.admm(yy, h, lam, plan, mask, mu, 9)
    with pytest.raises(binding.DeconvError) as e:
        (xa * gx).sum().backward()
    assert e.value.code == 8
    (xb * gx).sum().backward()
    torch.cuda.synchronize()
    assert torch.isfinite(yy.grad).all()


def test_reverse_pass_graph_replay():
    """The reverse pass captured as one graph (use_graph = 1) and replayed
    gives the gradients of the uncaptured reverse pass bit for bit, also
    when the contents of grad_x change between replays."""
    import torch
    from paper_1602_01410_amd import binding
    probs = _problems()
    y, mask, h, lam, mu = device_inputs(probs)
    g = torch.Generator(device="cpu").manual_seed(11)
    gx = torch.randn(y.numel(), generator=g).cuda()
    out = {}
    for use_graph in (0, 1):
        plan = binding.Plan([desc(p) for p in probs], ckpt_every=4, max_iters=10, use_graph=use_graph)
        res = []
        for rep in range(3):
            gx.copy_(torch.randn(y.numel(), generator=torch.Generator(device="cpu").manual_seed(20 + rep)).cuda())
            plan.run(y, mask, h, lam, mu, 10)
            res.append([t.clone() for t in plan.backward(y, mask, h, lam, mu, gx)])
        torch.cuda.synchronize()
        out[use_graph] = res
    for a, b in zip(out[0], out[1]):
        for u, v in zip(a, b):
            assert torch.equal(u, v)
    assert not torch.equal(out[1][0][0], out[1][1][0])
