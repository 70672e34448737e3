"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (batched, graph replay, residual check every 10 iterations).

* 1024^2 / 500 iterations: the whole image against the FP64 oracle.
* 2048^2 inpainting: the whole image against the oracle at the full 300
  iterations (and at 40); at 300 also the one-iteration relations of the
  method checked on the HIP path's own state.
* the 256-image mixed batch: one boundary and one decimated image of every
  side (128 ... 1024) against the oracle.
* early stopping on the residual test.
"""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, desc, device_inputs, explicit_mask, gpu_run, log, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

BENCH_OPTS = dict(batched=1, use_graph=1, check_every=10)


@pytest.mark.timeout(400)
def test_large_1024_full_500_iterations():
    p = synth.config_large_1024()
    log("1024^2 x 500 it: GPU")
    g = gpu_run([p], p["iters"], **BENCH_OPTS)
    log("1024^2 x 500 it: oracle (FP64, %d threads)" % oracle.num_threads())
    r = oracle_run(p, p["iters"])
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")


@pytest.mark.timeout(500)
def test_inpaint_2048_full_300_iterations():
    """The inpainting workload (2048^2, 21x21 motion blur, boundaries + 50%
    missing pixels) at its full 300 iterations, whole image against the FP64
    oracle."""
    p = synth.config_inpaint_2048()
    log("2048^2 x %d it: GPU" % p["iters"])
    g = gpu_run([p], p["iters"], **BENCH_OPTS)
    log("2048^2 x %d it: oracle (FP64, %d threads)" % (p["iters"], oracle.num_threads()))
    r = oracle_run(p, p["iters"])
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")


@pytest.mark.timeout(300)
def test_inpaint_2048_full_size_40_iterations():
    p = synth.config_inpaint_2048()
    g = gpu_run([p], 40, **BENCH_OPTS)
    log("2048^2 x 40 it: oracle")
    r = oracle_run(p, 40)
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")


def _step_relations(p, st0, st1, x1, alpha=2.0):
    """Check one iteration s0 -> (x1, s1) of the method in float64 with numpy
    FFTs: the x-step normal equations, the z-step, the prox and the dual
    update.  Returns the relative residuals."""
    M, N, K = p["M"], p["N"], p["K"]
    b = K // 2
    h = p["h"].astype(np.float64)
    hpad = np.zeros((M, N))
    for a in range(-b, b + 1):
        for c in range(-b, b + 1):
            hpad[a % M, c % N] += h[b + a, b + c]
    Hf = np.fft.fft2(hpad)
    H = lambda a, adj=False: np.real(np.fft.ifft2(np.fft.fft2(a) * (np.conj(Hf) if adj else Hf)))
    D = lambda a: (np.roll(a, -1, 1) - a, np.roll(a, -1, 0) - a)
    DT = lambda wh, wv: np.roll(wh, 1, 1) - wh + np.roll(wv, 1, 0) - wv
    yt0, v0, d0 = st0
    yt1, v1, d1 = st1
    mu, lam = float(np.float32(p["mu"])), float(np.float32(p["lam"]))
    rhs = H(yt0, True) + mu * DT(v0[..., 0] - d0[..., 0], v0[..., 1] - d0[..., 1])
    gh, gv = D(x1)
    lhs = H(H(x1), True) + mu * DT(gh, gv)
    r_x = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
    un = explicit_mask(p) == 0
    hx = H(x1)
    z_ref = yt0 + alpha * (hx - yt0)
    r_z = np.abs(yt1[un] - z_ref[un]).max() / np.abs(z_ref[un]).max()
    obs_same = np.array_equal(yt1[~un], yt0[~un])
    uh, uv = gh + d0[..., 0], gv + d0[..., 1]
    nr = np.sqrt(uh ** 2 + uv ** 2)
    tau = lam / mu
    s = np.where(nr > tau, 1.0 - tau / np.where(nr > 0, nr, 1.0), 0.0)
    vref = np.stack([s * uh, s * uv], -1)
    dref = np.stack([uh, uv], -1) - vref
    scale = np.linalg.norm(np.stack([uh, uv], -1))
    r_v = np.linalg.norm(v1 - vref) / scale
    r_d = np.linalg.norm(d1 - dref) / scale
    return r_x, r_z, obs_same, r_v, r_d


@pytest.mark.timeout(300)
def test_inpaint_2048_full_300_iterations_step_relations():
    """At the full iteration count: after 299 iterations, export the state;
    one more iteration must satisfy the method's relations (x-step normal
    equations to FP32 accuracy, z-step, prox, dual update)."""
    import torch
    from paper_1602_01410_amd import binding
    p = synth.config_inpaint_2048()
    plan = binding.Plan([desc(p)], **BENCH_OPTS)
    y, mask, h, lam, mu = device_inputs([p])
    x = torch.empty_like(y)
    plan.run(y, mask, h, lam, mu, p["iters"] - 1, x_out=x)
    sh = (p["M"], p["N"])
    st0 = [a.cpu().numpy().astype(np.float64) for a in plan.state_export(y.device)]
    st0 = (st0[0].reshape(sh), st0[1].reshape(sh + (2,)), st0[2].reshape(sh + (2,)))
    plan.cont(lam, mu, 1, x)
    st1 = [a.cpu().numpy().astype(np.float64) for a in plan.state_export(y.device)]
    st1 = (st1[0].reshape(sh), st1[1].reshape(sh + (2,)), st1[2].reshape(sh + (2,)))
    x1 = x.cpu().numpy().astype(np.float64).reshape(sh)
    r_x, r_z, obs_same, r_v, r_d = _step_relations(p, st0, st1, x1)
    log("step relations: x %.2e z %.2e v %.2e d %.2e" % (r_x, r_z, r_v, r_d))
    assert np.isfinite(x1).all()
    assert r_x <= 1e-4 and r_z <= 1e-5 and obs_same and r_v <= 1e-5 and r_d <= 1e-5


@pytest.mark.timeout(600)
def test_mixed_batch_256_sampled_images():
    """The 256-image batch as bench.py runs it (hybrid launches, graph
    replay); for every side that occurs, the first boundary-only and the
    first x4-decimated image are compared with the oracle."""
    probs = synth.config_batch()
    iters = 200
    g = gpu_run(probs, iters, **BENCH_OPTS)
    seen = {}
    for b, p in enumerate(probs):
        key = (p["M"], p["mask_kind"])
        if key not in seen:
            seen[key] = b
    picks = [seen[k] for k in sorted(seen)]
    log("%d sampled images: %s" % (len(picks), sorted(seen)))
    assert {k[0] for k in seen} == {128, 192, 256, 384, 512, 768, 1024}
    for b in picks:
        p = probs[b]
        log("image %d (%d^2, %s)" % (b, p["M"], "x4 decimated" if p["mask_kind"] == synth.MASK_DECIMATE else "boundary"))
        r = oracle_run(p, iters)
        assert_parity(g["x"][b], r["x"], what="img%d x" % b)
    for b, p in enumerate(probs):
        assert np.isfinite(g["x"][b]).all()
        assert g["stats"][b]["status"] == 0


def test_early_stop_on_residuals():
    """Images stop at the first check where both residual tests hold; their
    output is the iterate of that check; the others run to the end."""
    probs = [synth.problem(64, 64, 5, "rect", "box", bsnr=50.0, lam=1e-2, mu=0.2, seed=90),
             synth.problem(96, 72, 7, "rect", "gauss", sigma=1.5, bsnr=40.0, lam=2e-3, mu=0.01, seed=91)]
    iters, K = 300, 10
    g = gpu_run(probs, iters, want_state=True, batched=1, use_graph=1, check_every=K, tol_primal=2e-4,
                tol_dual=2e-4)
    stopped = 0
    for b, p in enumerate(probs):
        st = g["stats"][b]
        n = st["iters_done"]
        log("image %d stopped after %d iterations (r_p %.2e r_d %.2e)" % (b, n, st["r_primal"], st["r_dual"]))
        assert n % K == 0 and 0 < n <= iters
        r = oracle_run(p, n)
        assert_parity(g["x"][b], r["x"], what="img%d x at its stop" % b)
        if n < iters:
            stopped += 1
            # the state left behind is that of the stopping iteration
            sh = (p["M"], p["N"], 2)
            assert_parity(g["yt"][b], r["yt"], what="img%d ytilde at its stop" % b)
            assert_parity(g["v"][b].reshape(sh), np.stack([r["vh"], r["vv"]], -1), rel=1e-3, absfrac=1e-2,
                          what="img%d v at its stop" % b)
            assert_parity(g["d"][b].reshape(sh), np.stack([r["dh"], r["dv"]], -1), rel=1e-3, absfrac=1e-2,
                          what="img%d d at its stop" % b)
            sc = np.sqrt(2.0 * p["M"] * p["N"])
            assert st["r_primal"] <= 2e-4 * sc and st["r_dual"] <= 2e-4 * sc
            h = r["hist"][-1]
            assert h[0] <= 2e-4 * sc * 1.01 and h[1] <= 2e-4 * sc * 1.01
    assert stopped >= 1


@pytest.mark.timeout(400)
def test_batch_with_buffers_beyond_4gib():
    """136 images of 2048^2 in one plan (570 Mpx: the pixel-pair and spectrum
    buffers pass 4 GiB, so every 64-bit offset path is used): the first,
    a middle and the last image come out bit for bit as from a plan of that
    image alone, whose tiles are the same."""
    import torch
    from paper_1602_01410_amd import binding
    B, iters = 136, 4
    p = synth.problem(2048, 2048, 9, "rect", "gauss", sigma=1.5, bsnr=45.0, lam=1e-3, mu=0.05, seed=2048,
                      nrect=20)
    y1 = torch.from_numpy(p["y"].reshape(-1)).cuda()
    h1 = torch.from_numpy(p["h"].reshape(-1)).cuda()
    # each image scaled differently so that a mix-up between images shows
    scale = torch.arange(1, B + 1, dtype=torch.float32, device="cuda") / B
    y = (y1[None, :] * scale[:, None]).reshape(-1).contiguous()
    h = h1.repeat(B)
    lam = torch.full((B,), 1e-3, dtype=torch.float32, device="cuda")
    mu = torch.full((B,), 0.05, dtype=torch.float32, device="cuda")
    log("%d x 2048^2: %.2f GiB per float2 pixel buffer" % (B, y.numel() * 8 / 2 ** 30))
    plan = binding.Plan([desc(p)] * B, check_every=2)
    x, st = plan.run(y, None, h, lam, mu, iters, stats=True)
    torch.cuda.synchronize()
    n = 2048 * 2048
    picks = [0, B // 2, B - 1]
    xb = {b: x[b * n:(b + 1) * n].cpu() for b in picks}
    assert all(s["status"] == 0 and s["iters_done"] == iters for s in st)
    del x, plan
    torch.cuda.empty_cache()
    for b in picks:
        one = binding.Plan([desc(p)], check_every=2)
        xo, _ = one.run(y[b * n:(b + 1) * n].contiguous(), None, h1, lam[:1], mu[:1], iters)
        torch.cuda.synchronize()
        log("image %d: max |diff| %.3e" % (b, float((xo.cpu() - xb[b]).abs().max())))
        assert torch.equal(xo.cpu(), xb[b]), b
        one.close()
