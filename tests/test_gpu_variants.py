"""The variants of the method in Sec. III-B on the HIP path against the FP64
oracle: block-Gauss-Seidel passes per iteration ("Proposed-AD"), the
adaptive penalty of eq. (varying_penalty) with the rescaling of d, and the
quadratic warm start of z (eqs. (ini_x), (ini_z))."""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, desc, device_inputs, explicit_mask, gpu_run, log
from .test_gpu_parity import _mixed

pytestmark = pytest.mark.gpu


def oracle_variant(p, iters, **kw):
    return oracle.admm_run(p["y"].astype(np.float64), explicit_mask(p), p["h"].astype(np.float64),
                           float(np.float32(p["lam"])), float(np.float32(p["mu"])), iters, **kw)


def _inpaint_96(seed=41, mu=0.05):
    return synth.problem(96, 96, 7, "rect", "gauss", sigma=1.5, mask_kind=synth.MASK_EXPLICIT, missing=0.4,
                         bsnr=45.0, lam=2e-3, mu=mu, seed=seed)


@pytest.mark.parametrize("passes", [2, 4])
def test_bgs_passes_plain_72(passes):
    """72^2, 9x9 box (b = 4: Proposed-AD takes 4 passes), 100 iterations."""
    p = synth.config_plain_72()
    g = gpu_run([p], 100, bgs_passes=passes)
    r = oracle_variant(p, 100, passes=passes)
    assert_parity(g["x"][0], r["x"], what="P=%d x" % passes)
    assert_parity(g["yt"][0], r["yt"], what="P=%d ytilde" % passes)


def test_bgs_passes_mixed_batch_graph():
    """Uneven sizes and every mask kind in one plan, 3 passes, graph replay of
    check periods."""
    probs = _mixed(seed0=30)
    iters = 40
    g = gpu_run(probs, iters, bgs_passes=3, check_every=10, use_graph=1)
    for b, p in enumerate(probs):
        r = oracle_variant(p, iters, passes=3)
        assert_parity(g["x"][b], r["x"], what="img%d %dx%d x" % (b, p["M"], p["N"]))
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)


@pytest.mark.parametrize("mu0", [2.0, 1e-3])
def test_adaptive_penalty_decision_sequence(mu0):
    """mu after n iterations for n = 1..24 (one plan, restarted from the
    initial state each time) equals the oracle's sequence: every doubling,
    halving and keep decision is the same; x then agrees after 24."""
    import torch
    from paper_1602_01410_amd import binding
    p = synth.problem(72, 72, 9, "rect", "box", bsnr=50.0, lam=1e-3, mu=mu0, seed=synth.BASE_SEED, ramp_width=64)
    n_max = 24
    r = oracle_variant(p, n_max, adapt_t=3.0)
    seq = [float(h[4]) for h in r["hist"]] + [float(r["mu"])]   # mu before iteration n, then the final one
    plan = binding.Plan([desc(p)], adapt_t=3.0)
    y, mask, h, lam, mu = device_inputs([p])
    got = []
    for n in range(1, n_max + 1):
        x, st = plan.run(y, mask, h, lam, mu, n, stats=True)
        got.append(st[0]["mu"])
    torch.cuda.synchronize()
    log("oracle mu: %s" % " ".join("%.4g" % v for v in seq[1:]))
    log("GPU    mu: %s" % " ".join("%.4g" % v for v in got))
    changes = sum(1 for a, b in zip(seq[:-1], seq[1:]) if a != b)
    assert changes >= 2, "the workload should move the penalty"
    np.testing.assert_allclose(got, seq[1:], rtol=1e-6)
    assert_parity(x.cpu().numpy().astype(np.float64).reshape(p["M"], p["N"]), r["x"], what="x after 24")


def test_adaptive_penalty_graph_and_state():
    """Adaptive penalty under graph replay on an inpainting problem: x, the
    final mu and the rescaled dual state d agree with the oracle."""
    p = _inpaint_96(mu=0.5)
    iters = 50
    g = gpu_run([p], iters, want_state=True, adapt_t=3.0, check_every=10, use_graph=1)
    r = oracle_variant(p, iters, adapt_t=3.0)
    log("final mu: GPU %.6g oracle %.6g" % (g["stats"][0]["mu"], r["mu"]))
    assert g["stats"][0]["mu"] == pytest.approx(r["mu"], rel=1e-6)
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")
    d_ref = np.stack([r["dh"], r["dv"]], -1)
    assert_parity(g["d"][0].reshape(d_ref.shape), d_ref, rel=1e-3, absfrac=1e-2, what="d")


@pytest.mark.parametrize("iters,small", [(1, 0), (40, 0), (40, 1)])
def test_warm_start(iters, small):
    """100 warm-start steps with tau = 1e-3 on an inpainting problem, then
    `iters` iterations (on the whole-image-in-LDS kernel with small = 1)."""
    p = _inpaint_96()
    g = gpu_run([p], iters, warm_iters=100, warm_tau=1e-3, small_images=small)
    assert g["plan"].tiles()[3] == small
    r = oracle_variant(p, iters, warm_iters=100, warm_tau=1e-3)
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")


def test_proposed_ad_full_configuration():
    """The configuration of Sec. III-B together: b passes, adaptive penalty
    with t = 3, 100 warm-start steps; a decimated and an explicit-mask image
    of different sizes in one plan."""
    probs = [synth.problem(64, 96, 7, "rect", "gauss", sigma=1.2, mask_kind=synth.MASK_DECIMATE, decim=3,
                           bsnr=40.0, lam=1e-3, mu=0.05, seed=51),
             _inpaint_96(seed=52)]
    iters = 30
    # one pass count for the plan: b of the larger kernel (per-image counts
    # are tested below)
    passes = max(p["K"] // 2 for p in probs)
    g = gpu_run(probs, iters, bgs_passes=passes, adapt_t=3.0, warm_iters=100, warm_tau=1e-3)
    for b, p in enumerate(probs):
        r = oracle_variant(p, iters, passes=passes, adapt_t=3.0, warm_iters=100, warm_tau=1e-3)
        assert g["stats"][b]["mu"] == pytest.approx(r["mu"], rel=1e-6)
        assert_parity(g["x"][b], r["x"], what="img%d x" % b)
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)


def test_adaptive_penalty_continue_equals_longer_run():
    """run(a) then continue(b) with the adaptive penalty goes on from the
    adapted mu and its rescaled d: the result equals the oracle's run of
    a + b iterations, and the GPU's own run(a + b) bit for bit."""
    import torch
    from paper_1602_01410_amd import binding
    p = _inpaint_96(mu=0.5)
    a, b = 17, 23
    r = oracle_variant(p, a + b, adapt_t=3.0)
    y, mask, h, lam, mu = device_inputs([p])
    plan = binding.Plan([desc(p)], adapt_t=3.0, check_every=5)
    x_one, st_one = plan.run(y, mask, h, lam, mu, a + b, stats=True)
    x_one = x_one.clone()
    x = torch.empty_like(y)
    plan.run(y, mask, h, lam, mu, a, x_out=x)
    # a different mu passed to continue is ignored: the adapted one goes on
    _, st = plan.cont(lam, mu * 7.0, b, x, stats=True)
    torch.cuda.synchronize()
    log("mu: continued %.6g, one run %.6g, oracle %.6g" % (st[0]["mu"], st_one[0]["mu"], r["mu"]))
    assert st[0]["mu"] == pytest.approx(r["mu"], rel=1e-6)
    assert st[0]["mu"] == st_one[0]["mu"]
    assert_parity(x.cpu().numpy().astype(np.float64).reshape(p["M"], p["N"]), r["x"], what="x")
    assert torch.equal(x, x_one)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_proposed_ad_passes_per_image(use_graph):
    """bgs_passes = 0: every image takes b passes for its (2b+1)^2 blur, the
    rule of Sec. III-B, in one mixed batch (b = 1, 2, 4 and 6), with the
    adaptive penalty (t = 3) and 100 warm-start steps; each image against the
    oracle run with its own pass count."""
    probs = [synth.problem(64, 64, 3, "rect", "gauss", sigma=0.8, bsnr=45.0, lam=1e-3, mu=0.05, seed=61),
             synth.problem(72, 96, 5, "rect", "gauss", sigma=1.2, mask_kind=synth.MASK_DECIMATE, decim=2,
                           bsnr=40.0, lam=1e-3, mu=0.05, seed=62),
             synth.problem(96, 96, 9, "rect", "box", mask_kind=synth.MASK_EXPLICIT, missing=0.4, bsnr=45.0,
                           lam=2e-3, mu=0.05, seed=63),
             synth.problem(96, 128, 13, "rect", "motion", bsnr=40.0, lam=1e-3, mu=0.05, seed=64)]
    iters = 24
    g = gpu_run(probs, iters, bgs_passes=0, adapt_t=3.0, warm_iters=100, warm_tau=1e-3, check_every=8,
                use_graph=use_graph)
    for b, p in enumerate(probs):
        passes = max(1, p["K"] // 2)
        r = oracle_variant(p, iters, passes=passes, adapt_t=3.0, warm_iters=100, warm_tau=1e-3)
        log("img%d: K=%d, %d passes, mu GPU %.6g oracle %.6g" % (b, p["K"], passes, g["stats"][b]["mu"], r["mu"]))
        assert g["stats"][b]["mu"] == pytest.approx(r["mu"], rel=1e-6)
        assert_parity(g["x"][b], r["x"], what="img%d x" % b)
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)
