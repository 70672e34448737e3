"""The whole-image-in-LDS path (square images of side 32, 48, 64, 72 or 96:
one workgroup per image runs a whole check period with the image in LDS; by
default for sides up to 72, with option small_images = 1 for all) against the FP64 oracle, element by element: the 72^2 workload (config 1)
at its full 200 iterations, a batch of every side and mask kind, runs
without checks (launches of 50 iterations), early stopping, continue, and
NaN reporting.  The plan reports the path it takes."""
import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, desc, device_inputs, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


def _batch():
    out = []
    for q, (side, kind) in enumerate([(32, synth.MASK_BOUNDARY), (48, synth.MASK_EXPLICIT),
                                      (64, synth.MASK_DECIMATE), (72, synth.MASK_BOUNDARY),
                                      (96, synth.MASK_EXPLICIT), (96, synth.MASK_DECIMATE)]):
        out.append(synth.problem(side, side, 5 + 2 * (q % 3), "rect", "gauss", sigma=1.0 + 0.3 * q, mask_kind=kind,
                                 decim=3, missing=0.3, bsnr=40.0, lam=2e-3, mu=0.05, seed=950 + q, nrect=6))
    return out


def test_plain_72_full_run():
    p = synth.config_plain_72()
    g = gpu_run([p], p["iters"], check_every=10, use_graph=1, small_images=1)
    assert g["plan"].tiles()[3] == 1
    r = oracle_run(p, p["iters"])
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")
    assert g["stats"][0]["iters_done"] == p["iters"] and g["stats"][0]["status"] == 0
    # the residuals of the last check are the oracle's of iteration 200
    h = r["hist"][-1]
    assert g["stats"][0]["r_primal"] == pytest.approx(h[0], rel=1e-3)
    assert g["stats"][0]["r_dual"] == pytest.approx(h[1], rel=1e-3)


@pytest.mark.parametrize("check_every", [10, 0])
def test_every_side_and_mask(check_every):
    probs = _batch()
    iters = 120
    g = gpu_run(probs, iters, want_state=True, check_every=check_every, small_images=1)
    assert g["plan"].tiles()[3] == 1
    for b, p in enumerate(probs):
        r = oracle_run(p, iters)
        assert_parity(g["x"][b], r["x"], what="img%d %d^2 x" % (b, p["M"]))
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)
        d_ref = np.stack([r["dh"], r["dv"]], -1)
        assert_parity(g["d"][b].reshape(d_ref.shape), d_ref, rel=1e-3, absfrac=1e-2, what="img%d d" % b)


def test_same_iterates_as_the_two_pass_kernels():
    probs = _batch()[:4]
    a = gpu_run(probs, 40, check_every=10, small_images=1)
    b = gpu_run(probs, 40, check_every=10, small_images=0)
    assert a["plan"].tiles()[3] == 1 and b["plan"].tiles()[3] == 0
    for k in range(len(probs)):
        r = oracle_run(probs[k], 40)
        assert_parity(a["x"][k], r["x"], what="small path img%d" % k)
        assert_parity(b["x"][k], r["x"], what="two-pass img%d" % k)


def test_default_routing():
    """With the default option the plan takes the path for images of side at
    most 72 only, and only with the options the path supports."""
    from paper_1602_01410_amd import binding
    def path(sides, **kw):
        pl = binding.Plan([dict(height=s, width=s, ksize=5) for s in sides], **kw)
        try:
            return pl.tiles()[3]
        finally:
            pl.close()
    assert path([32, 48, 64, 72]) == 1
    assert path([72] * 8) == 1
    assert path([96]) == 0 and path([64, 96]) == 0
    assert path([96], small_images=1) == 1
    assert path([64], small_images=0) == 0
    assert path([64], bgs_passes=2) == 0 and path([64], adapt_t=3.0) == 0
    pl = binding.Plan([dict(height=64, width=48, ksize=5)])
    assert pl.tiles()[3] == 0
    pl.close()


@pytest.mark.parametrize("iters,tol,launches", [(200, 0.0, 1), (450, 0.0, 3), (200, 1e-30, 20)])
def test_launches_per_run(iters, tol, launches):
    """Without a stop test one launch runs up to 200 iterations (every check
    inside it recorded); with tolerances, one launch per check period so that
    the host can stop between them.  The residuals are those of the last
    check either way."""
    from paper_1602_01410_amd import binding
    p = synth.config_plain_72()
    plan = binding.Plan([desc(p)], check_every=10, profile=1, tol_primal=tol, tol_dual=tol)
    assert plan.tiles()[3] == 1
    y, mask, h, lam, mu = device_inputs([p])
    _, st = plan.run(y, mask, h, lam, mu, iters, stats=True)
    assert plan.kernel_times()[1] == launches
    assert st[0]["iters_done"] == iters and st[0]["status"] == 0
    r = oracle_run(p, iters)
    assert st[0]["r_primal"] == pytest.approx(r["hist"][-1][0], rel=1e-3)
    assert st[0]["r_dual"] == pytest.approx(r["hist"][-1][1], rel=1e-3)
    plan.close()


def test_early_stop_and_continue():
    import torch
    from paper_1602_01410_amd import binding
    probs = [synth.problem(64, 64, 5, "rect", "box", bsnr=50.0, lam=1e-2, mu=0.2, seed=90),
             synth.problem(72, 72, 7, "rect", "gauss", sigma=1.5, bsnr=40.0, lam=2e-3, mu=0.01, seed=91)]
    iters, K = 300, 10
    g = gpu_run(probs, iters, check_every=K, tol_primal=2e-4, tol_dual=2e-4, small_images=1)
    stopped = 0
    for b, p in enumerate(probs):
        n = g["stats"][b]["iters_done"]
        log("image %d stopped after %d iterations" % (b, n))
        assert n % K == 0 and 0 < n <= iters
        stopped += n < iters
        r = oracle_run(p, n)
        assert_parity(g["x"][b], r["x"], what="img%d x at its stop" % b)
    assert stopped >= 1
    # run(a) + continue(b) = run(a + b)
    p = probs[1]
    plan = binding.Plan([desc(p)], check_every=K, small_images=1)
    assert plan.tiles()[3] == 1
    y, mask, h, lam, mu = device_inputs([p])
    x = torch.empty_like(y)
    plan.run(y, mask, h, lam, mu, 37, x_out=x)
    plan.cont(lam, mu, 23, x)
    torch.cuda.synchronize()
    r = oracle_run(p, 60)
    assert_parity(x.cpu().numpy().astype(np.float64).reshape(72, 72), r["x"], what="continued x")


def test_nan_reported_for_its_image():
    from paper_1602_01410_amd import binding
    probs = _batch()[:3]
    plan = binding.Plan([desc(p) for p in probs], check_every=5, small_images=1)
    assert plan.tiles()[3] == 1
    y, mask, h, lam, mu = device_inputs(probs)
    off = probs[0]["M"] * probs[0]["N"]
    obs = np.flatnonzero(probs[1]["mask"].ravel())
    y[off + int(obs[0])] = float("nan")
    with pytest.raises(binding.DeconvError) as e:
        plan.run(y, mask, h, lam, mu, 10, stats=True)
    assert [s["status"] for s in e.value.stats] == [0, 4, 0]
