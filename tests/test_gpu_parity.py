"""HIP path vs the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth

from .gpu_util import (assert_parity, desc, device_inputs, gpu_run, log, oracle_run, rel_l2)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


# --------------------------------------------------------------------------
# a0: the transforms themselves
# --------------------------------------------------------------------------

FFT_SHAPES = [(8, 8), (12, 16), (18, 24), (36, 72), (72, 72), (96, 128), (144, 192), (256, 256),
              (288, 384), (512, 576), (768, 1024), (1152, 1536), (1024, 1024), (2048, 2048)]


@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft2_parity(torch_cuda, shape):
    torch = torch_cuda
    from paper_1602_01410_amd import binding
    M, N = shape
    count = 2 if M * N <= 1 << 20 else 1
    log("fft2 %dx%d x%d" % (M, N, count))
    rng = np.random.default_rng(M * 7 + N)
    x = (rng.standard_normal((count, M, N)) + 1j * rng.standard_normal((count, M, N))).astype(np.complex64)
    for inverse in (False, True):
        t = torch.from_numpy(x.copy()).cuda()
        binding.fft2(t, inverse=inverse)
        torch.cuda.synchronize()
        got = t.cpu().numpy()
        for c in range(count):
            ref = oracle.fft2(x[c].astype(np.complex128), +1 if inverse else -1)
            r = rel_l2(got[c], ref)
            assert r <= 1e-5, (shape, inverse, r)


def test_blur_spectrum_and_kappa(torch_cuda):
    """H^ of the embedded kernel (setup step) vs the oracle; kappa of the
    paper's tables for the blurs FP32 can resolve."""
    torch = torch_cuda
    from paper_1602_01410_amd import binding
    kernels = [synth.box_kernel(5), synth.box_kernel(13), synth.gaussian_kernel(5, np.sqrt(5)),
               synth.gaussian_kernel(13, np.sqrt(13)), synth.box_kernel(21), synth.gaussian_kernel(21, np.sqrt(21))]
    plan = binding.Plan([dict(height=256, width=256, ksize=k.shape[0]) for k in kernels])
    h = torch.from_numpy(np.concatenate([k.astype(np.float32).ravel() for k in kernels])).cuda()
    spec = plan.blur_spectrum(h).cpu().numpy().view(np.complex64).reshape(len(kernels), 256, 256)
    for k, s in zip(kernels, spec):
        ref = oracle.psf_spectrum(256, 256, k.astype(np.float32).astype(np.float64))
        assert rel_l2(s, ref) <= 1e-6
        # kappa: both sides' min |H| must be well above FP32 rounding of max |H|
        kap_ref = np.abs(ref).max() / np.abs(ref).min()
        if kap_ref < 1e5:
            kap = np.abs(s).max() / np.abs(s).min()
            assert abs(kap - kap_ref) <= 1e-2 * kap_ref, (kap, kap_ref)


# --------------------------------------------------------------------------
# a1..a7: iterations
# --------------------------------------------------------------------------

def _small(M, N, K, kind=synth.MASK_BOUNDARY, seed=0, decim=3, missing=0.3, blur="random", lam=1e-2, mu=0.05):
    return synth.problem(M, N, K, "rect", blur, mask_kind=kind, decim=decim, missing=missing, bsnr=40.0,
                         lam=lam, mu=mu, seed=seed, nrect=6)


@pytest.mark.parametrize("shape", [(512, 512, synth.MASK_EXPLICIT), (256, 2048, synth.MASK_DECIMATE),
                                   (1024, 1024, synth.MASK_BOUNDARY), (18, 512, synth.MASK_BOUNDARY)])
def test_half_height_row_tiles(torch_cuda, shape):
    """Plans of one width with few row tiles use tiles of half the rows (a
    512^2 image: 4-row tiles, 256 x 2048: 1-row tiles, 1024^2: 2-row tiles,
    18 x 512: 4-row tiles with a ragged last one), 1024 threads each;
    results agree with the oracle, with the check/store iterations, graphs
    and one BGS-pass variant exercising every row-pass mode."""
    M, N, kind = shape
    p = _small(M, N, 9, kind, seed=M + N, blur="gauss", lam=3e-3)
    iters = 30
    g = gpu_run([p], iters, check_every=10, use_graph=1)
    r = oracle_run(p, iters)
    assert_parity(g["x"][0], r["x"], what="%dx%d x" % (M, N))
    assert_parity(g["yt"][0], r["yt"], what="%dx%d ytilde" % (M, N))
    g2 = gpu_run([p], 12, bgs_passes=2, adapt_t=3.0)
    r2 = oracle.admm_run(p["y"].astype(np.float64), p["mask"].astype(np.uint8), p["h"].astype(np.float64),
                         float(np.float32(p["lam"])), float(np.float32(p["mu"])), 12, passes=2, adapt_t=3.0)
    assert_parity(g2["x"][0], r2["x"], what="%dx%d x, 2 passes + adaptive" % (M, N))


def test_half_height_row_tiles_batch(torch_cuda):
    """Several images of one width whose half tiles keep 4 rows (six 512^2
    images, 384 default tiles) take the half tiles too: every image agrees
    with one launch per image, and one with the oracle."""
    probs = [_small(512, 512, 7, synth.MASK_EXPLICIT if b % 2 else synth.MASK_BOUNDARY, seed=500 + b,
                    blur="gauss", lam=3e-3) for b in range(6)]
    iters = 12
    g = gpu_run(probs, iters, check_every=5)
    a = gpu_run(probs, iters, check_every=5, batched=0)
    for b in range(len(probs)):
        assert rel_l2(g["x"][b], a["x"][b]) <= 1e-6, b
    r = oracle_run(probs[3], iters)
    assert_parity(g["x"][3], r["x"], what="512^2 in a batch of six, x")


def test_one_iteration_full_state(torch_cuda):
    """x^1, ytilde^1, v^1, d^1 after one iteration, per image of a mixed batch."""
    probs = [_small(24, 32, 5, synth.MASK_EXPLICIT, seed=1), _small(48, 36, 7, synth.MASK_DECIMATE, seed=2),
             _small(72, 72, 9, synth.MASK_BOUNDARY, seed=3, blur="box")]
    g = gpu_run(probs, 1, want_state=True)
    for b, p in enumerate(probs):
        r = oracle_run(p, 1)
        log("image %d %dx%d" % (b, p["M"], p["N"]))
        assert rel_l2(g["x"][b], r["x"]) <= 1e-5
        assert rel_l2(g["yt"][b], r["yt"]) <= 1e-5
        vref = np.stack([r["vh"], r["vv"]], -1)
        dref = np.stack([r["dh"], r["dv"]], -1)
        # v, d: the soft threshold is 1-Lipschitz, so errors stay at the
        # level of u = D x + d; v may be all zero after one iteration
        scale = np.linalg.norm(vref) + np.linalg.norm(dref)
        assert np.linalg.norm(g["v"][b] - vref) <= 1e-5 * scale
        assert np.linalg.norm(g["d"][b] - dref) <= 1e-5 * scale


@pytest.mark.parametrize("small_images", [0, 2])
def test_plain_72_config_200_iterations(torch_cuda, small_images):
    """72x72 domain, 9x9 box, observed 64x64, BSNR 50, lambda 1e-3, mu 0.05,
    200 iterations: relative L2 <= 1e-4, max abs <= 1e-3 of the range, on the
    two-pass kernels and on the default path (the image in LDS)."""
    p = synth.config_plain_72()
    g = gpu_run([p], p["iters"], small_images=small_images)
    assert g["plan"].tiles()[3] == (1 if small_images else 0)
    r = oracle_run(p, p["iters"])
    assert_parity(g["x"][0], r["x"], what="x")
    assert_parity(g["yt"][0], r["yt"], what="ytilde")


MIXED = [
    dict(M=48, N=96, K=7, kind=synth.MASK_BOUNDARY),
    dict(M=96, N=72, K=5, kind=synth.MASK_DECIMATE),
    dict(M=64, N=64, K=9, kind=synth.MASK_EXPLICIT),
    dict(M=128, N=192, K=11, kind=synth.MASK_BOUNDARY),
    dict(M=36, N=18, K=3, kind=synth.MASK_EXPLICIT),
    dict(M=144, N=128, K=15, kind=synth.MASK_DECIMATE),
    dict(M=16, N=8, K=3, kind=synth.MASK_BOUNDARY),
]


def _mixed(seed0=10, blur="random"):
    return [_small(d["M"], d["N"], d["K"], d["kind"], seed=seed0 + i, blur=blur, lam=3e-3, mu=0.05)
            for i, d in enumerate(MIXED)]


@pytest.mark.parametrize("alpha", [2.0, 1.0])
def test_mixed_batch_parity(torch_cuda, alpha):
    """Uneven sizes, all mask kinds, asymmetric kernels, one batched plan."""
    probs = _mixed()
    iters = 60
    g = gpu_run(probs, iters, alpha=alpha)
    for b, p in enumerate(probs):
        r = oracle_run(p, iters, alpha=alpha)
        assert_parity(g["x"][b], r["x"], what="img%d %dx%d x" % (b, p["M"], p["N"]))
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)


def test_batched_plain_graph_agree(torch_cuda):
    """Same kernels whatever the launch schedule: batched, per image, graph
    replay -- bitwise identical outputs."""
    probs = _mixed(seed0=30)
    a = gpu_run(probs, 25, batched=1, use_graph=0, check_every=5)
    b = gpu_run(probs, 25, batched=0, use_graph=0, check_every=5)
    c = gpu_run(probs, 25, batched=1, use_graph=1, check_every=5)
    c2 = gpu_run(probs, 26, batched=1, use_graph=1, check_every=5)
    for i in range(len(probs)):
        assert np.array_equal(a["x"][i], b["x"][i])
        assert np.array_equal(a["x"][i], c["x"][i])
        assert np.array_equal(a["yt"][i], c["yt"][i])
    # 26 iterations through graph replays + direct launches vs the oracle
    r = oracle_run(probs[3], 26)
    assert_parity(c2["x"][3], r["x"], what="graph 26 it")


def test_residuals_match_oracle(torch_cuda):
    probs = _mixed(seed0=40)[:4]
    iters = 20
    g = gpu_run(probs, iters, check_every=1, use_graph=0)
    for b, p in enumerate(probs):
        r = oracle_run(p, iters)
        h = r["hist"][-1]
        st = g["stats"][b]
        assert st["iters_done"] == iters and st["status"] == 0
        for key, ref in (("r_primal", h[0]), ("r_dual", h[1]), ("r_z", h[2])):
            assert abs(st[key] - ref) <= 2e-3 * max(ref, 1e-8), (b, key, st[key], ref)


def test_continue_equals_longer_run(torch_cuda):
    import torch
    from paper_1602_01410_amd import binding
    probs = [_small(64, 48, 5, synth.MASK_BOUNDARY, seed=50), _small(32, 32, 3, synth.MASK_DECIMATE, seed=51)]
    plan = binding.Plan([desc(p) for p in probs])
    y, mask, h, lam, mu = device_inputs(probs)
    x1, _ = plan.run(y, mask, h, lam, mu, 15)
    x2 = torch.empty_like(x1)
    plan.cont(lam, mu, 10, x2)
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        r = oracle_run(p, 25)
        assert_parity(plan.split(x2)[b].cpu().numpy().astype(np.float64), r["x"], what="continue")


def test_error_paths(torch_cuda):
    import torch
    from paper_1602_01410_amd import binding
    p = _small(32, 32, 5, seed=60)
    plan = binding.Plan([desc(p)])
    y, mask, h, lam, mu = device_inputs([p])
    hz = h.clone()
    hz[0] = 1.0
    hz[1] = -1.0
    hz[2:] = 0.0
    with pytest.raises(binding.DeconvError) as e:
        plan.run(y, mask, hz, lam, mu, 3)
    assert e.value.code == 3
    with pytest.raises(binding.DeconvError) as e:
        plan.backward(y, mask, h, lam, mu, torch.zeros_like(y))
    assert e.value.code == 5
    with pytest.raises(binding.DeconvError) as e:
        binding.Plan([dict(height=100, width=64, ksize=5)])
    assert e.value.code == 2
    with pytest.raises(binding.DeconvError) as e:
        binding.Plan([dict(height=64, width=64, ksize=4)])
    assert e.value.code == 2
    # no iterations, and continuing a plan that never ran
    with pytest.raises(binding.DeconvError) as e:
        plan.run(y, mask, h, lam, mu, 0)
    assert e.value.code == 1
    fresh = binding.Plan([desc(p)])
    with pytest.raises(binding.DeconvError) as e:
        fresh.cont(lam, mu, 3, torch.empty_like(y))
    with pytest.raises(binding.DeconvError):
        fresh.state_export(y.device)
    # the plan still runs normally after the refused calls
    x, st = plan.run(y, mask, h, lam, mu, 4, stats=True)
    torch.cuda.synchronize()
    assert st[0]["status"] == 0 and bool(torch.isfinite(x).all())


def test_autotuned_schedules_agree(tmp_path):
    """Both launch shapes (one launch per line length, one launch for all)
    give the same iterates; the autotuner records its choice in the cache and
    a second plan for the same batch reuses it."""
    from paper_1602_01410_amd import binding
    probs = _mixed(seed0=80)
    a = gpu_run(probs, 12, schedule=1)
    b = gpu_run(probs, 12, schedule=2)
    for i in range(len(probs)):
        assert rel_l2(a["x"][i], b["x"][i]) <= 1e-6
    assert a["plan"].schedule() == (1, 1) and b["plan"].schedule() == (2, 2)
    cache = str(tmp_path / "tune.txt")
    p1 = binding.Plan([desc(p) for p in probs], tune_cache=cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "\t" in lines[0]
    p2 = binding.Plan([desc(p) for p in probs], tune_cache=cache)
    assert p2.schedule() == p1.schedule()
    assert len(open(cache).read().splitlines()) == 1


def test_hybrid_schedule_agrees(torch_cuda):
    """The hybrid launch shape (short lengths share one launch, lengths with
    many tiles keep their own) gives the iterates of one launch per length."""
    probs = [_small(512, 512, 7, synth.MASK_BOUNDARY, seed=300 + b, blur="gauss") for b in range(8)]
    probs += [_small(64, 96, 5, synth.MASK_DECIMATE, seed=310), _small(96, 64, 9, synth.MASK_EXPLICIT, seed=311),
              _small(128, 128, 5, synth.MASK_BOUNDARY, seed=312)]
    a = gpu_run(probs, 12, schedule=1)
    c = gpu_run(probs, 12, schedule=3)
    assert c["plan"].schedule() == (3, 3)
    for i in range(len(probs)):
        assert rel_l2(c["x"][i], a["x"][i]) <= 1e-6, i
    r = oracle_run(probs[8], 12)
    assert_parity(c["x"][8], r["x"], what="hybrid small image x")


def test_long_lengths_one_launch(torch_cuda):
    """One launch for all lengths when some rows are longer than the short
    multi-length kernel covers (the general multi-length kernels, forward and
    reverse): iterates and gradients agree with one launch per length, and a
    small image agrees with the oracle."""
    import torch
    from paper_1602_01410_amd import binding
    probs = [_small(96, 384, 7, synth.MASK_BOUNDARY, seed=400), _small(64, 576, 5, synth.MASK_EXPLICIT, seed=401),
             _small(72, 96, 9, synth.MASK_DECIMATE, seed=402), _small(48, 1024, 3, synth.MASK_BOUNDARY, seed=403)]
    a = gpu_run(probs, 10, schedule=1)
    b = gpu_run(probs, 10, schedule=2)
    assert a["plan"].schedule() == (1, 1) and b["plan"].schedule() == (2, 2)
    for i in range(len(probs)):
        assert rel_l2(b["x"][i], a["x"][i]) <= 1e-6, i
    r = oracle_run(probs[2], 10)
    assert_parity(b["x"][2], r["x"], what="72x96 in a long multi-length launch")
    y, mask, h, lam, mu = device_inputs(probs)
    gx = torch.ones_like(y)
    grads = []
    for sch in (1, 2):
        pl = binding.Plan([desc(p) for p in probs], schedule=sch, ckpt_every=5, max_iters=10)
        pl.run(y, mask, h, lam, mu, 10)
        grads.append([t.cpu().numpy().astype(np.float64) for t in pl.backward(y, mask, h, lam, mu, gx)])
        torch.cuda.synchronize()
    for g1, g2 in zip(*grads):
        assert rel_l2(g2, g1) <= 1e-5


def test_spectra_cache_hint_leaves_results_unchanged(torch_cuda):
    """Ordinary and non-temporal stores of the pass-to-pass spectra give the
    same bits (the hint only changes where the lines live)."""
    probs = _mixed(seed0=600)
    a = gpu_run(probs, 15, spectra_hint=1, check_every=5)
    b = gpu_run(probs, 15, spectra_hint=2, check_every=5)
    for i in range(len(probs)):
        assert np.array_equal(a["x"][i], b["x"][i]), i
        assert np.array_equal(a["yt"][i], b["yt"][i]), i
