"""Pins of the colour (vectorial TV) oracle of Sec. III-C against what the
mathematics fixes: one channel is the scalar method; with lambda = 0 the
channels decouple; C equal channels behave as one channel with
lambda / sqrt(C)."""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth


def _scalar(y, mask, h, lam, mu, iters, **kw):
    return oracle.admm_run(y, mask, h, lam, mu, iters, **kw)


@pytest.fixture(scope="module")
def rgb():
    return synth.rgb_problem(40, 48, 9, seed=7, bsnr=40.0, lam=2e-3, mu=0.05)


def test_one_channel_is_the_scalar_method(rgb):
    p = rgb
    y, m, h = p["ys"][:1].astype(np.float64), p["masks"][:1], p["h"].astype(np.float64)
    for kw in (dict(), dict(passes=3), dict(adapt_t=3.0), dict(warm_iters=20, warm_tau=1e-3)):
        v = oracle.admm_run_vec(y, m, h, 2e-3, 0.05, 30, **kw)
        s = _scalar(y[0], m[0], h, 2e-3, 0.05, 30, **kw)
        for k in ("x", "yt", "vh", "dv"):
            assert np.abs(v[k][0] - s[k]).max() <= 1e-12 * max(1.0, np.abs(s[k]).max()), (kw, k)
        assert v["mu"] == s["mu"]


def test_lambda_zero_decouples_channels(rgb):
    p = rgb
    ys, ms, h = p["ys"].astype(np.float64), p["masks"], p["h"].astype(np.float64)
    v = oracle.admm_run_vec(ys, ms, h, 0.0, 0.05, 25, passes=2)
    for c in range(3):
        s = _scalar(ys[c], ms[c], h, 0.0, 0.05, 25, passes=2)
        assert np.abs(v["x"][c] - s["x"]).max() <= 1e-12, c
        assert np.abs(v["yt"][c] - s["yt"]).max() <= 1e-12, c


def test_equal_channels_scale_lambda(rgb):
    """|(u, u, u)| = sqrt(3) |u|: the joint threshold at tau acts on each copy
    as the scalar threshold at tau / sqrt(3)."""
    p = rgb
    y, m, h = p["ys"][1].astype(np.float64), p["masks"][1], p["h"].astype(np.float64)
    lam = 5e-3
    v = oracle.admm_run_vec(np.stack([y, y, y]), np.stack([m, m, m]), h, lam, 0.05, 40)
    s = _scalar(y, m, h, lam / np.sqrt(3.0), 0.05, 40)
    for c in range(3):
        assert np.abs(v["x"][c] - s["x"]).max() <= 1e-9 * np.abs(s["x"]).max(), c
    # and the coupling is real: a distinct threshold gives a distinct result
    s2 = _scalar(y, m, h, lam, 0.05, 40)
    assert np.abs(s2["x"] - s["x"]).max() > 1e-6


def test_bayer_masks_partition_the_valid_region():
    ms = synth.bayer_masks(20, 24, 9)
    valid = synth.make_mask(20, 24, 9).astype(bool)
    tot = ms.astype(int).sum(0)
    assert (tot[valid] == 1).all() and (tot[~valid] == 0).all()
    assert ms[1].sum() == 2 * ms[0].sum() == 2 * ms[2].sum()
    b = 4
    assert ms[0][b, b] == 1 and ms[1][b, b + 1] == 1 and ms[1][b + 1, b] == 1 and ms[2][b + 1, b + 1] == 1


def test_even_box_support():
    h = synth.box_kernel_even(8)
    assert h.shape == (9, 9) and abs(h.sum() - 1.0) < 1e-15
    assert (h[8, :] == 0).all() and (h[:, 8] == 0).all()
