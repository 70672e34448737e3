"""Iteration parity with the FP64 oracle for the line lengths of the mixed
batch and the 2048-class workloads that no single-image test covers: row
passes of width 288, 384, 576, 768, 1152, 1536 and 1024 with the default
4-row tiles (no half tiles: the plans mix widths), column passes of height
288, 384, 576, 768, 1152 and 1024, under each launch shape (one launch per
length, one launch for all lengths, hybrid) and graph replay."""
import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

ITERS = 40


def _plan_a():
    """Four 1024^2 images (default row tiles of 4 rows), a decimated 768^2
    image, a 384 x 1536 image with 30% missing pixels."""
    ps = [synth.problem(1024, 1024, 13, "grf", "gauss", sigma=2.0, bsnr=50.0, lam=5e-4, mu=0.02, seed=801 + b)
          for b in range(4)]
    ps.append(synth.problem(768, 768, 9, "rect", "gauss", sigma=1.5, mask_kind=synth.MASK_DECIMATE, decim=4,
                            bsnr=40.0, lam=2e-3, mu=0.1, seed=805))
    ps.append(synth.problem(384, 1536, 11, "rect", "motion", mask_kind=synth.MASK_EXPLICIT, missing=0.3,
                            bsnr=45.0, lam=1e-3, mu=0.05, seed=806))
    return ps


def _plan_b():
    """Widths 1152, 576, 288 and heights 576, 1152, 288."""
    return [synth.problem(576, 1152, 15, "grf", "gauss", sigma=2.5, bsnr=45.0, lam=1e-3, mu=0.05, seed=811),
            synth.problem(1152, 576, 7, "rect", "box", mask_kind=synth.MASK_DECIMATE, decim=4, bsnr=35.0,
                          lam=3e-3, mu=0.15, seed=812),
            synth.problem(288, 288, 5, "rect", "gauss", sigma=1.0, mask_kind=synth.MASK_EXPLICIT, missing=0.5,
                          bsnr=40.0, lam=1e-3, mu=0.05, seed=813)]


_REF = {}


def _oracle(key, probs):
    if key not in _REF:
        _REF[key] = [oracle_run(p, ITERS) for p in probs]
    return _REF[key]


@pytest.mark.timeout(400)
@pytest.mark.parametrize("schedule", [1, 2, 3])
@pytest.mark.parametrize("which", ["a", "b"])
def test_lengths_vs_oracle(which, schedule):
    probs = _plan_a() if which == "a" else _plan_b()
    log("plan %s, schedule %d: %s" % (which, schedule, ", ".join("%dx%d" % (p["M"], p["N"]) for p in probs)))
    g = gpu_run(probs, ITERS, schedule=schedule, check_every=10, use_graph=1)
    assert g["plan"].schedule() == (schedule, schedule)
    ref = _oracle(which, probs)
    for b, (p, r) in enumerate(zip(probs, ref)):
        assert_parity(g["x"][b], r["x"], what="img%d %dx%d x" % (b, p["M"], p["N"]))
        assert_parity(g["yt"][b], r["yt"], what="img%d ytilde" % b)
        assert g["stats"][b]["status"] == 0
