"""The autotuner's tile knobs: row tiles of the default or half height, 512
or 1024 threads per half-height row tile, 256 or 512 threads per long column
tile.  Every forced combination meets the oracle bar on every image (the
combinations are different instantiations of the passes, so their rounding
may differ in the last bits), the autotuned plan reports one of them, and a
tune cache written by one plan is read back by the next."""
import itertools

import numpy as np
import pytest

from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, desc, device_inputs, log, oracle_run

pytestmark = pytest.mark.gpu


def _run(probs, iters, **opts):
    import torch
    from paper_1602_01410_amd import binding
    plan = binding.Plan([desc(p) for p in probs], check_every=10, **opts)
    y, mask, h, lam, mu = device_inputs(probs)
    yt = torch.empty_like(y)
    x, st = plan.run(y, mask, h, lam, mu, iters, ytilde_out=yt, stats=True)
    torch.cuda.synchronize()
    return plan, x.cpu(), yt.cpu(), st


CASES = {
    "one_1024": lambda: [synth.problem(1024, 1024, 11, "grf", "gauss", sigma=2.0, bsnr=50.0, lam=5e-4, mu=0.02,
                                       seed=931)],
    "four_512": lambda: [synth.problem(512, 512, 9, "rect", "gauss", sigma=1.5, mask_kind=synth.MASK_DECIMATE,
                                       decim=4, bsnr=40.0, lam=2e-3, mu=0.1, seed=932 + b) for b in range(4)],
    "mixed": lambda: [synth.problem(768, 512, 7, "rect", "box", bsnr=40.0, lam=1e-3, mu=0.05, seed=936),
                      synth.problem(512, 768, 9, "rect", "gauss", sigma=1.5, mask_kind=synth.MASK_EXPLICIT,
                                    missing=0.3, bsnr=45.0, lam=1e-3, mu=0.05, seed=937)],
}


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", sorted(CASES))
def test_tile_knobs_do_not_change_results(case):
    probs = CASES[case]()
    iters = 30
    refs = [oracle_run(p, iters) for p in probs]
    sizes = [p["M"] * p["N"] for p in probs]
    offs = np.cumsum([0] + sizes)

    def check(x, what):
        for b, (p, r) in enumerate(zip(probs, refs)):
            xb = x[offs[b]:offs[b + 1]].numpy().astype(np.float64).reshape(r["x"].shape)
            assert_parity(xb, r["x"], what="%s img%d x" % (what, b))

    plan, x0, yt0, st0 = _run(probs, iters)
    log("%s: autotuned shapes %s, tiles %s" % (case, plan.schedule(), plan.tiles()))
    rt, wr, wc = plan.tiles()[:3]
    assert rt in (1, 2) and wr in (512, 1024) and wc in (256, 512)
    check(x0, "autotuned")
    for row_tiles, row_threads, col_threads in itertools.product((1, 2), (512, 1024), (256, 512)):
        if row_tiles == 1 and row_threads == 1024:
            continue
        p2, x, yt, st = _run(probs, iters, schedule=3, row_tiles=row_tiles, row_threads=row_threads,
                             col_threads=col_threads)
        got = p2.tiles()[:3]
        log("  forced %s -> tiles %s, max |x - x_autotuned| %.2e" % ((row_tiles, row_threads, col_threads), got,
                                                                   float((x - x0).abs().max())))
        if len({p["N"] for p in probs}) == 1:
            assert got[0] == row_tiles and got[2] == col_threads
            assert row_tiles == 1 or got[1] == row_threads
        check(x, "forced %s" % ((row_tiles, row_threads, col_threads),))
        assert [s["iters_done"] for s in st] == [s["iters_done"] for s in st0]


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def test_tune_cache_round_trip(tmp_path):
    probs = CASES["four_512"]()
    cache = str(tmp_path / "tune.txt")
    p1, x1, _, _ = _run(probs, 12, tune_cache=cache)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and len(lines[0].split("\t")[1].split()) == 5, lines
    p2, x2, _, _ = _run(probs, 12, tune_cache=cache)
    assert open(cache).read().strip().splitlines() == lines   # read, not tuned again
    assert p2.schedule() == p1.schedule() and p2.tiles() == p1.tiles()
    assert torch_equal(x1, x2)   # the same choices: the same instantiations
