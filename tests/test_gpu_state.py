"""The resumable state w = [z; v; d] (Appendix B) through the C ABI: a state
computed by the FP64 oracle and imported into a fresh plan continues like the
oracle, and an exported state imported into another plan continues bit for bit
like the plan it came from."""
import numpy as np
import pytest

import oracle
from paper_1602_01410_amd import synth

from .gpu_util import assert_parity, desc, device_inputs, explicit_mask, log

pytestmark = pytest.mark.gpu

CASES = {
    "boundary": dict(M=96, N=128, K=7, mask_kind=synth.MASK_BOUNDARY),
    "missing": dict(M=72, N=96, K=5, mask_kind=synth.MASK_EXPLICIT),
    # square and small: the plan runs the whole-image-in-LDS kernel
    "small": dict(M=64, N=64, K=5, mask_kind=synth.MASK_DECIMATE),
}


def _problem(c):
    return synth.problem(c["M"], c["N"], c["K"], "rect", "gauss", sigma=1.5, mask_kind=c["mask_kind"],
                         missing=0.4, bsnr=40.0, lam=2e-3, mu=0.05, seed=77)


def _interleave(a, b):
    return np.stack([a, b], -1).astype(np.float32).ravel()


@pytest.mark.parametrize("case", sorted(CASES))
def test_import_oracle_state_then_continue(case):
    import torch
    from paper_1602_01410_amd import binding
    p = _problem(CASES[case])
    n0, n1 = 15, 25
    log("import oracle state: %s %dx%d K=%d, %d + %d iterations" % (case, p["M"], p["N"], p["K"], n0, n1))
    y64, h64, m = p["y"].astype(np.float64), p["h"].astype(np.float64), explicit_mask(p)
    lam, mu = float(np.float32(p["lam"])), float(np.float32(p["mu"]))
    st = oracle.init_state(y64, m, p["K"])
    oracle.admm_iterate(st, h64, m, lam, mu, n0)
    yt0 = st["yt"].astype(np.float32).ravel()
    v0, d0 = _interleave(st["vh"], st["vv"]), _interleave(st["dh"], st["dv"])
    x_ref, _, _, _ = oracle.admm_iterate(st, h64, m, lam, mu, n1)
    plan = binding.Plan([desc(p)])
    assert plan.tiles()[3] == (1 if case == "small" else 0)
    y, mask, h, lamt, mut = device_inputs([p])
    dev = y.device
    imp_mask = mask if p["mask_kind"] == synth.MASK_EXPLICIT else None
    plan.state_import(imp_mask, h, *(torch.from_numpy(a).to(dev) for a in (yt0, v0, d0)))
    x = torch.empty_like(y)
    yt = torch.empty_like(y)
    plan.cont(lamt, mut, n1, x, ytilde_out=yt)
    torch.cuda.synchronize()
    sh = (p["M"], p["N"])
    assert_parity(x.cpu().numpy().astype(np.float64).reshape(sh), x_ref, what="x")
    assert_parity(yt.cpu().numpy().astype(np.float64).reshape(sh), st["yt"], what="ytilde")


@pytest.mark.parametrize("case", ["missing", "small"])
def test_export_import_roundtrip_bitwise(case):
    import torch
    from paper_1602_01410_amd import binding
    p = _problem(CASES[case])
    log("export/import round trip: %dx%d, 12 + 9 iterations" % (p["M"], p["N"]))
    y, mask, h, lam, mu = device_inputs([p])
    a = binding.Plan([desc(p)], check_every=5)
    xa = torch.empty_like(y)
    a.run(y, mask, h, lam, mu, 12, x_out=xa)
    yt, v, d = a.state_export(y.device)
    b = binding.Plan([desc(p)], check_every=5)
    assert a.tiles()[3] == (1 if case == "small" else 0)
    b.state_import(mask, h, yt.clone(), v.clone(), d.clone())
    xb = torch.empty_like(y)
    b.cont(lam, mu, 9, xb)
    a.cont(lam, mu, 9, xa)
    torch.cuda.synchronize()
    log("  max |xa - xb| = %.3e" % float((xa - xb).abs().max()))
    assert torch.equal(xa, xb)


def test_import_requires_mask_for_explicit_plans():
    import torch
    from paper_1602_01410_amd import binding
    p = _problem(CASES["missing"])
    y, mask, h, lam, mu = device_inputs([p])
    plan = binding.Plan([desc(p)])
    z = torch.zeros_like(y)
    z2 = torch.zeros(2 * y.numel(), dtype=torch.float32, device=y.device)
    with pytest.raises(binding.DeconvError):
        plan.state_import(None, h, z, z2, z2)
    with pytest.raises(binding.DeconvError):
        plan.cont(lam, mu, 3, torch.empty_like(y))
