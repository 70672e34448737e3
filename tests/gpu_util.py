"""Helpers shared by the GPU tests: move synthetic problems to the device,
run them through the C ABI, and run the same problems through the oracle."""
import sys

import numpy as np

import oracle
from paper_1602_01410_amd import synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def explicit_mask(p):
    """The full byte mask the oracle consumes (1 = observed)."""
    return p["mask"].astype(np.uint8)


def desc(p):
    kind = p["mask_kind"]
    return dict(height=p["M"], width=p["N"], ksize=p["K"], mask_kind=kind, decim=p.get("decim", 1))


def pack(problems, key, dtype=np.float32):
    return np.concatenate([np.asarray(p[key], dtype=dtype).reshape(-1) for p in problems])


def device_inputs(problems, device="cuda"):
    import torch
    y = torch.from_numpy(pack(problems, "y")).to(device)
    h = torch.from_numpy(pack(problems, "h")).to(device)
    mask = torch.from_numpy(pack(problems, "mask", np.uint8)).to(device)
    lam = torch.tensor([p["lam"] for p in problems], dtype=torch.float32, device=device)
    mu = torch.tensor([p["mu"] for p in problems], dtype=torch.float32, device=device)
    return y, mask, h, lam, mu


def gpu_run(problems, iters, want_state=False, **opts):
    import torch
    from paper_1602_01410_amd import binding
    plan = binding.Plan([desc(p) for p in problems], **opts)
    y, mask, h, lam, mu = device_inputs(problems)
    yt = torch.empty_like(y)
    x, st = plan.run(y, mask, h, lam, mu, iters, ytilde_out=yt, stats=True)
    torch.cuda.synchronize()
    out = dict(x=[a.cpu().numpy().astype(np.float64) for a in plan.split(x)],
               yt=[a.cpu().numpy().astype(np.float64) for a in plan.split(yt)], stats=st, plan=plan)
    if want_state:
        ytv, v, d = plan.state_export(y.device)
        torch.cuda.synchronize()
        out["v"] = [a.cpu().numpy().astype(np.float64) for a in plan.split(v, 2)]
        out["d"] = [a.cpu().numpy().astype(np.float64) for a in plan.split(d, 2)]
    return out


def oracle_run(p, iters, alpha=2.0):
    """The oracle on the same float32 inputs promoted to float64."""
    return oracle.admm_run(p["y"].astype(np.float64), explicit_mask(p), p["h"].astype(np.float64),
                           float(np.float32(p["lam"])), float(np.float32(p["mu"])), iters, alpha=alpha)


def rel_l2(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def assert_parity(x, ref, rel=1e-4, absfrac=1e-3, what=""):
    """The parity bar for an image after N iterations: relative L2 <= rel and
    max abs error <= absfrac of the reference's dynamic range."""
    r = rel_l2(x, ref)
    rng = float(ref.max() - ref.min())
    m = float(np.abs(x - ref).max())
    log("  %s rel_l2=%.3e max_abs=%.3e range=%.3e" % (what, r, m, rng))
    assert r <= rel, (what, r)
    assert m <= absfrac * max(rng, 1e-12), (what, m, rng)
