#!/usr/bin/env python3
"""Throughput of the partial-ADMM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one deconv_admm_run over the workload (blur-spectrum setup, initial
state, all iterations with the FP64 residual checks), inputs resident in HBM.
Prints ONE JSON line on stdout; progress goes to stderr.

Default workload: one 1024 x 1024 image (GRF texture + rectangles), 19 x 19
Gaussian blur sigma 3, unknown boundaries (observed central 1006^2), BSNR 50
dB, lambda 5e-4, mu 0.02, 500 iterations.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s

# The paper's own timings (Sec. III-B, Tables I-IV): MATLAB on an Intel Core
# i7 3.2 GHz with 32 GB, FP64, 256^2 domain, one BGS pass per iteration; a
# least-squares line through the twelve Proposed-1 rows gives about 8.48 ms
# per iteration after a fixed start-up cost.
PAPER_CONTEXT = {"mpx_it_s": 7.7, "ms_per_iter_256x256": 8.48, "workload": "256^2, Proposed-1, Tables I-IV",
                 "hardware": "Intel Core i7 3.2 GHz, 32 GB, MATLAB (FP64)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1602_01410_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def workload(name):
    from paper_1602_01410_amd import synth
    if name == "large_1024":
        p = synth.config_large_1024()
        return [p], p["iters"], "1x1024^2 GRF+rects, 19x19 Gaussian s=3, unknown boundaries, 500 it"
    if name == "plain_72":
        p = synth.config_plain_72()
        return [p], p["iters"], "1x72^2 rects+ramp, 9x9 box, unknown boundaries, 200 it"
    if name == "inpaint_2048":
        p = synth.config_inpaint_2048()
        return [p], p["iters"], "1x2048^2, 21x21 motion blur, boundaries + 50% missing, 300 it"
    if name == "batch_256":
        ps = synth.config_batch()
        return ps, 200, "256 mixed images 128..1024, Gaussian blurs, half x4 decimated, 200 it"
    if name == "uniform_16x1024":
        ps = [synth.problem(1024, 1024, 19, "grf", "gauss", sigma=3.0, bsnr=50.0, lam=5e-4, mu=0.02,
                            seed=synth.BASE_SEED * 1000 + 500 + b) for b in range(16)]
        return ps, 500, "16x1024^2 GRF+rects, 19x19 Gaussian s=3, unknown boundaries, 500 it"
    if name == "grad_512":
        ps = synth.config_grad_512()
        return ps, ps[0]["iters"], \
            "16x512^2 rects+ramp, 15x15 Gaussian s=2, unknown boundaries, 50 it forward + reverse (checkpoint every 10)"
    if name == "demosaic_288x256":
        return colour_channels(synth.config_demosaic()), 200, \
            "RGB 288x256 (valid 280x248), 8x8 box, Bayer masks, vectorial TV, 4 BGS passes, adaptive mu, 200 it"
    raise ValueError(name)


def colour_channels(p):
    """The channels of a colour problem as consecutive grey images of one
    plan (opt.channels = 3)."""
    from paper_1602_01410_amd import synth
    out = []
    for c in range(3):
        out.append(dict(y=p["ys"][c], mask=p["masks"][c], h=p["h"], lam=p["lam"], mu=p["mu"], M=p["M"], N=p["N"],
                        K=p["K"], mask_kind=synth.MASK_EXPLICIT, decim=1, colour=p))
    return out


def plan_options(name):
    """Options of the method each workload runs with (beyond the defaults)."""
    if name == "demosaic_288x256":
        return dict(channels=3, bgs_passes=4, adapt_t=3.0)
    if name == "grad_512":
        return dict(ckpt_every=10, max_iters=50)
    return {}


def descs(problems):
    return [dict(height=p["M"], width=p["N"], ksize=p["K"], mask_kind=p["mask_kind"], decim=p.get("decim", 1))
            for p in problems]


def to_device(problems):
    import numpy as np
    import torch
    cat = lambda k, dt: torch.from_numpy(np.concatenate([np.asarray(p[k], dt).ravel() for p in problems])).cuda()
    y = cat("y", np.float32)
    h = cat("h", np.float32)
    mask = cat("mask", np.uint8)
    lam = torch.tensor([p["lam"] for p in problems], dtype=torch.float32, device="cuda")
    mu = torch.tensor([p["mu"] for p in problems], dtype=torch.float32, device="cuda")
    return y, mask, h, lam, mu


def unobserved_fraction(problems):
    import numpy as np
    n = sum(p["M"] * p["N"] for p in problems)
    k = sum(int(np.count_nonzero(p["mask"])) for p in problems)
    return (n - k) / n


def alg_bytes(problems, unobs):
    """Algorithmic bytes per launch of each pass (compulsory reads + writes of
    its own inputs and outputs, each once; halo re-reads excluded).
    row pass  per pixel: spectra in 16*nh/n' + ytilde 4 + d in 8 + d out 8
              + spectra out 16*nh/n' + z out 4*(unobserved fraction)
    col pass  per half-spectrum element: spectra in 16 + blur spectrum 8 + spectra out 16"""
    row = col = 0.0
    for p in problems:
        M, N = p["M"], p["N"]
        nh = N // 2 + 1
        row += M * nh * 32.0 + M * N * 20.0
        col += M * nh * 40.0
    row += 4.0 * unobs * sum(p["M"] * p["N"] for p in problems)
    return row, col


def bwd_alg_bytes(problems):
    """Modelled bytes per launch of the reverse passes (each input and output
    once; halo re-reads excluded).
    reverse row pass  per pixel: spectra in and out 32*nh/n' + ub in 8 + u 8
                      + y-bar or z-bar read 4 and write 4 + ub out 8
    reverse col pass  per half-spectrum element: spectra in 16 + blur spectrum
                      8 + stored (Y, X) 16 + FP64 blur-gradient sum read and
                      written 32 + spectra out 16"""
    row = col = 0.0
    for p in problems:
        M, N = p["M"], p["N"]
        nh = N // 2 + 1
        row += M * nh * 32.0 + M * N * 32.0
        col += M * nh * 88.0
    return row, col


def reverse_roofline(problems, inputs, iters, opts):
    """Per-launch time and modelled bytes of the reverse row and column
    passes (HIP events on the plan's stream; the reverse pass runs outside
    graphs when profiled)."""
    import torch
    from paper_1602_01410_amd import binding
    pplan = binding.Plan(descs(problems), batched=1, use_graph=0, profile=1, **opts)
    y, mask, h, lam, mu = inputs
    g = torch.Generator(device="cpu").manual_seed(7)
    gx = (torch.randn(pplan.npx, generator=g) / pplan.npx).cuda()
    pplan.run(y, mask, h, lam, mu, iters)
    pplan.backward(y, mask, h, lam, mu, gx)
    pplan.kernel_times()
    pplan.bwd_kernel_times()
    pplan.run(y, mask, h, lam, mu, iters)
    pplan.backward(y, mask, h, lam, mu, gx)
    brow_ms, brow_n, bcol_ms, bcol_n = pplan.bwd_kernel_times()
    pplan.close()
    rb, cb = bwd_alg_bytes(problems)
    ra, ca = brow_ms / max(brow_n, 1), bcol_ms / max(bcol_n, 1)
    log("reverse row pass %.2f us x %d, reverse column pass %.2f us x %d" % (ra * 1e3, brow_n, ca * 1e3, bcol_n))
    return {"bound": "hbm", "kernel": "bwd_row_kernel", "launch_us": round(ra * 1e3, 2),
            "alg_bytes_per_launch": int(rb), "achieved": round(rb / (ra * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(rb / (ra * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "other_pass": {"kernel": "bwd_col_kernel", "launch_us": round(ca * 1e3, 2),
                           "alg_bytes_per_launch": int(cb), "achieved": round(cb / (ca * 1e-3) / 1e9, 1)}}


def method_bytes_per_iter(problems, unobs):
    """Algorithmic bytes of one iteration of the method itself (what it must
    read and write, independent of how the transforms are organised):
    A = 44 + 4 d/N per pixel: read ytilde 4, v 8, d 8, the blur spectrum 8
    (complex64); write v 8, d 8, z 4 on the unobserved pixels."""
    npx = sum(p["M"] * p["N"] for p in problems)
    return (44.0 + 4.0 * unobs) * npx


def read_traffic(name):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % name)
    if not os.path.exists(path):
        return None, None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("src_hash") != src_hash():
        return None, kv.get("kernel")
    try:
        return float(kv["bytes_per_launch"]), kv.get("kernel")
    except (KeyError, ValueError):
        return None, None


def copy_bandwidth(mib=1024, reps=5):
    """GB/s of a plain device-to-device copy of `mib` MiB (read + write
    counted), best of `reps`, timed with events on the current stream."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / best / 1e9


def pass_roofline(problems, inputs, iters, check_every, unobs, name):
    """Per-launch GPU time of each pass (HIP events attached to the
    dispatches, on the plan's stream) and the modelled bytes per launch: the
    roofline object of the heavier pass, the other pass as a sub-object."""
    from paper_1602_01410_amd import binding
    pplan = binding.Plan(descs(problems), batched=1, use_graph=0, check_every=check_every, profile=1)
    y, mask, h, lam, mu = inputs
    pplan.run(y, mask, h, lam, mu, min(iters, 50))
    pplan.kernel_times()
    pplan.run(y, mask, h, lam, mu, iters)
    row_ms, row_n, col_ms, col_n = pplan.kernel_times()
    small = pplan.tiles()[3] == 1
    pplan.close()
    if small:
        # whole-image-in-LDS path: one launch reads and writes the state once
        # (ytilde 4, v 8, d 8 each way per pixel) and reads the blur half
        # spectrum (8 per entry); x (4) on the last
        avg = row_ms / max(row_n, 1)
        ab = sum(40.0 * p["M"] * p["N"] + 8.0 * p["M"] * (p["N"] // 2 + 1) for p in problems)
        log("whole-image-in-LDS launch %.2f us x %d" % (avg * 1e3, row_n))
        return {"bound": "hbm", "achieved": round(ab / (avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ab / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None, "traffic_frac": None,
                "kernel": "small_kernel", "launch_us": round(avg * 1e3, 2), "alg_bytes_per_launch": int(ab),
                "iters_per_launch": round(iters / max(row_n, 1), 1),
                "note": "the image stays in LDS for a whole launch (up to 200 iterations, a check every "
                        "check_every); one compute unit's VALU and LDS, not HBM, bound this path"}
    rb, cb = alg_bytes(problems, unobs)
    row_avg, col_avg = row_ms / max(row_n, 1), col_ms / max(col_n, 1)
    log("row pass %.2f us x %d, column pass %.2f us x %d" % (row_avg * 1e3, row_n, col_avg * 1e3, col_n))
    # the dominant kernel is the row pass; its algorithmic bytes per launch
    # are the method's A = 44 + 4 d/N per pixel-iteration times the pixels
    # one launch processes (one iteration of the whole batch)
    ab = method_bytes_per_iter(problems, unobs)
    achieved = ab / (row_avg * 1e-3) / 1e9
    traffic, tk = read_traffic(name)
    traffic = traffic if (traffic is not None and tk == "row_kernel") else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # measured bytes (counter traffic) over the same launch time
            "traffic_frac": round(traffic / (row_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "kernel": "row_kernel", "launch_us": round(row_avg * 1e3, 2), "alg_bytes_per_launch": int(ab),
            # the row pass's own inputs and outputs (spectra in and out, state)
            "pass_model": {"alg_bytes_per_launch": int(rb), "achieved": round(rb / (row_avg * 1e-3) / 1e9, 1),
                           "frac": round(rb / (row_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "other_pass": {"kernel": "col_kernel", "launch_us": round(col_avg * 1e3, 2),
                           "alg_bytes_per_launch": int(cb), "achieved": round(cb / (col_avg * 1e-3) / 1e9, 1)}}


def time_runs(plan, inputs, iters, steps, warmup, backward=False):
    """Seconds for `steps` runs (each: setup, init, all iterations; with
    backward also the reverse pass for a fixed dL/dx), and the wall time."""
    import torch
    y, mask, h, lam, mu = inputs
    x = torch.empty(plan.npx, dtype=torch.float32, device="cuda")
    gx = None
    if backward:
        g = torch.Generator(device="cpu").manual_seed(7)
        gx = (torch.randn(plan.npx, generator=g) / plan.npx).cuda()

    def step():
        plan.run(y, mask, h, lam, mu, iters, x_out=x)
        if backward:
            plan.backward(y, mask, h, lam, mu, gx)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s = plan.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(s)
    for k in range(steps):
        step()
        ev[k + 1].record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = [ev[k].elapsed_time(ev[k + 1]) / 1e3 for k in range(steps)]
    time_runs.per_step = per_step
    return ev[0].elapsed_time(ev[steps]) / 1e3, wall


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baselines(problems, opts=None):
    """The oracle on every host thread it is given (~12 s of work) and on
    one thread (~8 s), with the CPU model."""
    import oracle
    nthreads = oracle.num_threads()
    allc = cpu_baseline(problems, target_s=12.0, opts=opts)
    oracle.set_threads(1)
    try:
        one = cpu_baseline(problems, target_s=8.0, opts=opts)
    finally:
        oracle.set_threads(nthreads)
    allc["value"] = round(allc["value"], 4)
    allc["cpu_model"] = cpu_model()
    allc["single_thread"] = {"value": round(one["value"], 4), "cores": 1, "sample": one["sample"]}
    return allc


def cpu_baseline(problems, target_s=15.0, opts=None):
    """The FP64 oracle on the host cores, on a bounded sample of the
    workload: the first image, as many iterations as fit in ~target_s."""
    import numpy as np
    import oracle
    p = problems[0]
    if "colour" in p:
        c = p["colour"]
        args = (c["ys"].astype(np.float64), c["masks"], c["h"].astype(np.float64), float(c["lam"]), float(c["mu"]))
        kw = dict(passes=opts.get("bgs_passes", 1), adapt_t=opts.get("adapt_t", 0.0))
        t0 = time.perf_counter()
        oracle.admm_run_vec(*args, 2, **kw)
        t2 = time.perf_counter() - t0
        n = int(max(2, min(200, target_s / max(t2 / 2.0, 1e-6))))
        t0 = time.perf_counter()
        oracle.admm_run_vec(*args, n, **kw)
        t = time.perf_counter() - t0
        return dict(value=3 * c["M"] * c["N"] * n / t / 1e6, unit="Mpixel*ADMM-iters/s", cores=oracle.num_threads(),
                    kind="oracle", sample="colour image (3x%dx%d), %d iterations incl. setup, %.1f s" %
                    (c["M"], c["N"], n, t))
    args = (p["y"].astype(np.float64), p["mask"], p["h"].astype(np.float64), float(p["lam"]), float(p["mu"]))
    if opts and opts.get("ckpt_every"):
        # forward + reverse, as the GPU step
        gx = np.random.default_rng(7).standard_normal((p["M"], p["N"])) / (p["M"] * p["N"])
        run = lambda n: oracle.admm_backward(args[0], args[1].astype(np.uint8), args[2], args[3], args[4], n, gx)
        what = "forward + reverse"
    else:
        run = lambda n: oracle.admm_run(*args, n)
        what = "incl. setup"
    t0 = time.perf_counter()
    run(2)
    t2 = time.perf_counter() - t0
    n = int(max(2, min(200, target_s / max(t2 / 2.0, 1e-6))))
    t0 = time.perf_counter()
    run(n)
    t = time.perf_counter() - t0
    return dict(value=p["M"] * p["N"] * n / t / 1e6, unit="Mpixel*ADMM-iters/s", cores=oracle.num_threads(),
                kind="oracle", sample="image 0 (%dx%d), %d iterations %s, %.1f s" % (p["M"], p["N"], n, what, t))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_1024",
                    choices=["large_1024", "plain_72", "inpaint_2048", "batch_256", "uniform_16x1024",
                             "demosaic_288x256", "grad_512"])
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-compare", action="store_true")
    ap.add_argument("--no-uniform", action="store_true", help="skip the 16 x 1024^2 figure of the default line")
    ap.add_argument("--no-kernel-times", action="store_true")
    ap.add_argument("--iters", type=int, default=0, help="override the workload's iteration count")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1); %d requested" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1602_01410_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the kernel traffic figures
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4}), flush=True)
        return

    log("generating workload %s" % args.workload)
    problems, iters, wdesc = workload(args.workload)
    if args.iters:
        iters = args.iters
    npx = sum(p["M"] * p["N"] for p in problems)
    unobs = unobserved_fraction(problems)
    inputs = to_device(problems)
    popts = plan_options(args.workload)
    plan = binding.Plan(descs(problems), batched=1, use_graph=1, check_every=args.check_every, **popts)
    log("launch shapes (row, column; 1 = per length, 2 = one launch, 3 = hybrid): %s, tiles %s"
        % (plan.schedule(), plan.tiles()))
    log("timing %d steps (+%d warmup), %d images, %d px, %d iterations" % (args.steps, args.warmup,
                                                                          len(problems), npx, iters))
    grad = args.workload == "grad_512"
    t, wall = time_runs(plan, inputs, iters, args.steps, args.warmup, backward=grad)
    per_step = list(time_runs.per_step)
    value = npx * iters * args.steps / t / 1e6
    ms_step = t / args.steps * 1e3
    log("value %.1f Mpx*it/s, %.3f ms/step (wall %.3f s)" % (value, ms_step, wall))
    extra = {}
    if grad:
        tf, _ = time_runs(plan, inputs, iters, args.steps, 1)
        extra["forward_only_ms_per_step"] = round(tf / args.steps * 1e3, 4)
        extra["reverse_ms_per_step"] = round((t - tf) / args.steps * 1e3, 4)
        log("forward %.3f ms, reverse %.3f ms per step" % (tf / args.steps * 1e3, (t - tf) / args.steps * 1e3))
        if not args.no_kernel_times:
            extra["reverse_roofline"] = reverse_roofline(problems, inputs, iters, popts)

    roof = None
    # the byte model below is that of one pass per iteration (plain method)
    if not args.no_kernel_times and not popts:
        roof = pass_roofline(problems, inputs, iters, args.check_every, unobs, args.workload)
        roof["copy_gbs"] = round(copy_bandwidth(), 1)
        a_iter = method_bytes_per_iter(problems, unobs)
        rb, cb = alg_bytes(problems, unobs)
        # the method's own bytes (A per pixel-iteration) over the timed steps
        roof["frac_A"] = round(a_iter * iters * args.steps / t / 1e9 / HBM_PEAK_GBS, 4)
        roof["method_bytes_per_iter"] = int(a_iter)
        # both passes' modelled bytes over the whole iteration (timed steps)
        roof["frac_iter"] = round((rb + cb) * iters * args.steps / t / 1e9 / HBM_PEAK_GBS, 4)

    if args.workload == "large_1024" and not args.no_batch_compare:
        log("batched vs plain on the 256-image mixed batch")
        bp, bit, _ = workload("batch_256")
        bnpx = sum(p["M"] * p["N"] for p in bp)
        binp = to_device(bp)
        res = {}
        for mode, kw in (("batched_graph", dict(batched=1, use_graph=1)),
                         ("plain", dict(batched=0, use_graph=0)),
                         ("plain_graph", dict(batched=0, use_graph=1))):
            pl = binding.Plan(descs(bp), check_every=args.check_every, **kw)
            tt, _ = time_runs(pl, binp, bit, 3, 1)
            res[mode] = bnpx * bit * 3 / tt / 1e6
            log("  %s: %.1f Mpx*it/s (launch shapes %s)" % (mode, res[mode], pl.schedule()))
            pl.close()
            torch.cuda.empty_cache()
        extra["batch_256"] = {"mpx_it_s": {k: round(v, 1) for k, v in res.items()},
                              "batched_over_plain": round(res["batched_graph"] / res["plain"], 2),
                              "steps_per_mode": 3}
        del binp
        torch.cuda.empty_cache()

    if args.workload == "large_1024" and not args.no_uniform:
        # 16 images of the same recipe: a working set (about 0.8 GB) far beyond
        # the last-level cache, so this figure is HBM-bound, not cache-bound
        log("16 x 1024^2 (working set beyond the last-level cache)")
        up, uit, _ = workload("uniform_16x1024")
        unpx = sum(p["M"] * p["N"] for p in up)
        uunobs = unobserved_fraction(up)
        uinp = to_device(up)
        pl = binding.Plan(descs(up), batched=1, use_graph=1, check_every=args.check_every)
        tt, _ = time_runs(pl, uinp, uit, 3, 1)
        pl.close()
        ur = pass_roofline(up, uinp, uit, args.check_every, uunobs, "uniform_16x1024")
        ur["frac_A"] = round(method_bytes_per_iter(up, uunobs) * uit * 3 / tt / 1e9 / HBM_PEAK_GBS, 4)
        extra["uniform_16x1024"] = {"mpx_it_s": round(unpx * uit * 3 / tt / 1e6, 1),
                                    "ms_per_step": round(tt / 3 * 1e3, 3), "iters": uit, "roofline": ur}
        log("  %.1f Mpx*it/s" % extra["uniform_16x1024"]["mpx_it_s"])
        del uinp
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        cpu = cpu_baselines(problems, opts=popts)
        log("  %s" % cpu)

    out = {"metric": "Mpixel*ADMM-iters/s", "value": round(value, 2), "unit": "Mpixel*ADMM-iters/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": args.workload, "description": wdesc, "images": len(problems), "pixels": npx,
                      "iters": iters, "check_every": args.check_every, "unobserved_fraction": round(unobs, 4),
                      "options": popts},
           "roofline": roof, "cpu_baseline": cpu,
           "median_ms_per_step": round(1e3 * sorted(per_step)[len(per_step) // 2], 4),
           # the paper's own timings, for context (another machine, FP64)
           "paper_context": PAPER_CONTEXT}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
