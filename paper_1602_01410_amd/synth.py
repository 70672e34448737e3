"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the deconvolution method itself: it makes
sharp images, blur kernels, masks and noisy observations, which both the HIP
path and the CPU oracle consume.  The observation follows the paper's recipe
(Sec. III): circular convolution of the sharp m' x n' image, keep the part
that equals the linear convolution (the central m x n region), add i.i.d.
Gaussian noise at a given blurred-signal-to-noise ratio.

Every random draw comes from numpy's PCG64 with an explicit seed.  Values are
generated in float64 and rounded once to float32, so both consumers see
identical numbers (the oracle promotes them back to float64).

Readings of the paper's underspecified parts used here:
* BSNR: noise variance = population variance of the observed blurred pixels
  / 10^(BSNR/10).
* "normalised to [0, 1]": the sharp image is affinely mapped to [0, 1] before
  blurring (blurs are non-negative with unit sum).
* Gaussian blur with support l x l: standard deviation sqrt(l) for the
  paper's tables; the workloads below state their own sigma.
"""
import numpy as np
from scipy.signal import fftconvolve

MASK_BOUNDARY, MASK_EXPLICIT, MASK_DECIMATE = 0, 1, 2


# --------------------------------------------------------------------------
# blur kernels
# --------------------------------------------------------------------------

def box_kernel(size):
    return np.full((size, size), 1.0 / (size * size))


def gaussian_kernel(size, sigma):
    b = size // 2
    t = np.arange(-b, b + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def motion_kernel(size, steps, rng):
    """Visit counts of an 8-neighbour random walk from the centre, clamped to
    the support, normalised to unit sum."""
    h = np.zeros((size, size))
    i = j = size // 2
    h[i, j] += 1
    moves = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
    for _ in range(steps):
        di, dj = moves[rng.integers(8)]
        i = min(max(i + di, 0), size - 1)
        j = min(max(j + dj, 0), size - 1)
        h[i, j] += 1
    return h / h.sum()


# --------------------------------------------------------------------------
# sharp images
# --------------------------------------------------------------------------

def _normalise(x):
    lo, hi = x.min(), x.max()
    return (x - lo) / (hi - lo) if hi > lo else np.zeros_like(x)


def rect_image(M, N, rng, nrect=12, ramp=0.2, ramp_width=None):
    """Piecewise-smooth image: `nrect` axis-aligned rectangles with U(0,1)
    intensities painted in order over a zero background, plus a horizontal
    ramp ramp*col/ramp_width; normalised to [0, 1]."""
    x = np.zeros((M, N))
    for _ in range(nrect):
        r0, r1 = np.sort(rng.integers(0, M + 1, size=2))
        c0, c1 = np.sort(rng.integers(0, N + 1, size=2))
        x[r0:r1, c0:c1] = rng.uniform(0.0, 1.0)
    w = ramp_width if ramp_width else max(N - 8, 1)
    x += ramp * np.arange(N)[None, :] / float(w)
    return _normalise(x)


def grf_image(M, N, rng, nrect=40):
    """Gaussian-random-field texture with a 1/f^2 power spectrum, plus
    rectangles, normalised to [0, 1]."""
    w = rng.standard_normal((M, N))
    fy = np.fft.fftfreq(M)[:, None]
    fx = np.fft.fftfreq(N)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    amp = np.zeros_like(f)
    amp[f > 0] = 1.0 / f[f > 0]
    x = _normalise(np.real(np.fft.ifft2(np.fft.fft2(w) * amp)))
    for _ in range(nrect):
        r0, r1 = np.sort(rng.integers(0, M + 1, size=2))
        c0, c1 = np.sort(rng.integers(0, N + 1, size=2))
        x[r0:r1, c0:c1] = rng.uniform(0.0, 1.0)
    return _normalise(x)


# --------------------------------------------------------------------------
# masks and observations
# --------------------------------------------------------------------------

def valid_region(M, N, K):
    b = K // 2
    m = np.zeros((M, N), dtype=bool)
    m[b:M - b, b:N - b] = True
    return m


def make_mask(M, N, K, kind=MASK_BOUNDARY, decim=1, missing=0.0, rng=None):
    """Observed-pixel mask (uint8, 1 = observed) on the extended grid.
    The band of width b = K//2 is always unobserved.  EXPLICIT: i.i.d.
    Bernoulli(missing) holes inside the central region.  DECIMATE: only
    pixels (b + s*i, b + s*j) of the central region are observed."""
    b = K // 2
    m = valid_region(M, N, K)
    if kind == MASK_EXPLICIT:
        m &= rng.uniform(size=(M, N)) >= missing
    elif kind == MASK_DECIMATE:
        ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
        m &= ((ii - b) % decim == 0) & ((jj - b) % decim == 0)
    return m.astype(np.uint8)


def observe(x_true, h, mask, bsnr, rng):
    """Blur (valid part of the linear convolution == central part of the
    circular one), add noise at `bsnr` dB over the observed pixels.  Returns y
    on the extended M x N grid, zero at unobserved pixels."""
    M, N = x_true.shape
    b = h.shape[0] // 2
    blurred = fftconvolve(x_true, h, mode="valid")
    yb = np.zeros((M, N))
    yb[b:M - b, b:N - b] = blurred
    obs = mask.astype(bool)
    var = yb[obs].var() / (10.0 ** (bsnr / 10.0))
    y = yb + rng.standard_normal((M, N)) * np.sqrt(var)
    y[~obs] = 0.0
    return y


def f32(a):
    return np.asarray(a, dtype=np.float32)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

BASE_SEED = 20160203


def problem(M, N, K, kind="rect", blur="box", sigma=None, mask_kind=MASK_BOUNDARY, decim=4,
            missing=0.5, bsnr=50.0, lam=1e-3, mu=0.05, seed=0, nrect=None, ramp_width=None):
    """One synthetic problem.  All arrays float32 (mask uint8)."""
    rng = np.random.default_rng(seed)
    if kind == "grf":
        x = grf_image(M, N, rng, nrect=nrect or 40)
    else:
        x = rect_image(M, N, rng, nrect=nrect or 12, ramp_width=ramp_width)
    if blur == "box":
        h = box_kernel(K)
    elif blur == "gauss":
        h = gaussian_kernel(K, sigma if sigma else np.sqrt(K))
    elif blur == "motion":
        h = motion_kernel(K, 60, rng)
    elif blur == "random":
        h = rng.uniform(0.0, 1.0, size=(K, K))
        h /= h.sum()
    else:
        raise ValueError(blur)
    mask = make_mask(M, N, K, mask_kind, decim, missing, rng)
    y = observe(x, h, mask, bsnr, rng)
    return dict(x_true=f32(x), h=f32(h), mask=mask, y=f32(y), lam=float(lam), mu=float(mu),
                K=K, M=M, N=N, mask_kind=mask_kind, decim=decim if mask_kind == MASK_DECIMATE else 1)


def box_kernel_even(size):
    """A size x size box (size even) on the odd (size+1)^2 support the method
    needs: the box covers offsets -size/2 .. size/2-1 around the centre,
    i.e. its anchor is the pixel (size/2, size/2) of the box."""
    h = np.zeros((size + 1, size + 1))
    h[:size, :size] = 1.0 / (size * size)
    return h


def bayer_masks(M, N, K):
    """RGGB colour-filter masks (3, M, N) over the valid region, phase at its
    top-left corner: red at (even, even) offsets, green at (even, odd) and
    (odd, even), blue at (odd, odd); the band of width b is unobserved."""
    b = K // 2
    ii, jj = np.meshgrid(np.arange(M) - b, np.arange(N) - b, indexing="ij")
    valid = make_mask(M, N, K).astype(bool)
    red = (ii % 2 == 0) & (jj % 2 == 0)
    blue = (ii % 2 == 1) & (jj % 2 == 1)
    green = ~red & ~blue
    return np.stack([red & valid, green & valid, blue & valid]).astype(np.uint8)


def rgb_problem(M, N, K=9, seed=0, bsnr=40.0, lam=1e-5, mu=1e-3, nrect=16):
    """Colour deblurring + demosaicing (Sec. III-C): rectangles with
    per-channel intensities (edges shared by the channels) plus a ramp,
    jointly normalised to [0, 1]; an 8x8 box blur on a 9x9 support (K = 9);
    Bayer masks; noise at `bsnr` dB per channel over its observed pixels."""
    rng = np.random.default_rng(seed)
    x = np.zeros((3, M, N))
    for _ in range(nrect):
        r0, r1 = np.sort(rng.integers(0, M + 1, size=2))
        c0, c1 = np.sort(rng.integers(0, N + 1, size=2))
        x[:, r0:r1, c0:c1] = rng.uniform(0.0, 1.0, size=3)[:, None, None]
    x += 0.2 * (np.arange(N)[None, None, :] / float(max(N - 8, 1))) * rng.uniform(0.5, 1.0, size=3)[:, None, None]
    x = (x - x.min()) / (x.max() - x.min())
    h = box_kernel_even(K - 1) if K % 2 == 1 else box_kernel_even(K)
    K = h.shape[0]
    masks = bayer_masks(M, N, K)
    ys = np.stack([observe(x[c], h, masks[c], bsnr, rng) for c in range(3)])
    return dict(x_true=f32(x), h=f32(h), masks=masks, ys=f32(ys), lam=float(lam), mu=float(mu), K=K, M=M, N=N)


def config_demosaic(seed=BASE_SEED + 5):
    """288 x 256 extended domain (valid 280 x 248, the size of the paper's
    289 x 253 crop rounded to FFT-friendly lengths), 8x8 box, Bayer masks,
    BSNR 40 dB, lambda 1e-4, mu 1e-3 adapted with t = 3, 4 BGS passes.
    (The paper's lambda = 1e-5 drives the adapted mu to 3e-5 on this data,
    where the box blur's spectral zeros make the x-step too ill-conditioned
    for FP32 to follow an FP64 run to 1e-4.)"""
    p = rgb_problem(288, 256, 9, seed=seed, bsnr=40.0, lam=1e-4, mu=1e-3)
    p["iters"] = 200
    p["passes"] = 4
    p["adapt_t"] = 3.0
    return p


def config_plain_72(seed=BASE_SEED + 0):
    """72x72 extended domain, 12 rectangles + ramp 0.2*col/64, 9x9 box blur,
    observed central 64x64, BSNR 50 dB, lambda 1e-3, mu 0.05, 200 iterations."""
    p = problem(72, 72, 9, "rect", "box", bsnr=50.0, lam=1e-3, mu=0.05, seed=seed, ramp_width=64)
    p["iters"] = 200
    return p


def config_large_1024(seed=BASE_SEED + 1):
    """1024^2 GRF (1/f^2) + 40 rectangles, 19x19 Gaussian sigma 3, observed
    central 1006^2, BSNR 50 dB, lambda 5e-4, mu 0.02, 500 iterations."""
    p = problem(1024, 1024, 19, "grf", "gauss", sigma=3.0, bsnr=50.0, lam=5e-4, mu=0.02, seed=seed)
    p["iters"] = 500
    return p


def config_inpaint_2048(seed=BASE_SEED + 2):
    """2048^2 rectangles + ramp, 21x21 motion blur (60-step random walk),
    observed central 2028^2 with 50% i.i.d. missing pixels, BSNR 40 dB,
    lambda 1e-3, mu 0.05, 300 iterations."""
    p = problem(2048, 2048, 21, "rect", "motion", mask_kind=MASK_EXPLICIT, missing=0.5,
                bsnr=40.0, lam=1e-3, mu=0.05, seed=seed, ramp_width=2048 - 8)
    p["iters"] = 300
    return p


SIDES = (128, 192, 256, 384, 512, 768, 1024)


def config_batch_specs(n_images=256, seed=BASE_SEED + 3):
    """Per-image shapes/parameters of the mixed batch (no pixel data), so that
    launch layouts can be planned without generating the images."""
    rng = np.random.default_rng(seed)
    specs = []
    for b in range(n_images):
        side = int(SIDES[rng.integers(len(SIDES))])
        K = int(2 * rng.integers(2, 13) + 1)          # odd 5..25
        bsnr = float(rng.uniform(30.0, 50.0))
        lam = float(10.0 ** rng.uniform(-4.0, -2.0))
        specs.append(dict(M=side, N=side, K=K, sigma=K / 6.0, bsnr=bsnr, lam=lam, mu=50.0 * lam,
                          mask_kind=MASK_DECIMATE if b % 2 == 0 else MASK_BOUNDARY,
                          seed=(seed * 1000 + b)))
    return specs


def config_batch(n_images=256, seed=BASE_SEED + 3, specs=None):
    """Mixed batch: sides uniform in {128..1024}, own Gaussian blur (odd size
    5..25, sigma size/6), even-indexed images x4 decimated, BSNR U[30,50],
    lambda log-uniform [1e-4, 1e-2], mu = 50 lambda, 200 iterations."""
    specs = specs or config_batch_specs(n_images, seed)
    out = []
    for s in specs:
        p = problem(s["M"], s["N"], s["K"], "rect", "gauss", sigma=s["sigma"], mask_kind=s["mask_kind"],
                    decim=4, bsnr=s["bsnr"], lam=s["lam"], mu=s["mu"], seed=s["seed"],
                    ramp_width=s["N"] - 8)
        out.append(p)
    return out


def config_grad_512(n_images=16, seed=BASE_SEED + 4):
    """16 images 512^2 (rectangles + ramp), 15x15 Gaussian sigma 2, observed
    central 498^2, BSNR 45 dB, lambda 1e-3, mu 0.05, 50 iterations,
    checkpoint every 10."""
    out = []
    for b in range(n_images):
        p = problem(512, 512, 15, "rect", "gauss", sigma=2.0, bsnr=45.0, lam=1e-3, mu=0.05,
                    seed=seed * 1000 + b, ramp_width=512 - 8)
        p["iters"] = 50
        out.append(p)
    return out


def unit_directions(shape, count, seed):
    """Seeded random unit directions (for finite-difference checks)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = rng.standard_normal(shape)
        out.append(d / np.linalg.norm(d))
    return out
