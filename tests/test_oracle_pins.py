"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: every expected value comes from
the paper's printed numbers, from an independent library routine (numpy /
scipy), from a closed form, from a dense linear-algebra formulation of the same
problem, or from finite differences.
"""
import os

import numpy as np
import pytest
from scipy.signal import convolve2d

import oracle
from paper_1602_01410_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s=0):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# FFT and PSF embedding
# --------------------------------------------------------------------------

def _kappa_rows():
    rows = []
    with open(os.path.join(GOLDEN, "kappa_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, size, kappa = line.split()[:3]
            rows.append((kind, int(size), float(kappa)))
    return rows


@pytest.mark.parametrize("kind,size,kappa", _kappa_rows())
def test_kappa_table(kind, size, kappa):
    """kappa(H) of Table I / appendix tables, reproduced with the oracle's own
    FFT on the 256 x 256 domain.  Printed values are rounded to 0.1 (x 10^3);
    the largest one differs from a float64 evaluation in its last digit by
    0.057 (8e-8 relative), so the bound is max(0.05, 1e-7 relative)."""
    h = synth.box_kernel(size) if kind == "box" else synth.gaussian_kernel(size, np.sqrt(size))
    Hs = oracle.psf_spectrum(256, 256, h)
    a = np.abs(Hs)
    k = a.max() / a.min() / 1e3
    assert abs(k - kappa) <= max(0.05, 1e-7 * kappa), (k, kappa)


@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 64, 72, 96, 100, 128, 192, 384, 768, 1024])
def test_fft1_vs_numpy(n):
    x = _rng(n).standard_normal(n) + 1j * _rng(n + 1).standard_normal(n)
    ref = np.fft.fft(x)
    scale = max(np.abs(ref).max(), 1.0)
    assert np.abs(oracle.fft1(x) - ref).max() / scale < 1e-13
    assert np.abs(oracle.fft1(x, +1) - np.fft.ifft(x) * n).max() / scale < 1e-13


@pytest.mark.parametrize("shape", [(8, 8), (9, 12), (12, 9), (6, 10)])
def test_fft2_vs_direct_dft(shape):
    x = _rng(3).standard_normal(shape) + 1j * _rng(4).standard_normal(shape)
    d = oracle.dft2_direct(x)
    f = oracle.fft2(x)
    assert np.abs(f - d).max() / np.abs(d).max() < 1e-13
    assert np.abs(d - np.fft.fft2(x)).max() / np.abs(d).max() < 1e-13


def test_parseval_and_inverse():
    x = _rng(5).standard_normal((72, 96)) + 1j * _rng(6).standard_normal((72, 96))
    X = oracle.fft2(x)
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / x.size) < 1e-10 * np.sum(np.abs(x) ** 2)
    back = oracle.fft2(X, +1) / x.size
    assert np.abs(back - x).max() < 1e-13


def test_difference_stencil_spectrum():
    """DFT of the periodic forward-difference stencil has |.|^2 =
    4 sin^2(pi k / n) per axis (the |D^|^2 of the x-step denominator)."""
    M, N = 12, 18
    e = np.zeros((M, N))
    e[0, 0] = 1.0
    gh, gv = oracle.grad(e)
    # D_h e is the impulse response of D_h (a circulant matrix): its spectrum
    # is the eigenvalue of D_h at each frequency
    Fh = oracle.fft2(gh.astype(complex))
    Fv = oracle.fft2(gv.astype(complex))
    ky = np.arange(M)[:, None]
    kx = np.arange(N)[None, :]
    assert np.allclose(np.abs(Fh) ** 2, np.broadcast_to(4 * np.sin(np.pi * kx / N) ** 2, (M, N)), atol=1e-13)
    assert np.allclose(np.abs(Fv) ** 2, np.broadcast_to(4 * np.sin(np.pi * ky / M) ** 2, (M, N)), atol=1e-13)


# --------------------------------------------------------------------------
# Operators H, H^T, D, D^T
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,K", [((8, 8), 3), ((9, 12), 5), ((72, 72), 9), ((10, 7), 7)])
def test_conv_fft_vs_direct(shape, K):
    rng = _rng(K)
    h = rng.uniform(size=(K, K))
    x = rng.standard_normal(shape)
    a = oracle.conv_fft(h, x)
    b = oracle.conv_direct(h, x)
    assert np.abs(a - b).max() < 1e-12 * max(1.0, np.abs(b).max())


def test_valid_region_is_linear_convolution():
    """The central m x n part of the circular convolution equals the 'valid'
    linear convolution (Sec. III, data generation), computed by scipy."""
    rng = _rng(11)
    K = 7
    h = rng.uniform(size=(K, K))           # asymmetric: pins orientation
    x = rng.standard_normal((30, 26))
    circ = oracle.conv_direct(h, x)
    b = K // 2
    lin = convolve2d(x, h, mode="valid")
    assert np.abs(circ[b:-b, b:-b] - lin).max() < 1e-12


def test_adjoint_identities():
    rng = _rng(12)
    M, N, K = 20, 24, 5
    h = rng.uniform(size=(K, K))
    x = rng.standard_normal((M, N))
    w = rng.standard_normal((M, N))
    lhs = np.sum(oracle.conv_fft(h, x) * w)
    rhs = np.sum(x * oracle.conv_fft(h, w, adjoint=True))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    wh, wv = rng.standard_normal((M, N)), rng.standard_normal((M, N))
    gh, gv = oracle.grad(x)
    assert abs(np.sum(gh * wh + gv * wv) - np.sum(x * oracle.gradT(wh, wv))) < 1e-11
    # D against np.roll (independent expression of periodic forward differences)
    assert np.array_equal(gh, np.roll(x, -1, axis=1) - x)
    assert np.array_equal(gv, np.roll(x, -1, axis=0) - x)


# --------------------------------------------------------------------------
# helpers: dense operators built from the definitions (independent of oracle)
# --------------------------------------------------------------------------

def dense_conv(M, N, h):
    K = h.shape[0]
    b = K // 2
    n = M * N
    A = np.zeros((n, n))
    for i in range(M):
        for j in range(N):
            for p in range(-b, b + 1):
                for q in range(-b, b + 1):
                    A[i * N + j, ((i - p) % M) * N + (j - q) % N] += h[b + p, b + q]
    return A


def dense_diff(M, N):
    n = M * N
    Dh = np.zeros((n, n))
    Dv = np.zeros((n, n))
    for i in range(M):
        for j in range(N):
            k = i * N + j
            Dh[k, k] -= 1
            Dh[k, i * N + (j + 1) % N] += 1
            Dv[k, k] -= 1
            Dv[k, ((i + 1) % M) * N + j] += 1
    return Dh, Dv


def small_problem(M=12, N=12, K=3, seed=0, full=False, blur="random", missing=0.0):
    kind = synth.MASK_EXPLICIT if missing > 0 else synth.MASK_BOUNDARY
    p = synth.problem(M, N, K, "rect", blur, mask_kind=kind, missing=missing, bsnr=40.0,
                      lam=1e-2, mu=0.05, seed=seed, nrect=4)
    y = p["y"].astype(np.float64)
    mask = p["mask"].copy()
    if full:
        # every pixel observed: the blurred image on the whole periodic domain
        mask[:] = 1
        y = oracle.conv_direct(p["h"].astype(np.float64), p["x_true"].astype(np.float64))
    return y, mask, p["h"].astype(np.float64)


# --------------------------------------------------------------------------
# x-step and z-step of one iteration
# --------------------------------------------------------------------------

def test_x_step_is_exact_solve_and_z_step():
    """x^{i+1} solves (H^T H + mu D^T D) x = H^T ytilde + mu D^T (v - d)
    (eq. dual_x_iter_resolved_boundaries) and, with alpha = 1, the new z is
    M_z H x^{i+1} (eq. dual_z_iter_resolved_boundaries).  Residual evaluated
    with numpy FFTs and np.roll differences."""
    y, mask, h = small_problem(16, 14, 5, seed=1)
    st = oracle.init_state(y, mask, 5)
    rng = _rng(2)
    for k in ("vh", "vv", "dh", "dv"):
        st[k][...] = rng.standard_normal(st[k].shape) * 0.1
    before = {k: v.copy() for k, v in st.items()}
    mu = 0.07
    x, hist, _, mi = oracle.admm_iterate(st, h, mask, 1e-2, mu, 1, alpha=1.0)
    assert mi < 1e-12
    M, N = y.shape
    hpad = np.zeros((M, N))
    b = 2
    for p in range(-b, b + 1):
        for q in range(-b, b + 1):
            hpad[p % M, q % N] += h[b + p, b + q]
    Hf = np.fft.fft2(hpad)

    def H(a, adj=False):
        return np.real(np.fft.ifft2(np.fft.fft2(a) * (np.conj(Hf) if adj else Hf)))

    def D(a):
        return np.roll(a, -1, 1) - a, np.roll(a, -1, 0) - a

    def DT(wh, wv):
        return np.roll(wh, 1, 1) - wh + np.roll(wv, 1, 0) - wv

    gh, gv = D(x)
    res = H(H(x), True) - H(before["yt"], True) + mu * (DT(gh, gv) - DT(before["vh"] - before["dh"],
                                                                      before["vv"] - before["dv"]))
    assert np.abs(res).max() < 1e-11
    Hx = H(x)
    un = mask == 0
    assert np.abs(st["yt"][un] - Hx[un]).max() < 1e-12
    assert np.array_equal(st["yt"][~un], before["yt"][~un])


def test_init_state_replicates_border():
    y, mask, h = small_problem(14, 16, 5, seed=3, missing=0.3)
    st = oracle.init_state(y, mask, 5)
    b = 2
    obs = mask.astype(bool)
    assert np.array_equal(st["yt"][obs], y[obs])
    mean = y[obs].mean()
    valid = synth.valid_region(14, 16, 5)
    assert np.allclose(st["yt"][valid & ~obs], mean)
    for i in range(14):
        for j in range(16):
            if not valid[i, j]:
                si, sj = min(max(i, b), 14 - b - 1), min(max(j, b), 16 - b - 1)
                assert st["yt"][i, j] == st["yt"][si, sj]
    gh, gv = oracle.grad(st["yt"])
    assert np.array_equal(st["vh"], gh) and np.array_equal(st["vv"], gv)
    assert not st["dh"].any() and not st["dv"].any()


def test_init_state_is_edge_padding():
    """The initial state against library routines (Sec. III-B: the observed
    image padded by repeating its border pixels).  With only the boundary band
    unobserved, ytilde^0 = numpy.pad(y_valid, b, mode='edge'); with holes
    inside, the holes first take numpy's mean of the observed pixels.  v^0 is
    the periodic forward difference of ytilde^0 (numpy.roll), d^0 = 0."""
    for (M, N, K, missing, seed) in ((14, 16, 5, 0.0, 5), (20, 18, 7, 0.35, 6), (12, 12, 3, 0.0, 7)):
        y, mask, h = small_problem(M, N, K, seed=seed, missing=missing)
        b = K // 2
        st = oracle.init_state(y, mask, K)
        core = y[b:M - b, b:N - b].copy()
        obs = mask[b:M - b, b:N - b].astype(bool)
        core[~obs] = np.mean(y[mask.astype(bool)])
        want = np.pad(core, b, mode="edge")
        assert np.array_equal(st["yt"], want), (M, N, K, missing)
        assert np.array_equal(st["vh"], np.roll(want, -1, axis=1) - want)
        assert np.array_equal(st["vv"], np.roll(want, -1, axis=0) - want)
        assert not st["dh"].any() and not st["dv"].any()


# --------------------------------------------------------------------------
# closed forms of the whole iteration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("iters", [1, 7, 40])
def test_lambda0_all_observed_closed_form(iters):
    """lambda = 0, all pixels observed, v^0 = D x^0, d^0 = 0: then d stays 0,
    v^i = D x^i and per frequency X^N = a^N X^0 + (1 - a^N) Y/H with
    a = mu|D|^2 / (|H|^2 + mu|D|^2) (from the x-step closed form)."""
    y, mask, h = small_problem(16, 16, 5, seed=4, full=True)
    M, N = y.shape
    mu = 0.05
    st = oracle.init_state(y, mask, 5)
    x0 = st["yt"].copy()
    x, _, _, _ = oracle.admm_iterate(st, h, mask, 0.0, mu, iters, alpha=2.0)
    Hf = oracle.psf_spectrum(M, N, h)
    ky = np.arange(M)[:, None]
    kx = np.arange(N)[None, :]
    dd = 4 * np.sin(np.pi * kx / N) ** 2 + 4 * np.sin(np.pi * ky / M) ** 2
    a = mu * dd / (np.abs(Hf) ** 2 + mu * dd)
    X0 = np.fft.fft2(x0)
    Y = np.fft.fft2(y)
    XN = a ** iters * X0 + (1 - a ** iters) * Y / Hf
    ref = np.real(np.fft.ifft2(XN))
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()


def test_quadratic_all_observed_tikhonov_limit():
    """Quadratic phi = lambda/2 |Dx|^2, all observed: the fixed point is
    X = conj(H) Y / (|H|^2 + lambda |D|^2)."""
    y, mask, h = small_problem(16, 16, 3, seed=5, full=True, blur="box")
    M, N = y.shape
    lam, mu = 0.02, 0.02
    st = oracle.init_state(y, mask, 3)
    x, _, _, _ = oracle.admm_iterate(st, h, mask, lam, mu, 3000, alpha=1.0, phi="quad")
    Hf = oracle.psf_spectrum(M, N, h)
    ky = np.arange(M)[:, None]
    kx = np.arange(N)[None, :]
    dd = 4 * np.sin(np.pi * kx / N) ** 2 + 4 * np.sin(np.pi * ky / M) ** 2
    ref = np.real(np.fft.ifft2(np.conj(Hf) * np.fft.fft2(y) / (np.abs(Hf) ** 2 + lam * dd)))
    assert np.abs(x - ref).max() < 1e-9


@pytest.mark.parametrize("alpha", [1.0, 2.0])
def test_quadratic_masked_normal_equations(alpha):
    """Quadratic phi with unknown boundaries and missing pixels on 16 x 16:
    the limit solves (H^T M_y^T M_y H + lambda D^T D) x = H^T M_y^T y, solved
    densely with matrices built from the definitions."""
    y, mask, h = small_problem(16, 16, 5, seed=6, missing=0.3)
    M, N = y.shape
    lam, mu = 0.01, 0.01
    st = oracle.init_state(y, mask, 5)
    x, _, _, _ = oracle.admm_iterate(st, h, mask, lam, mu, 20000, alpha=alpha, phi="quad")
    Hd = dense_conv(M, N, h)
    Dh, Dv = dense_diff(M, N)
    obs = mask.reshape(-1).astype(bool)
    My = np.eye(M * N)[obs]
    A = Hd.T @ My.T @ My @ Hd + lam * (Dh.T @ Dh + Dv.T @ Dv)
    rhs = Hd.T @ My.T @ y.reshape(-1)[obs]
    ref = np.linalg.solve(A, rhs).reshape(M, N)
    assert np.abs(x - ref).max() < 1e-9, np.abs(x - ref).max()


def _dense_standard_admm_tv(y, mask, h, lam, mu, iters):
    """Standard ADMM on u = [x; z] (eqs. admm_xz_1..3) with the joint
    (x, z) step solved densely; independent of the oracle."""
    M, N = y.shape
    n = M * N
    Hd = dense_conv(M, N, h)
    Dh, Dv = dense_diff(M, N)
    D = np.vstack([Dh, Dv])
    un = ~mask.reshape(-1).astype(bool)
    Su = np.eye(n)[un]
    So = np.eye(n)[~un]
    dcount = Su.shape[0]
    yo = y.reshape(-1)[~un]
    # normal equations of 1/2|So^T y + Su^T z - H x|^2 + mu/2|a - Dx|^2 + mu/2|c - z|^2
    A = np.block([[Hd.T @ Hd + mu * D.T @ D, -Hd.T @ Su.T],
                  [-Su @ Hd, (1 + mu) * np.eye(dcount)]])
    Ainv = np.linalg.inv(A)
    x = np.zeros(n)
    z = np.zeros(dcount)
    vx = D @ x
    dx = np.zeros(2 * n)
    vz = z.copy()
    dz = np.zeros(dcount)
    tau = lam / mu
    for _ in range(iters):
        rhs = np.concatenate([Hd.T @ (So.T @ yo) + mu * D.T @ (vx - dx), mu * (vz - dz)])
        u = Ainv @ rhs
        x, z = u[:n], u[n:]
        t = D @ x + dx
        th, tv = t[:n], t[n:]
        nr = np.sqrt(th * th + tv * tv)
        s = np.where(nr > tau, (nr - tau) / np.where(nr > 0, nr, 1), 0.0)
        vx = np.concatenate([s * th, s * tv])
        vz = z + dz
        dx = dx - (vx - D @ x)
        dz = dz - (vz - z)
    return x.reshape(M, N)


@pytest.mark.slow
def test_tv_converges_to_standard_admm_solution():
    """TV: the partial ADMM and a dense standard ADMM reach the same minimiser
    (the paper reports all methods agreeing to RMSE < 1e-7)."""
    y, mask, h = small_problem(8, 8, 3, seed=7, blur="box")
    lam, mu = 1e-2, 0.05
    st = oracle.init_state(y, mask, 3)
    x, _, _, _ = oracle.admm_iterate(st, h, mask, lam, mu, 60000, alpha=1.0)
    ref = _dense_standard_admm_tv(y, mask, h, lam, mu, 60000)
    rmse = np.sqrt(np.mean((x - ref) ** 2))
    assert rmse < 1e-7, rmse


def test_alpha2_same_fixed_point_as_alpha1():
    y, mask, h = small_problem(12, 12, 3, seed=8, blur="box")
    st1 = oracle.init_state(y, mask, 3)
    st2 = oracle.init_state(y, mask, 3)
    x1, _, _, _ = oracle.admm_iterate(st1, h, mask, 1e-2, 0.05, 40000, alpha=1.0)
    x2, _, _, _ = oracle.admm_iterate(st2, h, mask, 1e-2, 0.05, 40000, alpha=2.0)
    assert np.sqrt(np.mean((x1 - x2) ** 2)) < 1e-7


def test_objective_decreases_towards_minimum():
    """The objective of (problem_xz) at the converged iterate is below that at
    the initial point and at perturbations of the converged point."""
    y, mask, h = small_problem(12, 12, 3, seed=9, blur="box")
    lam = 1e-2
    st = oracle.init_state(y, mask, 3)
    yt0 = st["yt"].copy()
    f0 = oracle.objective(h, yt0, yt0, lam)
    x, _, _, _ = oracle.admm_iterate(st, h, mask, lam, 0.05, 20000, alpha=1.0)
    f = oracle.objective(h, st["yt"], x, lam)
    assert f < f0
    rng = _rng(10)
    for _ in range(5):
        dx = rng.standard_normal(x.shape) * 1e-3
        # optimal z for a given x is M_z H x: perturb x and re-optimise z
        yt = st["yt"].copy()
        hx = oracle.conv_fft(h, x + dx)
        yt[mask == 0] = hx[mask == 0]
        assert oracle.objective(h, yt, x + dx, lam) >= f - 1e-12


# --------------------------------------------------------------------------
# dynamics: Lemma 2 and Lemma 3 (Appendix B), alpha = 1, fixed mu, one pass
# --------------------------------------------------------------------------

def test_lemma2_fejer_and_lemma3_monotone_steps():
    y, mask, h = small_problem(10, 10, 3, seed=13, blur="box")
    lam, mu = 1e-2, 0.05
    ref = oracle.init_state(y, mask, 3)
    oracle.admm_iterate(ref, h, mask, lam, mu, 100000, alpha=1.0)
    un = mask == 0
    st = oracle.init_state(y, mask, 3)

    def gdist(a, b):
        return (np.sum((a["yt"][un] - b["yt"][un]) ** 2)
                + mu * np.sum((a["vh"] - b["vh"]) ** 2 + (a["vv"] - b["vv"]) ** 2)
                + mu * np.sum((a["dh"] - b["dh"]) ** 2 + (a["dv"] - b["dv"]) ** 2))

    dist = [gdist(st, ref)]
    steps = []
    for _ in range(400):
        _, hist, _, _ = oracle.admm_iterate(st, h, mask, lam, mu, 1, alpha=1.0)
        dist.append(gdist(st, ref))
        steps.append(hist[0, 3])
    dist = np.array(dist)
    steps = np.array(steps)
    # Lemma 2: |w^i - w*|_G^2 - |w^{i+1} - w*|_G^2 >= |w^{i+1} - w^i|_G^2
    gap = dist[:-1] - dist[1:] - steps
    assert (gap >= -1e-12 * dist[0]).all(), gap.min()
    # Lemma 3: the step norms are non-increasing and tend to 0
    assert (np.diff(steps) <= 1e-12 * steps[0]).all()
    assert steps[-1] < 1e-3 * steps[0]


# --------------------------------------------------------------------------
# Proposed-AD passes, adaptive penalty, warm start (same minimiser)
# --------------------------------------------------------------------------

def test_many_bgs_passes_solve_joint_xz_step():
    """With many BGS passes, one iteration's inner loop converges to the joint
    minimiser of (admm_xz_1a) over (x, z), which the dense system gives."""
    y, mask, h = small_problem(10, 10, 3, seed=14, blur="box")
    M, N = y.shape
    n = M * N
    mu = 0.05
    st = oracle.init_state(y, mask, 3)
    before = {k: v.copy() for k, v in st.items()}
    x, _, _, _ = oracle.admm_iterate(st, h, mask, 1e-2, mu, 1, alpha=1.0, passes=3000)
    Hd = dense_conv(M, N, h)
    Dh, Dv = dense_diff(M, N)
    D = np.vstack([Dh, Dv])
    un = ~mask.reshape(-1).astype(bool)
    Su = np.eye(n)[un]
    So = np.eye(n)[~un]
    A = np.block([[Hd.T @ Hd + mu * D.T @ D, -Hd.T @ Su.T], [-Su @ Hd, np.eye(Su.shape[0])]])
    a = np.concatenate([(before["vh"] - before["dh"]).reshape(-1), (before["vv"] - before["dv"]).reshape(-1)])
    rhs = np.concatenate([Hd.T @ So.T @ y.reshape(-1)[~un] + mu * D.T @ a, np.zeros(Su.shape[0])])
    u = np.linalg.solve(A, rhs)
    assert np.abs(x.reshape(-1) - u[:n]).max() < 1e-9


def test_adaptive_mu_and_passes_reach_same_minimiser():
    y, mask, h = small_problem(12, 12, 5, seed=15, blur="box")
    lam = 1e-2
    base = oracle.admm_run(y, mask, h, lam, 0.05, 30000, alpha=1.0)
    ad = oracle.admm_run(y, mask, h, lam, 0.05, 30000, alpha=2.0, adapt_t=3.0)
    pp = oracle.admm_run(y, mask, h, lam, 0.05, 15000, alpha=2.0, passes=2)
    ws = oracle.admm_run(y, mask, h, lam, 0.05, 30000, alpha=2.0, warm_iters=100)
    for other in (ad, pp, ws):
        assert np.sqrt(np.mean((base["x"] - other["x"]) ** 2)) < 1e-7
    # the penalty rule moved mu and kept it a power-of-two multiple of mu^0
    mus = ad["hist"][:, 4]
    r = np.log2(mus / 0.05)
    assert np.allclose(r, np.round(r))


def _one_step(st, h, mask, lam, mu, adapt_t):
    """One oracle iteration from a copy of `st`; returns (new state, hist row, mu')."""
    s = {k: v.copy() for k, v in st.items()}
    x, hist, mu_f, _ = oracle.admm_iterate(s, h, mask, lam, mu, 1, alpha=2.0, adapt_t=adapt_t)
    return s, hist[0], mu_f


def _check_penalty_step(st, h, mask, lam, mu, t=3.0):
    """eq. (varying_penalty) on one iteration: the x-, z-, v- and d-steps are
    those of the fixed penalty; then mu doubles when |d'-d| > t|v'-v| and
    halves when |v'-v| > t|d'-d|, and the scaled dual d is rescaled so that
    the unscaled multiplier mu*d is unchanged (halved d with doubled mu and
    the reverse).  Returns the decision (+1 double, -1 halve, 0 keep)."""
    fixed, hrow, mu_fixed = _one_step(st, h, mask, lam, mu, 0.0)
    ad, _, mu_new = _one_step(st, h, mask, lam, mu, t)
    assert mu_fixed == mu
    nd, nv = hrow[0], hrow[1]
    # the steps before the penalty update do not depend on it
    for k in ("yt", "vh", "vv"):
        assert np.array_equal(ad[k], fixed[k]), k
    if nd > t * nv:
        want = 1
    elif nv > t * nd:
        want = -1
    else:
        want = 0
    assert mu_new == mu * {1: 2.0, -1: 0.5, 0: 1.0}[want], (nd, nv, mu, mu_new)
    # the unscaled multiplier is invariant (powers of two: exact)
    for k in ("dh", "dv"):
        assert np.array_equal(mu_new * ad[k], mu * fixed[k]), k
    return want


def test_adaptive_penalty_rule_on_built_states():
    """Hand-built states on either side of the thresholds of eq.
    (varying_penalty).  (a) lambda so large that the soft threshold zeroes
    every u and v = 0: then v' - v = 0 while d' - d = D x' != 0, so mu must
    double and d halve.  (b) lambda = 0 and d = 0: v' = u = D x', d' = 0
    (so d' - d = 0 while v' - v = D x' - v != 0): mu must halve (d' = 0 is
    invariant under the rescaling, so (c) repeats it with d != 0 and a tiny
    lambda: d' is then tau u/|u| per pixel, |d' - d| stays below |v' - v|/t)."""
    y, mask, h = small_problem(12, 14, 5, seed=31)
    st = oracle.init_state(y, mask, 5)
    mu = 0.05
    # (a)
    sa = {k: v.copy() for k, v in st.items()}
    sa["vh"][:] = 0.0
    sa["vv"][:] = 0.0
    assert _check_penalty_step(sa, h, mask, 1e6, mu) == 1
    # the halving of d is visible (d' = u != 0)
    ad, _, mu_new = _one_step(sa, h, mask, 1e6, mu, 3.0)
    fx, _, _ = _one_step(sa, h, mask, 1e6, mu, 0.0)
    assert mu_new == 2 * mu and np.abs(fx["dh"]).max() > 0
    np.testing.assert_array_equal(ad["dh"], 0.5 * fx["dh"])
    # (b)
    sb = {k: v.copy() for k, v in st.items()}
    sb["vh"][:] = 0.0
    sb["vv"][:] = 0.0
    assert _check_penalty_step(sb, h, mask, 0.0, mu) == -1
    # (c)
    rng = _rng(32)
    sc = {k: v.copy() for k, v in st.items()}
    sc["dh"] = 1e-4 * rng.standard_normal(sc["dh"].shape)
    sc["dv"] = 1e-4 * rng.standard_normal(sc["dv"].shape)
    sc["vh"][:] = 0.0
    sc["vv"][:] = 0.0
    assert _check_penalty_step(sc, h, mask, 1e-9, mu) == -1
    ad, _, mu_new = _one_step(sc, h, mask, 1e-9, mu, 3.0)
    fx, _, _ = _one_step(sc, h, mask, 1e-9, mu, 0.0)
    assert mu_new == 0.5 * mu and np.abs(fx["dh"]).max() > 0
    np.testing.assert_array_equal(ad["dh"], 2.0 * fx["dh"])


def test_adaptive_penalty_rule_along_a_run():
    """Every iteration of an adaptive run (t = 3, the value of Sec. III-B)
    obeys eq. (varying_penalty) and keeps mu*d invariant; the run takes all
    three decisions."""
    y, mask, h = small_problem(16, 16, 5, seed=33, missing=0.2)
    lam = 1e-3
    st = oracle.init_state(y, mask, 5)
    mu = 1e-2
    seen = set()
    for _ in range(60):
        seen.add(_check_penalty_step(st, h, mask, lam, mu))
        x, hist, mu, _ = oracle.admm_iterate(st, h, mask, lam, mu, 1, alpha=2.0, adapt_t=3.0)
    assert seen == {1, -1, 0}, seen


def test_warm_start_fixed_point():
    """The quadratic warm start (ini_x, ini_z) converges to the minimiser of
    f(x, z) + tau/2 |x|^2; checked densely."""
    y, mask, h = small_problem(10, 10, 3, seed=16, blur="box")
    M, N = y.shape
    n = M * N
    tau = 1e-1
    st = oracle.init_state(y, mask, 3)
    oracle.warm_start(st, h, mask, tau, 5000)
    Hd = dense_conv(M, N, h)
    obs = mask.reshape(-1).astype(bool)
    My = np.eye(n)[obs]
    A = Hd.T @ My.T @ My @ Hd + tau * np.eye(n)
    x = np.linalg.solve(A, Hd.T @ My.T @ y.reshape(-1)[obs])
    z = (Hd @ x)[~obs]
    assert np.abs(st["yt"].reshape(-1)[~obs] - z).max() < 1e-8


# --------------------------------------------------------------------------
# reverse mode (the FP64 adjoint) against central finite differences
# --------------------------------------------------------------------------

@pytest.mark.parametrize("phi,alpha", [("tv", 2.0), ("tv", 1.0), ("quad", 2.0)])
def test_backward_vs_finite_differences(phi, alpha):
    y, mask, h = small_problem(12, 10, 5, seed=17, missing=0.2)
    lam, mu, iters = 3e-3, 0.05, 6
    rng = _rng(18)
    x_target = rng.standard_normal(y.shape)

    def loss(yy, ll, hh):
        r = oracle.admm_run(yy, mask, hh, ll, mu, iters, alpha=alpha, phi=phi)
        return 0.5 * np.sum((r["x"] - x_target) ** 2), r["x"]

    L0, x = loss(y, lam, h)
    gy, gl, gh = oracle.admm_backward(y, mask, h, lam, mu, iters, x - x_target, alpha=alpha, phi=phi)
    assert not gy[mask == 0].any()
    eps = 1e-6
    for t in range(3):
        dy = rng.standard_normal(y.shape) * mask
        dh = rng.standard_normal(h.shape)
        fd_y = (loss(y + eps * dy, lam, h)[0] - loss(y - eps * dy, lam, h)[0]) / (2 * eps)
        fd_h = (loss(y, lam, h + eps * dh)[0] - loss(y, lam, h - eps * dh)[0]) / (2 * eps)
        assert abs(fd_y - np.sum(gy * dy)) <= 1e-6 * max(1.0, abs(fd_y)), (fd_y, np.sum(gy * dy))
        assert abs(fd_h - np.sum(gh * dh)) <= 1e-6 * max(1.0, abs(fd_h)), (fd_h, np.sum(gh * dh))
    el = 1e-7
    fd_l = (loss(y, lam + el, h)[0] - loss(y, lam - el, h)[0]) / (2 * el)
    assert abs(fd_l - gl) <= 1e-5 * max(1.0, abs(fd_l)), (fd_l, gl)
