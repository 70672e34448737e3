"""FP64 CPU oracle for the partial ADMM (arXiv 1602.01410, Sec. II-B / III-B).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
The arithmetic lives in ``oracle.c`` (plain C, double precision, its own
radix-2 + Bluestein FFT).  This module only compiles it with gcc and marshals
numpy arrays through ctypes.  It shares no code with the HIP library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB names another build of oracle.c to load instead (the sanitizer
# test runs the pins against an ASan/UBSan build)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "_oracle.so")
_lib = None

PHI = {"tv": 0, "quad": 1}


def build(force=True, out=None, sanitize=False):
    """Compile oracle.c into _oracle.so (gcc, -O3, OpenMP, IEEE semantics);
    sanitize=True: an AddressSanitizer + UndefinedBehaviorSanitizer build
    (-O1 -g) into `out`."""
    out = out or _LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O3"]
    cmd = ["gcc"] + opt + ["-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I = ctypes.c_int
_F = ctypes.c_double


def _declare(L):
    L.or_fft1.argtypes = [_I, _D, _D, _I]
    L.or_fft2.argtypes = [_I, _I, _D, _D, _I]
    L.or_dft2_direct.argtypes = [_I, _I, _D, _D, _D, _D, _I]
    L.or_psf_spectrum.argtypes = [_I, _I, _I, _D, _D, _D]
    L.or_conv_direct.argtypes = [_I, _I, _I, _D, _D, _D]
    L.or_conv_fft.argtypes = [_I, _I, _I, _D, _D, _D, _I]
    L.or_grad.argtypes = [_I, _I, _D, _D, _D]
    L.or_gradT.argtypes = [_I, _I, _D, _D, _D]
    L.or_init_state.argtypes = [_I, _I, _I, _D, _U8, _D, _D, _D, _D, _D]
    L.or_admm_iterate.argtypes = [_I, _I, _I, _D, _U8, _F, _D, _F, _I, _I, _I, _F,
                                  _D, _D, _D, _D, _D, _D, _D]
    L.or_admm_iterate.restype = ctypes.c_double
    L.or_admm_iterate_vec.argtypes = [_I, _I, _I, _I, _D, _U8, _F, _D, _F, _I, _I, _F,
                                      _D, _D, _D, _D, _D, _D, _D]
    L.or_admm_iterate_vec.restype = ctypes.c_double
    L.or_warm_start.argtypes = [_I, _I, _I, _D, _U8, _F, _I, _D]
    L.or_objective.argtypes = [_I, _I, _I, _D, _D, _D, _F, _I]
    L.or_objective.restype = ctypes.c_double
    L.or_admm_backward.argtypes = [_I, _I, _I, _D, _D, _U8, _F, _F, _F, _I, _I, _D, _D, _D, _D]
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_threads.argtypes = [_I]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_U8)


def num_threads():
    return lib().or_num_threads()


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().or_set_threads(int(n))


def fft1(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    re, pr = _d(x.real.copy())
    im, pi = _d(x.imag.copy())
    lib().or_fft1(x.size, pr, pi, sign)
    return re + 1j * im


def fft2(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    M, N = x.shape
    re, pr = _d(x.real.copy())
    im, pi = _d(x.imag.copy())
    lib().or_fft2(M, N, pr, pi, sign)
    return re + 1j * im


def dft2_direct(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    M, N = x.shape
    re, pr = _d(x.real.copy())
    im, pi = _d(x.imag.copy())
    ore, por = _d(np.zeros((M, N)))
    oim, poi = _d(np.zeros((M, N)))
    lib().or_dft2_direct(M, N, pr, pi, por, poi, sign)
    return ore + 1j * oim


def psf_spectrum(M, N, h):
    h, ph = _d(h)
    re, pr = _d(np.zeros((M, N)))
    im, pi = _d(np.zeros((M, N)))
    lib().or_psf_spectrum(M, N, h.shape[0], ph, pr, pi)
    return re + 1j * im


def conv_direct(h, x):
    h, ph = _d(h)
    x, px = _d(x)
    out, po = _d(np.zeros_like(x))
    lib().or_conv_direct(x.shape[0], x.shape[1], h.shape[0], ph, px, po)
    return out


def conv_fft(h, x, adjoint=False):
    h, ph = _d(h)
    x, px = _d(x)
    out, po = _d(np.zeros_like(x))
    lib().or_conv_fft(x.shape[0], x.shape[1], h.shape[0], ph, px, po, int(adjoint))
    return out


def grad(x):
    x, px = _d(x)
    gh, ph = _d(np.zeros_like(x))
    gv, pv = _d(np.zeros_like(x))
    lib().or_grad(x.shape[0], x.shape[1], px, ph, pv)
    return gh, gv


def gradT(wh, wv):
    wh, ph = _d(wh)
    wv, pv = _d(wv)
    out, po = _d(np.zeros_like(wh))
    lib().or_gradT(wh.shape[0], wh.shape[1], ph, pv, po)
    return out


def init_state(y, mask, K):
    y, py = _d(y)
    m, pm = _u8(mask)
    M, N = y.shape
    st = {k: np.zeros((M, N)) for k in ("yt", "vh", "vv", "dh", "dv")}
    ptr = {k: st[k].ctypes.data_as(_D) for k in st}
    lib().or_init_state(M, N, K, py, pm, ptr["yt"], ptr["vh"], ptr["vv"], ptr["dh"], ptr["dv"])
    return st


def warm_start(state, h, mask, tau=1e-3, iters=100):
    h, ph = _d(h)
    m, pm = _u8(mask)
    yt = state["yt"]
    M, N = yt.shape
    lib().or_warm_start(M, N, h.shape[0], ph, pm, tau, iters, yt.ctypes.data_as(_D))
    return state


def admm_iterate(state, h, mask, lam, mu, iters, alpha=2.0, passes=1, phi="tv", adapt_t=0.0):
    """Advance `state` (dict of float64 arrays, updated in place) by `iters`
    iterations.  Returns (x, hist, mu_final, max_imag)."""
    h, ph = _d(h)
    m, pm = _u8(mask)
    M, N = state["yt"].shape
    for k in ("yt", "vh", "vv", "dh", "dv"):
        assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
    x = np.zeros((M, N))
    hist = np.zeros((max(iters, 1), 5))
    mu_c = ctypes.c_double(mu)
    mi = lib().or_admm_iterate(M, N, h.shape[0], ph, pm, lam, ctypes.byref(mu_c), alpha, passes,
                               PHI[phi], iters, adapt_t,
                               *(state[k].ctypes.data_as(_D) for k in ("yt", "vh", "vv", "dh", "dv")),
                               x.ctypes.data_as(_D), hist.ctypes.data_as(_D))
    return x, hist[:iters], mu_c.value, mi


def admm_run_vec(ys, masks, h, lam, mu, iters, alpha=2.0, passes=1, adapt_t=0.0, warm_iters=0,
                 warm_tau=1e-3):
    """Colour images with vectorial TV (Sec. III-C, demosaicing): ys, masks
    (C, M, N); one blur h for all channels.  Each channel is initialised (and
    warm-started) on its own; the iterations couple them in the v-step.
    Returns a dict of (C, M, N) arrays x, yt, vh, vv, dh, dv and hist, mu."""
    ys = np.asarray(ys, dtype=np.float64)
    masks = np.ascontiguousarray(np.asarray(masks), dtype=np.uint8)
    C, M, N = ys.shape
    K = np.asarray(h).shape[0]
    chans = [init_state(ys[c], masks[c], K) for c in range(C)]
    if warm_iters:
        for c in range(C):
            warm_start(chans[c], h, masks[c], warm_tau, warm_iters)
    st = {k: np.ascontiguousarray(np.stack([ch[k] for ch in chans])) for k in ("yt", "vh", "vv", "dh", "dv")}
    hh, ph = _d(h)
    x = np.zeros((C, M, N))
    hist = np.zeros((max(iters, 1), 5))
    mu_c = ctypes.c_double(mu)
    mi = lib().or_admm_iterate_vec(M, N, K, C, ph, masks.ctypes.data_as(_U8), lam, ctypes.byref(mu_c), alpha,
                                   passes, iters, adapt_t,
                                   *(st[k].ctypes.data_as(_D) for k in ("yt", "vh", "vv", "dh", "dv")),
                                   x.ctypes.data_as(_D), hist.ctypes.data_as(_D))
    st.update(x=x, hist=hist[:iters], mu=mu_c.value, max_imag=mi)
    return st


def admm_run(y, mask, h, lam, mu, iters, alpha=2.0, passes=1, phi="tv", adapt_t=0.0,
             warm_iters=0, warm_tau=1e-3):
    """Initialise from y (Sec. III-B) and run `iters` iterations."""
    st = init_state(y, mask, np.asarray(h).shape[0])
    if warm_iters:
        warm_start(st, h, mask, warm_tau, warm_iters)
    x, hist, mu_f, mi = admm_iterate(st, h, mask, lam, mu, iters, alpha, passes, phi, adapt_t)
    st.update(x=x, hist=hist, mu=mu_f, max_imag=mi)
    return st


def objective(h, yt, x, lam, phi="tv"):
    h, ph = _d(h)
    yt, py = _d(yt)
    x, px = _d(x)
    return lib().or_objective(x.shape[0], x.shape[1], h.shape[0], ph, py, px, lam, PHI[phi])


def admm_backward(y, mask, h, lam, mu, iters, grad_x, alpha=2.0, phi="tv"):
    """Reverse mode through init + `iters` iterations; returns (dy, dlam, dh)."""
    y, py = _d(y)
    m, pm = _u8(mask)
    h, ph = _d(h)
    g, pg = _d(grad_x)
    M, N = y.shape
    gy, pgy = _d(np.zeros((M, N)))
    gh, pgh = _d(np.zeros_like(h))
    gl = ctypes.c_double(0.0)
    lib().or_admm_backward(M, N, h.shape[0], ph, py, pm, lam, mu, alpha, PHI[phi], iters,
                           pg, pgy, ctypes.byref(gl), pgh)
    return gy, gl.value, gh
