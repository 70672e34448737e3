"""Thin Python binding of the C ABI in include/deconv.h.

Argument marshalling only: tensors are PyTorch device tensors, their data
pointers go straight to libdeconv.so, and every step of the method runs in the
library's HIP kernels.  If the library is missing this module raises; there is
no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdeconv.so")

MASK_BOUNDARY, MASK_EXPLICIT, MASK_DECIMATE = 0, 1, 2

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported size", 3: "singular blur (sum(h) == 0)",
          4: "non-finite values", 5: "no checkpoints", 6: "HIP error", 7: "out of memory", 8: "call order"}


class DeconvError(RuntimeError):
    def __init__(self, code, where, stats=None):
        super().__init__("%s: %s (status %d)" % (where, STATUS.get(code, "?"), code))
        self.code = code
        self.stats = stats   # per-image statistics, when the call filled them


class ImageDesc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("ksize", ctypes.c_int32),
                ("mask_kind", ctypes.c_int32), ("decim", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("check_every", ctypes.c_int32),
                ("tol_primal", ctypes.c_double), ("tol_dual", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("bgs_passes", ctypes.c_int32),
                ("adapt_t", ctypes.c_double), ("warm_iters", ctypes.c_int32),
                ("warm_tau", ctypes.c_float), ("channels", ctypes.c_int32),
                ("spectra_hint", ctypes.c_int32), ("row_tiles", ctypes.c_int32),
                ("row_threads", ctypes.c_int32), ("col_threads", ctypes.c_int32),
                ("small_images", ctypes.c_int32), ("separable_blur", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("r_primal", ctypes.c_double),
                ("r_dual", ctypes.c_double), ("r_z", ctypes.c_double), ("status", ctypes.c_int32),
                ("mu", ctypes.c_float)]


EXPORTS = ("deconv_options_default", "deconv_plan_workspace_size", "deconv_plan_create",
           "deconv_plan_destroy", "deconv_admm_run", "deconv_admm_continue", "deconv_state_export",
           "deconv_state_import", "deconv_admm_backward", "deconv_plan_run_id", "deconv_blur_spectrum",
           "deconv_fft2", "deconv_plan_kernel_times", "deconv_plan_bwd_kernel_times", "deconv_plan_schedule",
           "deconv_plan_tiles", "deconv_plan_separable",
           "deconv_status_str",
           "deconv_admm_run_static")

_lib = None


def lib():
    """Open libdeconv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdeconv.so not built: run `python -m paper_1602_01410_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I32 = ctypes.c_int32
        L.deconv_options_default.argtypes = [ctypes.POINTER(Options)]
        L.deconv_plan_workspace_size.argtypes = [I32, ctypes.POINTER(ImageDesc), ctypes.POINTER(Options),
                                                 ctypes.POINTER(ctypes.c_size_t)]
        L.deconv_plan_create.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(ImageDesc),
                                         ctypes.POINTER(Options), P, P, ctypes.c_size_t]
        L.deconv_plan_destroy.argtypes = [P]
        L.deconv_admm_run.argtypes = [P, P, P, P, P, P, I32, P, P, ctypes.POINTER(Stats)]
        L.deconv_admm_continue.argtypes = [P, P, P, I32, P, P, ctypes.POINTER(Stats)]
        L.deconv_state_export.argtypes = [P, P, P, P]
        L.deconv_state_import.argtypes = [P, P, P, P, P, P]
        L.deconv_admm_backward.argtypes = [P, P, P, P, P, P, P, P, P, P, ctypes.c_uint64]
        L.deconv_plan_run_id.argtypes = [P, ctypes.POINTER(ctypes.c_uint64)]
        L.deconv_admm_run_static.argtypes = [I32, ctypes.POINTER(ImageDesc), ctypes.POINTER(Options), P, P, P, P,
                                             P, P, I32, P, P, ctypes.POINTER(Stats)]
        L.deconv_blur_spectrum.argtypes = [P, P, P]
        L.deconv_fft2.argtypes = [I32, I32, I32, P, I32, P]
        L.deconv_plan_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        L.deconv_plan_bwd_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        L.deconv_plan_schedule.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.deconv_plan_tiles.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.deconv_plan_separable.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.deconv_status_str.argtypes = [I32]
        L.deconv_status_str.restype = ctypes.c_char_p
        for f in EXPORTS:
            if f != "deconv_status_str":
                getattr(L, f).restype = I32
        _lib = L
    return _lib


def _check(code, where, stats=None):
    if code != 0:
        raise DeconvError(code, where, stats)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_options(**kw):
    o = Options()
    _check(lib().deconv_options_default(ctypes.byref(o)), "options")
    names = {f[0] for f in Options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError("unknown option %r" % k)
        if k == "tune_cache" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def _descs(images):
    arr = (ImageDesc * len(images))()
    for i, d in enumerate(images):
        arr[i] = ImageDesc(int(d["height"]), int(d["width"]), int(d["ksize"]),
                           int(d.get("mask_kind", MASK_BOUNDARY)), int(d.get("decim", 1)))
    return arr


def workspace_size(images, **opts):
    n = ctypes.c_size_t(0)
    o = default_options(**opts)
    d = _descs(images)
    _check(lib().deconv_plan_workspace_size(len(images), d, ctypes.byref(o), ctypes.byref(n)), "workspace_size")
    return n.value


class Plan:
    """A plan for a batch of images.  images: list of dicts with height,
    width, ksize, mask_kind, decim.  Keyword options: the fields of
    deconv_options.  The plan allocates its own workspace on the current
    device and runs on `stream` (torch stream, default: current)."""

    def __init__(self, images, stream=None, workspace=None, **opts):
        self.images = [dict(d) for d in images]
        self.opts = default_options(**opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.sizes = [int(d["height"]) * int(d["width"]) for d in images]
        self.ksq = [int(d["ksize"]) ** 2 for d in images]
        self.npx = sum(self.sizes)
        self.handle = ctypes.c_void_p()
        # workspace: a caller-owned device tensor of at least workspace_size
        # bytes (kept alive by the plan), or None for a plan-owned one
        self.workspace = workspace
        wp, wn = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
        descs = _descs(images)
        _check(lib().deconv_plan_create(ctypes.byref(self.handle), len(images), descs, ctypes.byref(self.opts),
                                        _stream_ptr(self.stream), wp, wn), "plan_create")

    @property
    def batch(self):
        return len(self.images)

    def close(self):
        if self.handle:
            lib().deconv_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stats(self, want):
        return (Stats * self.batch)() if want else None

    @staticmethod
    def _stats_list(st):
        if st is None:
            return None
        return [dict(iters_done=s.iters_done, r_primal=s.r_primal, r_dual=s.r_dual, r_z=s.r_z, status=s.status,
                     mu=s.mu) for s in st]

    def run(self, y, mask, h, lam, mu, iters, x_out=None, ytilde_out=None, stats=False):
        dev = y.device
        x_out = x_out if x_out is not None else torch.empty(self.npx, dtype=torch.float32, device=dev)
        st = self._stats(stats)
        code = lib().deconv_admm_run(self.handle, _ptr(y), _ptr(mask), _ptr(h), _ptr(lam), _ptr(mu),
                                     int(iters), _ptr(x_out), _ptr(ytilde_out), st)
        # non-finite values (status 4) are reported per image in the stats
        _check(code, "admm_run", self._stats_list(st) if code == 4 else None)
        return x_out, self._stats_list(st)

    def cont(self, lam, mu, iters, x_out, ytilde_out=None, stats=False):
        st = self._stats(stats)
        code = lib().deconv_admm_continue(self.handle, _ptr(lam), _ptr(mu), int(iters), _ptr(x_out),
                                          _ptr(ytilde_out), st)
        _check(code, "admm_continue", self._stats_list(st) if code == 4 else None)
        return x_out, self._stats_list(st)

    def backward(self, y, mask, h, lam, mu, grad_x, run_id=0):
        """Reverse pass through the last run; run_id (from run_id() right
        after that run, 0 = unchecked) makes it fail with status 8 when the
        plan has run since."""
        dev = y.device
        gy = torch.empty(self.npx, dtype=torch.float32, device=dev)
        gl = torch.empty(self.batch, dtype=torch.float32, device=dev)
        gh = torch.empty(sum(self.ksq), dtype=torch.float32, device=dev)
        _check(lib().deconv_admm_backward(self.handle, _ptr(y), _ptr(mask), _ptr(h), _ptr(lam), _ptr(mu),
                                          _ptr(grad_x), _ptr(gy), _ptr(gl), _ptr(gh), ctypes.c_uint64(run_id)),
               "admm_backward")
        return gy, gl, gh

    def run_id(self):
        """Id of the state the plan holds (0: none)."""
        out = ctypes.c_uint64(0)
        _check(lib().deconv_plan_run_id(self.handle, ctypes.byref(out)), "run_id")
        return out.value

    def blur_spectrum(self, h):
        out = torch.empty(2 * self.npx, dtype=torch.float32, device=h.device)
        _check(lib().deconv_blur_spectrum(self.handle, _ptr(h), _ptr(out)), "blur_spectrum")
        return out

    def state_export(self, device):
        yt = torch.empty(self.npx, dtype=torch.float32, device=device)
        v = torch.empty(2 * self.npx, dtype=torch.float32, device=device)
        d = torch.empty(2 * self.npx, dtype=torch.float32, device=device)
        _check(lib().deconv_state_export(self.handle, _ptr(yt), _ptr(v), _ptr(d)), "state_export")
        return yt, v, d

    def schedule(self):
        """(row, column) launch shapes: 1 = per line length, 2 = one launch,
        3 = hybrid (short lengths share one launch)."""
        out = (ctypes.c_int32 * 2)()
        _check(lib().deconv_plan_schedule(self.handle, out), "schedule")
        return tuple(out)

    def tiles(self):
        """(row tile class 1/2, threads per half-height row tile, threads per
        long column tile, 1 if the whole-image-in-LDS path runs) in use."""
        out = (ctypes.c_int32 * 4)()
        _check(lib().deconv_plan_tiles(self.handle, out), "tiles")
        return tuple(out)

    def separable(self):
        """Per image: 1 if the column pass takes the blur spectrum as the
        product of 1-D spectra (separable_blur), as set by the last run."""
        out = (ctypes.c_int32 * self.batch)()
        _check(lib().deconv_plan_separable(self.handle, out), "separable")
        return tuple(out)

    def kernel_times(self):
        """(row_ms, row_launches, col_ms, col_launches) since the last call
        (plan created with profile=1; launches outside graphs only)."""
        out = (ctypes.c_double * 4)()
        _check(lib().deconv_plan_kernel_times(self.handle, out), "kernel_times")
        return tuple(out)

    def bwd_kernel_times(self):
        """As kernel_times, for the reverse row and column passes."""
        out = (ctypes.c_double * 4)()
        _check(lib().deconv_plan_bwd_kernel_times(self.handle, out), "bwd_kernel_times")
        return tuple(out)

    def state_import(self, mask, h, yt, v, d):
        """Load a resumable state (ytilde, v, d as packed device tensors, v and d
        interleaved per pixel) so that `cont` continues from it; `mask` is
        the packed byte mask (None when every image's mask is implicit)."""
        _check(lib().deconv_state_import(self.handle, _ptr(mask), _ptr(h), _ptr(yt), _ptr(v), _ptr(d)),
               "state_import")

    # helpers to split packed outputs per image
    def split(self, flat, per_px=1):
        out, o = [], 0
        for b, d in enumerate(self.images):
            n = self.sizes[b] * per_px
            shape = (d["height"], d["width"]) if per_px == 1 else (d["height"], d["width"], per_px)
            out.append(flat[o:o + n].view(*shape))
            o += n
        return out


def run_static(images, y, mask, h, lam, mu, iters, x_out, ytilde_out=None, stats=False, stream=None, **opts):
    """deconv_admm_run_static: one whole run (plan, setup, iterations) whose
    workspace is the library's static device array: the call allocates no
    device memory (x_out and the optional ytilde_out are the caller's)."""
    o = default_options(**opts)
    d = _descs(images)
    st = (Stats * len(images))() if stats else None
    _check(lib().deconv_admm_run_static(len(images), d, ctypes.byref(o), _stream_ptr(stream), _ptr(y), _ptr(mask),
                                        _ptr(h), _ptr(lam), _ptr(mu), int(iters), _ptr(x_out), _ptr(ytilde_out), st),
           "admm_run_static")
    return x_out, Plan._stats_list(st)


def fft2(data, inverse=False, stream=None):
    """In-place batched 2-D complex DFT of a complex64 tensor [count, H, W]
    (or [H, W]) with the library's FFT; unnormalised both ways."""
    assert data.dtype == torch.complex64 and data.is_cuda and data.is_contiguous()
    shp = data.shape
    t = data.view(-1, shp[-2], shp[-1])
    _check(lib().deconv_fft2(t.shape[0], shp[-2], shp[-1], ctypes.c_void_p(t.data_ptr()), int(inverse),
                             _stream_ptr(stream)), "fft2")
    return data


class DeconvADMM(torch.autograd.Function):
    """x = partial-ADMM deconvolution after `iters` iterations, differentiable
    with respect to y, h and lambda through the library's adjoint kernels.
    The plan must have been created with ckpt_every > 0 and max_iters >= iters."""

    @staticmethod
    def forward(ctx, y, h, lam, plan, mask, mu, iters):
        x, _ = plan.run(y, mask, h, lam, mu, iters)
        ctx.plan = plan
        # the reverse pass replays this run's checkpoints: if the plan runs
        # again before backward(), the library refuses (status 8)
        ctx.run_id = plan.run_id()
        ctx.save_for_backward(y, h, lam, mu)
        ctx.mask = mask
        return x

    @staticmethod
    def backward(ctx, gx):
        y, h, lam, mu = ctx.saved_tensors
        gy, gl, gh = ctx.plan.backward(y, ctx.mask, h, lam, mu, gx.contiguous(), run_id=ctx.run_id)
        return gy, gh, gl, None, None, None, None


def admm(y, h, lam, plan, mask, mu, iters):
    return DeconvADMM.apply(y, h, lam, plan, mask, mu, iters)
