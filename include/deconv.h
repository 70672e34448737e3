/*
 * deconv.h -- C ABI of the MI355X partial-ADMM deconvolution library.
 *
 * The library runs the "partial ADMM" of Simoes, Almeida, Bioucas-Dias and
 * Chanussot, "A Framework for Fast Image Deconvolution with Incomplete
 * Observations" (arXiv 1602.01410), Sec. II-B, eqs. (admm_aprox_1)-(admm_aprox_4)
 * with the closed forms (dual_x_iter_resolved_boundaries) and
 * (dual_z_iter_resolved_boundaries) and the over-relaxed z-update that follows
 * them, and the isotropic TV regulariser of Sec. III-B.
 *
 * Problem (Sec. I-A, model (4); Sec. II-A): the sharp image x lives on a
 * periodic "extended" domain of height x width = m' x n' pixels.  The blurred
 * image on that domain is H x (circular convolution with the (2b+1)^2 kernel h
 * centred at the origin); only some of its pixels are observed:
 *     y = M_y H x + n,
 * and the others (z) are estimated along with x.  The method minimises
 *     1/2 | [y; z] - H x |^2 + lambda sum_j sqrt((D_h x)_j^2 + (D_v x)_j^2)
 * with one block-Gauss-Seidel pass (x-step then z-step) per ADMM iteration.
 * The paper leaves several choices open; this library takes:
 *   - D_h, D_v: periodic forward differences, x[i,j+1]-x[i,j], x[i+1,j]-x[i,j];
 *   - vector soft threshold of u = D x^{i+1} + d^i with tau = lambda / mu
 *     (|u| <= tau gives v = 0);
 *   - z-update z <- z + alpha (M_z H x - z) (alpha = 2 is the paper's practice,
 *     alpha = 1 the exact minimisation);
 *   - initial state: observed pixels keep y, unobserved pixels inside the
 *     central m x n region take the mean of the observed pixels, unobserved
 *     pixels of the band of width b copy the nearest central pixel (Sec. III-B,
 *     "repeating the border pixels"); x^0 = that image, v^0 = D x^0, d^0 = 0;
 *   - the output x^N is the result of the N-th x-step.
 *
 * Memory: every pointer argument documented as "device" is HIP device memory
 * owned by the caller; the library never frees or retains it beyond the call
 * (except the workspace, retained for the plan's lifetime).  "host" pointers are
 * read during the call only.  Execution is asynchronous on the plan's stream
 * unless stated otherwise.  A plan is not thread-safe.
 *
 * Images of a batch are packed back to back: image b occupies
 * height_b * width_b consecutive elements (row-major) starting at
 * sum_{c<b} height_c * width_c.  Blur kernels are packed the same way with
 * ksize_b^2 elements each.
 *
 * Supported sizes: every height and width must be 2^a * 3^c with c <= 2 and
 * 8 <= size <= 2048 (DECONV_ERR_UNSUPPORTED_SIZE otherwise); ksize odd,
 * 1 <= ksize, and 2 * (ksize / 2) < min(height, width).
 *
 * Errors: argument errors detected on the host return synchronously and leave
 * the plan unchanged.  HIP errors return DECONV_ERR_HIP.  Non-finite residuals
 * found on the device are reported in deconv_stats.status and by the next
 * synchronising call.
 */
#ifndef DECONV_H
#define DECONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DECONV_OK = 0,
  DECONV_ERR_INVALID_ARG = 1,      /* null pointer, bad option, lambda < 0, mu <= 0, ... */
  DECONV_ERR_UNSUPPORTED_SIZE = 2, /* length not 2^a 3^c (c <= 2) in [8, 2048], bad ksize */
  DECONV_ERR_SINGULAR = 3,         /* sum(h) == 0: H^T H + mu D^T D singular at DC (Sec. III-B) */
  DECONV_ERR_NONFINITE = 4,        /* NaN / Inf reached the residuals */
  DECONV_ERR_NO_CHECKPOINTS = 5,   /* backward without a checkpointed forward run */
  DECONV_ERR_HIP = 6,              /* a HIP runtime call failed */
  DECONV_ERR_OOM = 7,              /* workspace too small / allocation failed */
  DECONV_ERR_STATE = 8             /* call order violated (e.g. continue before run) */
} deconv_status;

enum {
  DECONV_MASK_BOUNDARY = 0, /* unknown boundaries: only the central m x n region observed */
  DECONV_MASK_EXPLICIT = 1, /* caller's byte mask over the whole extended grid (1 = observed) */
  DECONV_MASK_DECIMATE = 2  /* boundary + super-resolution: central pixels (b+s*i, b+s*j) only */
};

typedef struct deconv_plan_s* deconv_plan; /* opaque */

/* One image of a batch. */
typedef struct {
  int32_t height, width; /* m', n': the periodic extended domain (= sharp image size) */
  int32_t ksize;         /* 2b+1: blur support, odd */
  int32_t mask_kind;     /* DECONV_MASK_* */
  int32_t decim;         /* s for DECONV_MASK_DECIMATE (>= 1), ignored otherwise */
} deconv_image_desc;

typedef struct {
  float alpha;          /* z over-relaxation (default 2.0; must be in (0, 2]) */
  int32_t check_every;  /* compute FP64 residuals every K iterations (0 = never) */
  double tol_primal;    /* stop an image when |d'-d|/sqrt(2N) <= tol_primal ... */
  double tol_dual;      /* ... and |v'-v|/sqrt(2N) <= tol_dual (0 = never stop) */
  int32_t use_graph;    /* capture the iteration in a hipGraph (default 1) */
  int32_t batched;      /* 1: one launch per phase for all images of a length
                           (default); 0: one launch per image per phase */
  int32_t ckpt_every;   /* keep the state every k iterations for the backward
                           pass (0 = no backward support); needs bgs_passes = 1,
                           adapt_t = 0 and warm_iters = 0 */
  int32_t max_iters;    /* upper bound on iters, sizes the checkpoint store */
  int32_t profile;      /* 1: bracket every row / column pass launched outside a
                           graph with HIP events (read by deconv_plan_kernel_times) */
  int32_t schedule;     /* batched launch shape of each pass: 0 = autotune at
                           plan creation (default), 1 = one launch per line
                           length, 2 = one launch for all lengths, 3 = one
                           launch for the lengths with few tiles and one per
                           other length */
  const char* tune_cache; /* nullable: file of autotuning decisions, read before
                           tuning and appended after (one line per batch
                           signature) */
  int32_t bgs_passes;   /* block-Gauss-Seidel passes of the x- and z-steps per
                           iteration, v and d frozen between them (Sec. III-B;
                           "Proposed-AD" takes b of a (2b+1)^2 blur), 1..64 for
                           every image; 0: each image its own b = ksize/2 (at
                           least 1), as Sec. III-B sets them (images with fewer
                           passes than the batch's most skip the extra inner
                           ones).  Default 1. */
  double adapt_t;       /* > 0: adapt mu every iteration with threshold t and
                           rescale d (eq. (varying_penalty), t = 3 in Sec.
                           III-B); 0 = fixed mu (default) */
  int32_t warm_iters;   /* > 0: start z from that many steps of the quadratic
                           warm start of eqs. (ini_x), (ini_z) (Sec. III-B uses
                           100); 0 = edge replication only (default) */
  float warm_tau;       /* tau of the warm start (default 1e-3) */
  int32_t channels;     /* C > 1: colour images with vectorial TV (Sec. III-C,
                           demosaicing).  Images c*C .. c*C+C-1 of the batch are
                           the channels of one colour image: same size and
                           ksize, each with its own data, mask and blur; the
                           prox is one soft threshold over the 2C differences
                           of a pixel, with lambda and mu of the first channel
                           (pass equal values).  C <= 4; no reverse pass.
                           Default 1. */
  int32_t spectra_hint; /* cache hint for the spectra the two passes hand each
                           other: 0 = automatic (non-temporal stores when both
                           spectrum buffers together take at most 40 MB, i.e.
                           the working set stays in the last-level cache),
                           1 = ordinary stores, 2 = non-temporal stores.
                           Results do not depend on it.  Default 0. */
  int32_t row_tiles;    /* row-pass tile height: 0 = autotuned with the launch
                           shapes (schedule 0) or chosen by the plan's size,
                           1 = the default height (about 4096 pixels per
                           tile), 2 = half of it (plans whose images share
                           one width and keep no checkpoints; otherwise 1).
                           Results do not depend on it.  Default 0. */
  int32_t row_threads;  /* threads per half-height row tile: 0 = as
                           row_tiles, 512 or 1024.  Default 0. */
  int32_t col_threads;  /* threads per column tile of length >= 512: 0 = as
                           row_tiles, 256 or 512.  Default 0. */
  int32_t small_images; /* Plans whose images are all square with a side
                           of 32, 48, 64, 72 or 96 and that use one BGS pass,
                           a fixed penalty, grey images and no checkpoints
                           can run up to 200 iterations (one check period
                           with tolerances) in one workgroup per image, the
                           image held in LDS (one launch instead of two per
                           iteration).  2 (default): such plans whose sides
                           are all at most 72 take it (on MI355X it is 1.1x
                           (72^2) to 2.7x (32^2) as fast there; one 96^2
                           image is faster on the two-pass kernels); 1:
                           every such plan takes it; 0: never.  The
                           iterates agree with the two-pass kernels' to
                           within rounding. */
  int32_t separable_blur; /* 1 (default): the column pass of an image whose
                           blur kernel is the outer product of two 1-D kernels
                           (to within 1e-6 of its largest tap: box and
                           Gaussian blurs) takes the blur spectrum as the
                           product of their 1-D spectra, U(ky) V(kx), computed
                           at setup, instead of reading the stored 2-D half
                           spectrum (one 8-byte value per frequency and
                           iteration less HBM traffic); 0: always the stored
                           spectrum.  Results agree to rounding. */
} deconv_options;

typedef struct {
  int32_t iters_done;   /* iterations applied to this image */
  double r_primal;      /* |d' - d| at the last check (FP64) */
  double r_dual;        /* |v' - v| at the last check */
  double r_z;           /* |z' - z| at the last check */
  int32_t status;       /* DECONV_OK or DECONV_ERR_NONFINITE */
  float mu;             /* penalty after the last iteration (differs from the
                           input only with opt.adapt_t > 0) */
} deconv_stats;

/* Fill *opt with the defaults above. */
deconv_status deconv_options_default(deconv_options* opt);

/* Bytes of device workspace a plan for this batch needs (host call).
   desc: host array [batch]. */
deconv_status deconv_plan_workspace_size(int32_t batch, const deconv_image_desc* desc,
                                         const deconv_options* opt, size_t* bytes);

/* Create a plan (host call; synchronous).  desc: host array [batch], copied.
   opt: NULL for defaults.  stream: hipStream_t (NULL = default stream) on
   which every later call runs.  workspace: device buffer of at least
   deconv_plan_workspace_size bytes, owned by the caller and used until
   deconv_plan_destroy; NULL makes the plan allocate (and free) its own. */
deconv_status deconv_plan_create(deconv_plan* out, int32_t batch, const deconv_image_desc* desc,
                                 const deconv_options* opt, void* stream, void* workspace,
                                 size_t workspace_bytes);

deconv_status deconv_plan_destroy(deconv_plan p);

/*
 * Blur spectrum setup + initial state + `iters` partial-ADMM iterations.
 *   y      device float, packed images: observed values (others ignored)
 *   mask   device uint8, packed images, 1 = observed; read only for images of
 *          kind DECONV_MASK_EXPLICIT (may be NULL if there are none)
 *   h      device float, packed kernels (convolution, centre (b, b)); each
 *          must have a non-zero sum, else DECONV_ERR_SINGULAR.  The host
 *          checks the sums once the run's work is queued (waiting only for
 *          the spectrum setup; plans given a workspace wait for it before
 *          queuing the iterations); on DECONV_ERR_SINGULAR the call returns
 *          after the queued work has finished and the outputs and the
 *          plan's state are unspecified
 *   lambda device float [batch], >= 0 (TV weight)
 *   mu     device float [batch], > 0 (ADMM penalty)
 *   iters  >= 1
 *   x_out  device float, packed: x^iters on the whole extended domain
 *   ytilde_out  device float, packed, nullable: [y; z] after the last z-step
 *   stats  host array [batch], nullable; when given the call synchronises
 *          and fills it.  An image whose status is DECONV_ERR_NONFINITE
 *          stopped early and its x_out is unspecified.
 * The state (ytilde, v, d) stays in the plan for deconv_admm_continue,
 * deconv_state_export and, with checkpoints, deconv_admm_backward.
 */
deconv_status deconv_admm_run(deconv_plan p, const float* y, const uint8_t* mask, const float* h,
                              const float* lambda, const float* mu, int32_t iters, float* x_out,
                              float* ytilde_out, deconv_stats* stats);

/* `iters` more iterations from the plan's current state (lambda / mu are read
   again).  Outputs as deconv_admm_run.  Plans with explicit masks reuse the mask
   pointer of the last deconv_admm_run, which must still be valid
   (DECONV_ERR_STATE if there was no run).  With opt.adapt_t > 0 the penalty
   goes on from the last adapted value, for which d is scaled (eq.
   (varying_penalty)): `mu` is then ignored, except after deconv_state_import,
   where it starts the adaptation.  So run(a) followed by continue(b) equals
   run(a + b). */
deconv_status deconv_admm_continue(deconv_plan p, const float* lambda, const float* mu,
                                   int32_t iters, float* x_out, float* ytilde_out,
                                   deconv_stats* stats);

/* Copy the resumable state w = [z; v; d] (Appendix B) out of / into the plan.
   ytilde: packed float (observed pixels hold y); v, d: packed float2 per
   pixel (horizontal, vertical).  Import also takes the observation mask
   (device bytes, packed; null for plans whose masks are all implicit, and
   kept, like deconv_admm_run's, for deconv_admm_continue) and h for the
   spectrum (device float, packed); the buffers are copied, the caller keeps
   them.  After an import deconv_admm_continue starts from this state; the
   checkpoints of an earlier run are dropped.  Export needs a run or an import
   first (DECONV_ERR_STATE). */
deconv_status deconv_state_export(deconv_plan p, float* ytilde, float* v, float* d);
deconv_status deconv_state_import(deconv_plan p, const uint8_t* mask, const float* h,
                                  const float* ytilde, const float* v, const float* d);

/*
 * Reverse mode through the last deconv_admm_run (which must have had
 * opt.ckpt_every > 0 and iters <= opt.max_iters).  Inputs are those of that
 * run; grad_x = dL/dx^N (device float, packed).  Outputs (device):
 *   grad_y       packed float, dL/dy, zero at unobserved pixels
 *   grad_lambda  float [batch]
 *   grad_h       packed float [ksize_b^2 per image]
 *   run_id       the id deconv_plan_run_id gave right after that run: if the
 *                plan has run, continued or imported a state since, the
 *                checkpoints are another run's and the call returns
 *                DECONV_ERR_STATE; 0 skips the check
 * Recomputes the forward iterations between checkpoints; with opt.use_graph
 * the whole reverse pass is captured once per argument set as one graph and
 * replayed on later calls.  The reverse pass
 * uses the forward state (ytilde, v, d) as scratch: afterwards
 * deconv_admm_continue and deconv_state_export return DECONV_ERR_STATE until
 * the next run.  The checkpoints stay, so the same reverse pass can be asked
 * for again.  DECONV_ERR_NO_CHECKPOINTS without a checkpointed run.
 */
deconv_status deconv_admm_backward(deconv_plan p, const float* y, const uint8_t* mask,
                                   const float* h, const float* lambda, const float* mu,
                                   const float* grad_x, float* grad_y, float* grad_lambda,
                                   float* grad_h, uint64_t run_id);

/* Id of the state the plan holds (host call): a new, process-unique value
   after every deconv_admm_run, deconv_admm_continue and deconv_state_import;
   0 when the plan holds no state (before a run, after a reverse pass). */
deconv_status deconv_plan_run_id(deconv_plan p, uint64_t* out);

/* Blur spectrum H^ = DFT2(h embedded circularly centred at the origin) for
   every image (device float2 packed, full height x width per image): by
   direct sums over the taps (FP32, one launch for the batch) when every
   kernel has at most 65 taps a side, else with the library's own FFT, as the
   plan's runs compute the half of it they read (except that for a kernel
   taken as separable, see separable_blur, a run forms it as the product of
   the two 1-D spectra, equal to within about 1e-6 relative).  Synchronous.
   The plan's own blur spectrum, state and checkpoints are left as they
   were. */
deconv_status deconv_blur_spectrum(deconv_plan p, const float* h, float* spectrum_out);

/* Batched 2-D complex DFT with the library's FFT (unnormalised; inverse = 1
   uses exp(+2 pi i jk/n)).  data: device float2 [count][height][width],
   transformed in place.  Same size rules as images.  Runs on `stream`. */
deconv_status deconv_fft2(int32_t count, int32_t height, int32_t width, float* data,
                          int32_t inverse, void* stream);

/* With opt.profile = 1: GPU time of the row and column passes launched since
   the last call, from HIP events on the plan's stream (synchronises).
   out[0] = row-pass milliseconds, out[1] = row-pass launches,
   out[2] = column-pass milliseconds, out[3] = column-pass launches.
   Passes replayed inside a graph are not bracketed.  On the
   whole-image-in-LDS path (deconv_plan_tiles out[3] = 1) out[0..1] count
   its launches (up to 200 iterations each) and out[2..3] are 0. */
deconv_status deconv_plan_kernel_times(deconv_plan p, double* out);

/* As deconv_plan_kernel_times for the passes of the reverse pass
   (deconv_admm_backward): out[0] = reverse row-pass milliseconds, out[1] =
   launches, out[2] = reverse column-pass milliseconds, out[3] = launches.
   With opt.profile = 1 the reverse pass runs outside graphs. */
deconv_status deconv_plan_bwd_kernel_times(deconv_plan p, double* out);

/* Launch shapes in use (after autotuning): out[0] = row pass, out[1] =
   column pass, each 1 (one launch per line length), 2 (one launch for all
   lengths) or 3 (hybrid, see deconv_options.schedule).  On the
   whole-image-in-LDS path these are the shapes of the two-pass kernels that
   a warm start runs.  Host call. */
deconv_status deconv_plan_schedule(deconv_plan p, int32_t* out);

/* Tile knobs in use (after autotuning), host call: out[0] = row tile
   height class (1 default, 2 half), out[1] = threads per half-height row
   tile (512 or 1024), out[2] = threads per long column tile (256 or 512),
   out[3] = 1 if the plan runs the whole-image-in-LDS path (small_images). */
deconv_status deconv_plan_tiles(deconv_plan p, int32_t* out);

/* Which images' column passes take the blur spectrum as the product of 1-D
   spectra (deconv_options.separable_blur): out[b] = 1 or 0, host array
   [batch], as set by the last run or state import (0 before any).  Host
   call; synchronises the plan's stream. */
deconv_status deconv_plan_separable(deconv_plan p, int32_t* out);

const char* deconv_status_str(deconv_status s);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * deconv_plan_create + deconv_admm_run + deconv_plan_destroy in one call,
 * whose workspace is a device array inside the library (64 MiB, one copy per
 * GPU, held until the process ends) instead of an allocation.  Arguments as
 * those three calls; the call allocates no device memory and creates no
 * streams, events or graphs, so opt.use_graph, opt.profile and opt.tune_cache
 * are ignored and schedule 0 (autotuning) means 3 (hybrid).  opt.ckpt_every
 * must be 0 (DECONV_ERR_INVALID_ARG): no plan is left for a reverse pass.  A
 * batch whose workspace (deconv_plan_workspace_size) exceeds 64 MiB returns
 * DECONV_ERR_OOM (one 1024 x 1024 image fits).  Host-side bookkeeping uses the
 * C++ heap.  Every call on one GPU uses the same array: calls that overlap on
 * one GPU (other streams, other threads) race and give undefined results;
 * calls on one stream are ordered.  The array keeps the last call's contents;
 * each call clears what it needs cleared.
 */
deconv_status deconv_admm_run_static(int32_t batch, const deconv_image_desc* desc,
                                     const deconv_options* opt, void* stream, const float* y,
                                     const uint8_t* mask, const float* h, const float* lambda,
                                     const float* mu, int32_t iters, float* x_out, float* ytilde_out,
                                     deconv_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* DECONV_H */
