// Host side of the partial-ADMM library: plans, workspace layout, launch
// schedule and the C ABI declared in include/deconv.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <fstream>
#include <sstream>
#include <array>
#include <new>
#include <vector>
#include <cstdint>
#include <atomic>

#include "../../include/deconv.h"
#include "launch.hpp"
#include "small.hpp"
#include "setup.hpp"
#include "backward_setup.hpp"

using namespace dcv;

#define HIPCHK(expr)                                                      \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "deconv: %s failed: %s (%s:%d)\n", #expr,           \
              hipGetErrorString(e_), __FILE__, __LINE__);                 \
      return DECONV_ERR_HIP;                                              \
    }                                                                     \
  } while (0)

#define STCHK(expr)                                \
  do {                                             \
    deconv_status s_ = (expr);                     \
    if (s_ != DECONV_OK) return s_;                \
  } while (0)

static size_t fftrow_lds_bytes(int L) {
  int lpw = std::max(1, std::min(32, 4096 / L));
  return (size_t)(lpw * lstride(L) + L) * sizeof(float2);
}
static size_t fftcol_lds_bytes(int L) { return (size_t)(2 * c_for(L) * lstride(L) + L) * sizeof(float2); }

static hipError_t launch_fft_rows(int L, float2* data, long long nrows, const float2* tw, int inverse,
                                  hipStream_t s) {
  int lpw = std::max(1, std::min(32, 4096 / L));
  int grid = (int)((nrows + lpw - 1) / lpw);
  void* args[] = {&data, &nrows, &tw, &inverse};
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(fft_rows_kernel<n>, grid, fftrow_lds_bytes(n), s, args, kNT);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}
static hipError_t launch_fft_cols(int L, float2* data, int W, int count, const float2* tw, int inverse,
                                  hipStream_t s) {
  int cw = 2 * c_for(L);
  int grid = count * ((W + cw - 1) / cw);
  void* args[] = {&data, &W, &count, &tw, &inverse};
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(fft_cols_kernel<n>, grid, fftcol_lds_bytes(n), s, args, kNT);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

// LDS available to one workgroup; without a device (host-only checks) assume
// the 160 KiB of gfx950, the only target this library is built for
static int max_lds_bytes() {
  static int v = -1;
  if (v < 0) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 163840;
    v = (int)p.sharedMemPerBlock;
  }
  return v;
}

// twiddle tables exp(-2 pi i t / L), computed in double, stored as float
static void twiddles(int L, std::vector<float2>& out) {
  out.resize(L);
  for (int t = 0; t < L; ++t) {
    double a = -2.0 * M_PI * (double)t / (double)L;
    out[t] = make_float2((float)cos(a), (float)sin(a));
  }
}

// process-wide twiddle cache for the diagnostic FFT entry point (per device)
static std::mutex g_tw_mu;
static std::map<std::pair<int, int>, float2*> g_tw;
static const float2* cached_twiddles(int L) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto key = std::make_pair(dev, L);
  auto it = g_tw.find(key);
  if (it != g_tw.end()) return it->second;
  std::vector<float2> h;
  twiddles(L, h);
  float2* d = nullptr;
  if (hipMalloc(&d, sizeof(float2) * L) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), sizeof(float2) * L, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  g_tw[key] = d;
  return d;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// one launch of a pass: line length L (-Lmax = several lengths up to Lmax,
// dispatched per tile) over tiles [tile0, tile0 + ntiles) of the tile table
struct Group {
  int L;
  long long tile0;
  int ntiles;
  size_t lds;
  int rt;   // row pass: rows per tile (0 = rt_for(L))
};

// A tile of a pass: image, first row (row pass) or column block (column
// pass), and its relative cost.
struct TileRef {
  int img, pos;
  double cost;
};

// Dispatch order of one launch.  Workgroups go round-robin to the 8 XCDs
// (block b to XCD b mod 8), each with its own L2.  Every XCD gets contiguous
// runs of an image's tiles (neighbouring row tiles share halo rows, which then
// meet in one L2); images with many tiles are split into 8 runs; runs are
// given to the least-loaded XCD, largest first; within an XCD the costliest
// tiles come first.  Slots left over are padding (image -1).
static void xcd_schedule(const std::vector<std::vector<TileRef>>& images, std::vector<int4>& out) {
  constexpr int kXcd = 8;
  struct Run { int img; size_t a, b; double cost, tile_cost; };
  std::vector<Run> runs;
  for (size_t i = 0; i < images.size(); ++i) {
    const auto& t = images[i];
    if (t.empty()) continue;
    const size_t n = t.size();
    const size_t parts = n >= 2 * kXcd ? kXcd : 1;
    for (size_t k = 0; k < parts; ++k) {
      size_t a = n * k / parts, b = n * (k + 1) / parts;
      double c = 0;
      for (size_t q = a; q < b; ++q) c += t[q].cost;
      runs.push_back(Run{(int)i, a, b, c, t[a].cost});
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) { return x.cost > y.cost; });
  std::vector<double> load(kXcd, 0.0);
  std::vector<std::vector<Run>> per(kXcd);
  for (const Run& r : runs) {
    int best = 0;
    for (int x = 1; x < kXcd; ++x)
      if (load[x] < load[best]) best = x;
    load[best] += r.cost;
    per[best].push_back(r);
  }
  size_t maxlen = 0;
  std::vector<std::vector<int4>> lists(kXcd);
  for (int x = 0; x < kXcd; ++x) {
    std::stable_sort(per[x].begin(), per[x].end(),
                     [](const Run& u, const Run& w) { return u.tile_cost > w.tile_cost; });
    for (const Run& r : per[x])
      for (size_t q = r.a; q < r.b; ++q) lists[x].push_back(make_int4(r.img, images[r.img][q].pos, 0, 0));
    maxlen = std::max(maxlen, lists[x].size());
  }
  for (size_t k = 0; k < maxlen; ++k)
    for (int x = 0; x < kXcd; ++x)
      out.push_back(k < lists[x].size() ? lists[x][k] : make_int4(-1, 0, 0, 0));
}

struct deconv_plan_s {
  int batch = 0;
  std::vector<deconv_image_desc> desc;
  deconv_options opt{};
  hipStream_t stream = nullptr;     // the caller's stream: every call runs here
  hipStream_t cap_stream = nullptr; // private stream, used only to capture graphs
  hipStream_t ls = nullptr;         // stream the launch helpers enqueue on
  // graph branches: while a graph is captured, the launches of one pass
  // (one per line length) fork onto these streams and join again, so that
  // their kernels overlap in the replayed graph
  std::vector<hipStream_t> side;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  std::vector<ImgMeta> meta;

  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;

  // device views into the workspace
  ImgMeta* d_meta = nullptr;
  int4* d_tiles = nullptr;
  float* yt = nullptr;
  float2* dbuf[2] = {nullptr, nullptr};
  float2* v = nullptr;
  float4* specA = nullptr;
  float4* specB = nullptr;
  float2* hh = nullptr;
  float* tab = nullptr;
  int* npass = nullptr;       // per image: BGS passes per iteration
  int max_pass = 1;
  float2* hsep = nullptr;     // separable blurs: 1-D spectra U, V (offsets of tab)
  int* sep = nullptr;         // per image: 1 = the column pass uses U V
  float2* tw = nullptr;
  double* partials = nullptr;
  int* done = nullptr;
  int* nonfinite = nullptr;
  int* iters_done = nullptr;
  int* stop_buf = nullptr;    // d buffer holding a stopped image's last d
  double* res = nullptr;
  double* mean = nullptr;     // per image and row block: observed sum, count
  long long* goff = nullptr;
  long long* hoff = nullptr;
  float2* hsum = nullptr;     // DC term of each spectrum (host check)
  // plans that allocate their own memory: the DC terms come back through
  // pinned memory, checked once the run's work is queued (hsum_ev)
  float2* hsum_host = nullptr;
  hipEvent_t hsum_ev = nullptr;
  bool hsum_pending = false;
  float* mu_cur = nullptr;    // adaptive penalty: current mu per image
  float* dscale = nullptr;    // adaptive penalty: rescale of d per image
  // whole-image-in-LDS path: image indices grouped by side, one launch per
  // group (side, first, count)
  bool small = false;
  int* d_small = nullptr;
  std::vector<std::array<int, 3>> small_groups;
  // backward support
  float* ck_yt = nullptr;     // checkpoints: ytilde, v, d per stored iteration
  float2* ck_v = nullptr;
  float2* ck_d = nullptr;
  float2* seg_u = nullptr;    // per iteration of a segment: u = D x + d
  float4* seg_spec = nullptr; // per iteration of a segment: (Y, X) half spectra
  float2* adj_a = nullptr;    // backward: ub ping-pong
  float2* adj_b = nullptr;
  float2* adj_vb = nullptr;   // backward: adjoint state at segment boundaries
  float2* adj_db = nullptr;
  double* adj_mean = nullptr; // backward: per-block partials of the mean adjoint
  float* adj_z = nullptr;
  float* adj_y = nullptr;
  double2* adj_S = nullptr;   // accumulated spectral h-gradient (half, tiled, FP64)
  double2* adj_T = nullptr;   // h-gradient: row-stage sums (max m' K per image, FP64)
  double2* tw64 = nullptr;    // FP64 twiddle tables (same offsets as tw), for the tap sums
  double* adj_lam = nullptr;  // per row tile partial of dL/dlambda
  int nck = 0;                // checkpoints stored

  long long total_px = 0, total_sp = 0, total_hh = 0, total_tab = 0, total_tw = 0, total_rt = 0;
  long long total_h = 0;      // packed blur kernel elements
  std::vector<long long> hoff_h;
  std::map<int, long long> tw_off;
  // batched launch shapes: [0] one group per line length, [1] one group for
  // all lengths; row_sched / col_sched pick one (autotuned)
  std::vector<Group> row_sets[3], col_sets[3];  // per length, one launch, hybrid
  int row_sched = 0, col_sched = 0;
  std::vector<Group> row_groups, col_groups;  // the chosen sets
  std::vector<int4> h_tiles;  // all tile tables, uploaded at plan creation
  std::vector<std::vector<Group>> row_img, col_img;  // per-image launches (batched = 0)

  const uint8_t* mask = nullptr;  // explicit masks of the last run (caller-owned)
  int cur_d = 0;        // index of the d buffer holding the current state
  int max_height = 0;   // tallest image of the batch
  bool have_state = false;
  bool wide_col = false;     // column tiles of kNTCWide threads (few tiles)
  bool wide_row = false;     // half-height row tiles of kNTRWide threads (few tiles)
  // autotuner's choices of the tile knobs (-1: none, the heuristics decide)
  int tune_half = -1, tune_wrow = -1, tune_wcol = -1;
  int last_iters = 0;   // iterations of the last run (for the backward)
  bool ck_valid = false;
  bool mu_valid = false;   // mu_cur holds an adapted penalty (adapt_t > 0)
  uint64_t run_id = 0;     // id of the state the plan holds (0: none)
  uint64_t ck_run_id = 0;  // id of the run whose checkpoints the plan holds

  // per-launch timing (opt.profile): event pairs around row / column passes
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_row, ev_col, ev_brow, ev_bcol;
  std::vector<hipEvent_t> ev_pool;

  // graph cache: one executable graph per (check period, buffer parity,
  // argument pointers); replayed for every whole check period of a run
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
  // reverse passes: one graph per argument set and starting d parity, with
  // the d parity it ends on
  std::map<std::vector<uintptr_t>, std::pair<hipGraphExec_t, int>> bwd_graphs;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  size_t off_meta, off_tiles, off_yt, off_d0, off_d1, off_v, off_specA, off_specB, off_hh, off_tab, off_tw,
      off_part, off_done, off_nonf, off_itd, off_stopbuf, off_res, off_mean, off_goff, off_hoff, off_hsum, off_mu,
      off_dscale, off_small, off_npass, off_hsep, off_sep;
  size_t off_ck_yt, off_ck_v, off_ck_d, off_seg_u, off_seg_spec, off_adj_a, off_adj_b, off_adj_z, off_adj_y,
      off_adj_S, off_adj_lam, off_adj_vb, off_adj_db, off_adj_mean, off_tw64, off_adj_T;
  size_t total;
};

static deconv_status validate(int32_t batch, const deconv_image_desc* desc, const deconv_options* opt) {
  if (batch <= 0 || !desc) return DECONV_ERR_INVALID_ARG;
  if (opt) {
    if (!(opt->alpha > 0.f && opt->alpha <= 2.f)) return DECONV_ERR_INVALID_ARG;
    if (opt->check_every < 0 || opt->ckpt_every < 0 || opt->max_iters < 0) return DECONV_ERR_INVALID_ARG;
    if (opt->tol_primal < 0 || opt->tol_dual < 0) return DECONV_ERR_INVALID_ARG;
    if (opt->ckpt_every > 0 && opt->max_iters <= 0) return DECONV_ERR_INVALID_ARG;
    if (opt->schedule < 0 || opt->schedule > 3) return DECONV_ERR_INVALID_ARG;
    // the reverse pass replays every iteration: no early stopping with it
    if (opt->ckpt_every > 0 && (opt->tol_primal > 0 || opt->tol_dual > 0)) return DECONV_ERR_INVALID_ARG;
    if (opt->bgs_passes < 0 || opt->bgs_passes > 64) return DECONV_ERR_INVALID_ARG;
    if (!(opt->adapt_t >= 0.0) || opt->warm_iters < 0) return DECONV_ERR_INVALID_ARG;
    if (opt->warm_iters > 0 && !(opt->warm_tau > 0.f)) return DECONV_ERR_INVALID_ARG;
    // the reverse pass is derived for one pass, a fixed penalty and the plain
    // initial state
    if (opt->ckpt_every > 0 && (opt->bgs_passes != 1 || opt->adapt_t > 0 || opt->warm_iters > 0))
      return DECONV_ERR_INVALID_ARG;
    // colour groups: consecutive images of one size; no reverse pass
    if (opt->channels < 1 || opt->channels > kMaxChannels || batch % opt->channels != 0)
      return DECONV_ERR_INVALID_ARG;
    if (opt->channels > 1 && opt->ckpt_every > 0) return DECONV_ERR_INVALID_ARG;
    if (opt->spectra_hint < 0 || opt->spectra_hint > 2) return DECONV_ERR_INVALID_ARG;
    if (opt->row_tiles < 0 || opt->row_tiles > 2) return DECONV_ERR_INVALID_ARG;
    if (opt->row_threads != 0 && opt->row_threads != kNTR && opt->row_threads != kNTRWide)
      return DECONV_ERR_INVALID_ARG;
    if (opt->col_threads != 0 && opt->col_threads != kNTC && opt->col_threads != kNTCWide)
      return DECONV_ERR_INVALID_ARG;
    if (opt->small_images < 0 || opt->small_images > 2) return DECONV_ERR_INVALID_ARG;
    if (opt->separable_blur < 0 || opt->separable_blur > 1) return DECONV_ERR_INVALID_ARG;
    for (int b = 0; b < batch; ++b) {
      const deconv_image_desc& f = desc[b - b % opt->channels];
      if (desc[b].height != f.height || desc[b].width != f.width || desc[b].ksize != f.ksize)
        return DECONV_ERR_INVALID_ARG;
    }
  }
  for (int b = 0; b < batch; ++b) {
    const deconv_image_desc& d = desc[b];
    if (!supported_len(d.height) || !supported_len(d.width)) return DECONV_ERR_UNSUPPORTED_SIZE;
    if (d.ksize < 1 || d.ksize % 2 == 0) return DECONV_ERR_UNSUPPORTED_SIZE;
    if (2 * (d.ksize / 2) >= std::min(d.height, d.width)) return DECONV_ERR_UNSUPPORTED_SIZE;
    if (d.mask_kind < 0 || d.mask_kind > 2) return DECONV_ERR_INVALID_ARG;
    if (d.mask_kind == DECONV_MASK_DECIMATE && (d.decim < 1 || d.decim > 2048)) return DECONV_ERR_INVALID_ARG;
    if ((int)row_lds_bytes(d.width) > max_lds_bytes() || (int)col_lds_bytes(d.height) > max_lds_bytes())
      return DECONV_ERR_UNSUPPORTED_SIZE;
  }
  return DECONV_OK;
}

static int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, v = 0;
    n = (hipGetDevice(&dev) == hipSuccess &&
         hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            ? v
            : 256;
  }
  return n;
}

static bool has_half_rt(int L) {
  switch (L) {
#define DCV_CASE(n) case n: return true;
    DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return false;
}

// A plan whose images share one width takes tiles of half the rows (twice
// the workgroups, each with a shorter chain of dependent steps) when it has
// fewer default row tiles than two per compute unit (one 1024^2 image: 256),
// or fewer than six when the half tiles still hold 4 rows or more (measured:
// 16 x 512^2 gains 13%; 2048^2, whose half tiles are single rows with a whole
// halo line each, loses 9%).  Not with checkpoints: the reverse pass uses the
// default tiles.
static bool half_rt_allowed(const deconv_plan_s* p) {
  std::set<int> ws;
  for (auto& d : p->desc) ws.insert(d.width);
  return ws.size() == 1 && has_half_rt(*ws.begin()) && p->opt.ckpt_every == 0;
}

static bool half_rt_heuristic(const deconv_plan_s* p) {
  long long tiles = 0;
  for (auto& d : p->desc) tiles += (d.height + rt_for(d.width) - 1) / rt_for(d.width);
  return tiles < (rt_half(p->desc[0].width) >= 4 ? 6 : 2) * (long long)num_cus();
}

// row tiles of half height: forced by opt.row_tiles, else the autotuner's
// choice (tune_half), else the heuristic above
static bool use_half_rt(const deconv_plan_s* p) {
  if (!half_rt_allowed(p)) return false;
  if (p->opt.row_tiles > 0) return p->opt.row_tiles == 2;
  if (p->tune_half >= 0) return p->tune_half != 0;
  return half_rt_heuristic(p);
}

static void build_tiles(deconv_plan_s* p, bool half);

// build per-image metadata, tile tables and the workspace layout; the tile
// and partial tables are sized for either row tile height, so that the
// autotuner can switch between them without a new workspace
static void build_layout(deconv_plan_s* p, Layout& lay) {
  long long ntiles = 0, rt = 0;
  if (half_rt_allowed(p)) {
    for (bool h : {false, true}) {
      build_tiles(p, h);
      ntiles = std::max(ntiles, (long long)p->h_tiles.size());
      rt = std::max(rt, p->total_rt);
    }
  }
  build_tiles(p, use_half_rt(p));
  ntiles = std::max(ntiles, (long long)p->h_tiles.size());
  rt = std::max(rt, p->total_rt);
  const int B = p->batch;
  const long long px = p->total_px, sp = p->total_sp, hhp = p->total_hh, tab = p->total_tab, tw = p->total_tw;

  const size_t A = 256;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1), A); return r; };
  lay.off_meta = take(sizeof(ImgMeta) * B);
  lay.off_tiles = take(sizeof(int4) * ntiles);
  lay.off_yt = take(sizeof(float) * px);
  lay.off_d0 = take(sizeof(float2) * px);
  lay.off_d1 = take(sizeof(float2) * px);
  lay.off_v = take(sizeof(float2) * px);
  lay.off_specA = take(sizeof(float4) * sp);
  lay.off_specB = take(sizeof(float4) * sp);
  lay.off_hh = take(sizeof(float2) * hhp);
  lay.off_tab = take(sizeof(float) * tab);
  lay.off_tw = take(sizeof(float2) * tw);
  lay.off_part = take(sizeof(double) * 3 * rt);
  // done .. res back to back: reset_counters clears them with one fill
  lay.off_done = take(sizeof(int) * B);
  lay.off_nonf = take(sizeof(int) * B);
  lay.off_itd = take(sizeof(int) * B);
  lay.off_stopbuf = take(sizeof(int) * B);
  lay.off_res = take(sizeof(double) * 3 * B);
  lay.off_mean = take(sizeof(double) * 2 * kMeanBlocks * B);
  lay.off_goff = take(sizeof(long long) * B);
  lay.off_hoff = take(sizeof(long long) * B);
  lay.off_hsum = take(sizeof(float2) * B);
  lay.off_mu = take(sizeof(float) * B);
  lay.off_dscale = take(sizeof(float) * B);
  lay.off_small = take(sizeof(int) * B);
  lay.off_npass = take(sizeof(int) * B);
  lay.off_hsep = take(sizeof(float2) * tab);
  lay.off_sep = take(sizeof(int) * B);
  const int ck = p->opt.ckpt_every;
  if (ck > 0) {
    const int nck = (p->opt.max_iters + ck - 1) / ck + 1;
    lay.off_ck_yt = take(sizeof(float) * px * nck);
    lay.off_ck_v = take(sizeof(float2) * px * nck);
    lay.off_ck_d = take(sizeof(float2) * px * nck);
    lay.off_seg_u = take(sizeof(float2) * px * ck);
    lay.off_seg_spec = take(sizeof(float4) * sp * ck);
    lay.off_adj_a = take(sizeof(float2) * px);
    lay.off_adj_b = take(sizeof(float2) * px);
    lay.off_adj_z = take(sizeof(float) * px);
    lay.off_adj_y = take(sizeof(float) * px);
    lay.off_adj_S = take(sizeof(double2) * hhp);
    lay.off_tw64 = take(sizeof(double2) * tw);
    lay.off_adj_lam = take(sizeof(double) * rt);
    lay.off_adj_vb = take(sizeof(float2) * px);
    lay.off_adj_db = take(sizeof(float2) * px);
    lay.off_adj_mean = take(sizeof(double) * 64 * B);
    long long mk = 1;
    for (auto& d : p->desc) mk = std::max(mk, (long long)d.height * d.ksize);
    lay.off_adj_T = take(sizeof(double2) * mk * B);
  } else {
    lay.off_ck_yt = lay.off_ck_v = lay.off_ck_d = lay.off_seg_u = lay.off_seg_spec = 0;
    lay.off_adj_a = lay.off_adj_b = lay.off_adj_z = lay.off_adj_y = lay.off_adj_S = lay.off_adj_lam = 0;
    lay.off_adj_vb = lay.off_adj_db = lay.off_adj_mean = lay.off_tw64 = lay.off_adj_T = 0;
  }
  lay.total = o;
}

// per-image metadata and the tile tables of every launch shape
static void build_tiles(deconv_plan_s* p, bool half) {
  const int B = p->batch;
  p->meta.assign(B, ImgMeta{});
  p->hoff_h.assign(B, 0);
  long long px = 0, sp = 0, hhp = 0, tab = 0, rt = 0, hk = 0;
  std::map<int, long long> twoff;
  long long tw = 0;
  for (int b = 0; b < B; ++b) {
    const deconv_image_desc& d = p->desc[b];
    ImgMeta& m = p->meta[b];
    m.m = d.height; m.n = d.width; m.b = d.ksize / 2;
    m.mask_kind = d.mask_kind; m.decim = d.mask_kind == DECONV_MASK_DECIMATE ? d.decim : 1;
    m.dmagic = m.decim > 1 ? (unsigned)((1ull << 32) / (unsigned)m.decim) + 1u : 0u;
    m.nh = d.width / 2 + 1;
    m.C = c_for(d.height);
    m.logC = 0; while ((1 << m.logC) < m.C) ++m.logC;
    m.nb = (m.nh + m.C - 1) / m.C;
    m.rt = half ? rt_half(d.width) : rt_for(d.width);
    m.nrt = (d.height + m.rt - 1) / m.rt;
    m.rtmagic = m.rt > 1 ? (unsigned)((1ull << 32) / (unsigned)m.rt) + 1u : 0u;
    // the spectra the column pass leaves for the row pass come in row blocks
    // of rb rows (longer contiguous runs for its stores), rb a multiple of
    // the row tile height
    m.rb = rt_for(d.width) * DCV_ROW_BLOCK_MULT;
    m.rbmagic = m.rb > 1 ? (unsigned)((1ull << 32) / (unsigned)m.rb) + 1u : 0u;
    m.px = px; m.sp = sp; m.hh = hhp; m.tab = tab; m.rt0 = rt;
    m.nch = std::max(1, p->opt.channels);
    m.group = b - b % m.nch;
    for (int L : {d.width, d.height})
      if (!twoff.count(L)) { twoff[L] = tw; tw += L; }
    m.twr = twoff[d.width]; m.twc = twoff[d.height];
    p->hoff_h[b] = hk;
    px += (long long)d.height * d.width;
    // spectra: whole row blocks (the row-block layout pads the last one)
    sp += (long long)std::max((long long)m.nrt * m.rt, (long long)((d.height + m.rb - 1) / m.rb) * m.rb) *
          m.nb * m.C;
    hhp += (long long)d.height * m.nb * m.C;
    tab += d.height + m.nb * m.C;
    rt += m.nrt;
    hk += (long long)d.ksize * d.ksize;
  }
  // Half-height tiles fewer than three per compute unit (one 1024^2 image:
  // 512) run with 1024 threads: a shorter dependent chain per tile (row pass
  // 16.7 -> 15.7 us); batches lose 5-10% that way.
  p->wide_row = half && (p->opt.row_threads > 0 ? p->opt.row_threads == kNTRWide
                                               : p->tune_wrow >= 0 ? p->tune_wrow != 0 : rt < 3LL * num_cus());
  p->total_px = px; p->total_sp = sp; p->total_hh = hhp; p->total_tab = tab; p->total_tw = tw;
  p->total_rt = rt; p->total_h = hk; p->tw_off = twoff;

  // tile tables: one XCD-interleaved schedule per pass for the batched launch
  // and one per image for the per-image launches (batched = 0)
  p->h_tiles.clear();
  p->row_groups.clear(); p->col_groups.clear();
  for (int k = 0; k < 3; ++k) { p->row_sets[k].clear(); p->col_sets[k].clear(); }
  p->row_img.assign(B, {}); p->col_img.assign(B, {});
  std::vector<std::vector<TileRef>> rt_tiles(B), ct_tiles(B);
  std::set<int> widths, heights;
  for (int b = 0; b < B; ++b) {
    const ImgMeta& m = p->meta[b];
    widths.insert(m.n);
    heights.insert(m.m);
    const double lr = std::log2((double)m.n), lc = std::log2((double)m.m);
    for (int t = 0; t < m.nrt; ++t) {
      const int nr = std::min(m.rt, m.m - t * m.rt);
      rt_tiles[b].push_back(TileRef{b, t * m.rt, (double)(nr + 2) * m.n * lr});
    }
    for (int t = 0; t < m.nb; ++t) ct_tiles[b].push_back(TileRef{b, t, (double)m.C * m.m * lc});
  }
  // Fewer than three column tiles per compute unit: nothing to overlap a
  // tile's dependent chain with, so twice the threads per tile (one 1024^2
  // image: column pass 12.4 -> 11.4 us; with many tiles the narrow
  // workgroups overlap better: 16 x 1024^2, 77 -> 83 us if widened).
  long long ncol = 0;
  for (int b = 0; b < B; ++b) ncol += (long long)ct_tiles[b].size();
  p->wide_col = p->opt.col_threads > 0 ? p->opt.col_threads == kNTCWide
                                       : p->tune_wcol >= 0 ? p->tune_wcol != 0 : ncol < 3LL * num_cus();
  size_t rlds = 0, clds = 0;
  const int grt = half ? rt_half(*widths.begin()) : 0;
  for (int w : widths) rlds = std::max(rlds, row_lds_bytes(w, grt));
  for (int h : heights) clds = std::max(clds, col_lds_bytes(h));
  auto add_group = [&](std::vector<Group>& dst, int L, size_t lds, const std::vector<std::vector<TileRef>>& imgs,
                       int rt) {
    const long long t0 = (long long)p->h_tiles.size();
    xcd_schedule(imgs, p->h_tiles);
    dst.push_back(Group{L, t0, (int)((long long)p->h_tiles.size() - t0), lds, rt});
  };
  add_group(p->row_sets[1], widths.size() == 1 ? *widths.begin() : -*widths.rbegin(), rlds, rt_tiles, grt);
  add_group(p->col_sets[1], heights.size() == 1 ? *heights.begin() : -*heights.rbegin(), clds, ct_tiles, 0);
  if (widths.size() == 1) {
    p->row_sets[0] = p->row_sets[1];
  } else {
    for (int w : widths) {
      std::vector<std::vector<TileRef>> sel(B);
      for (int b = 0; b < B; ++b)
        if (p->meta[b].n == w) sel[b] = rt_tiles[b];
      add_group(p->row_sets[0], w, row_lds_bytes(w), sel, 0);
    }
  }
  if (heights.size() == 1) {
    p->col_sets[0] = p->col_sets[1];
  } else {
    for (int h : heights) {
      std::vector<std::vector<TileRef>> sel(B);
      for (int b = 0; b < B; ++b)
        if (p->meta[b].m == h) sel[b] = ct_tiles[b];
      add_group(p->col_sets[0], h, col_lds_bytes(h), sel, 0);
    }
  }
  // hybrid: the lengths whose tiles cannot fill the chip twice over (or that
  // are short) share one launch, the others keep a launch each
  auto hybrid = [&](bool rows) {
    std::vector<Group>& dst = rows ? p->row_sets[2] : p->col_sets[2];
    const std::set<int>& lens = rows ? widths : heights;
    const auto& tiles = rows ? rt_tiles : ct_tiles;
    std::map<int, long long> count;
    for (int b = 0; b < B; ++b) count[rows ? p->meta[b].n : p->meta[b].m] += (long long)tiles[b].size();
    std::set<int> small;
    for (int L : lens)
      if (L <= 256 || count[L] < 2LL * num_cus()) small.insert(L);
    if (small.size() < 2 || small.size() == lens.size()) {
      dst = small.size() == lens.size() ? (rows ? p->row_sets[1] : p->col_sets[1])
                                        : (rows ? p->row_sets[0] : p->col_sets[0]);
      return;
    }
    std::vector<std::vector<TileRef>> sel(B);
    size_t lds = 0;
    for (int b = 0; b < B; ++b) {
      const int L = rows ? p->meta[b].n : p->meta[b].m;
      if (small.count(L)) sel[b] = tiles[b];
    }
    for (int L : small) lds = std::max(lds, rows ? row_lds_bytes(L) : col_lds_bytes(L));
    add_group(dst, -*small.rbegin(), lds, sel, 0);
    for (int L : lens) {
      if (small.count(L)) continue;
      std::vector<std::vector<TileRef>> one(B);
      for (int b = 0; b < B; ++b)
        if ((rows ? p->meta[b].n : p->meta[b].m) == L) one[b] = tiles[b];
      add_group(dst, L, rows ? row_lds_bytes(L) : col_lds_bytes(L), one, 0);
    }
  };
  hybrid(true);
  hybrid(false);
  // schedule 1, 2, 3 -> set 0, 1, 2; autotuning (0) starts from one launch
  const int rs = p->opt.schedule >= 1 ? p->opt.schedule - 1 : 1, cs = rs;
  p->row_sched = rs;
  p->col_sched = cs;
  p->row_groups = p->row_sets[rs];
  p->col_groups = p->col_sets[cs];
  for (int b = 0; b < B; ++b) {
    std::vector<std::vector<TileRef>> one(B);
    one[b] = rt_tiles[b];
    add_group(p->row_img[b], p->meta[b].n, row_lds_bytes(p->meta[b].n, grt), one, grt);
    one[b].clear();
    one[b] = ct_tiles[b];
    add_group(p->col_img[b], p->meta[b].m, col_lds_bytes(p->meta[b].m), one, 0);
  }
}

template <typename T>
static T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

extern "C" deconv_status deconv_options_default(deconv_options* opt) {
  if (!opt) return DECONV_ERR_INVALID_ARG;
  opt->alpha = 2.0f;
  opt->check_every = 0;
  opt->tol_primal = 0.0;
  opt->tol_dual = 0.0;
  opt->use_graph = 1;
  opt->batched = 1;
  opt->ckpt_every = 0;
  opt->max_iters = 0;
  opt->profile = 0;
  opt->schedule = 0;
  opt->tune_cache = nullptr;
  opt->bgs_passes = 1;
  opt->adapt_t = 0.0;
  opt->warm_iters = 0;
  opt->warm_tau = 1e-3f;
  opt->channels = 1;
  opt->spectra_hint = 0;
  opt->row_tiles = 0;
  opt->row_threads = 0;
  opt->col_threads = 0;
  opt->small_images = 2;
  opt->separable_blur = 1;
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_workspace_size(int32_t batch, const deconv_image_desc* desc,
                                                    const deconv_options* opt, size_t* bytes) {
  if (!bytes) return DECONV_ERR_INVALID_ARG;
  STCHK(validate(batch, desc, opt));
  deconv_plan_s tmp;
  tmp.batch = batch;
  tmp.desc.assign(desc, desc + batch);
  if (opt) tmp.opt = *opt; else deconv_options_default(&tmp.opt);
  Layout lay;
  build_layout(&tmp, lay);
  *bytes = lay.total;
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_destroy(deconv_plan p) {
  if (!p) return DECONV_ERR_INVALID_ARG;
  if (p->hsum_pending) (void)hipEventSynchronize(p->hsum_ev);   // a copy into hsum_host in flight
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (auto st : p->side) (void)hipStreamDestroy(st);
  for (auto e : p->join_ev) (void)hipEventDestroy(e);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  for (auto& e : p->ev_row) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& e : p->ev_col) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& e : p->ev_brow) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& e : p->ev_bcol) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& kv : p->bwd_graphs) (void)hipGraphExecDestroy(kv.second.first);
  for (auto& e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->own_ws && p->ws) (void)hipFree(p->ws);
  if (p->hsum_host) (void)hipHostFree(p->hsum_host);
  if (p->hsum_ev) (void)hipEventDestroy(p->hsum_ev);
  delete p;
  return DECONV_OK;
}

static deconv_status autotune(deconv_plan_s* p);

extern "C" deconv_status deconv_plan_create(deconv_plan* out, int32_t batch, const deconv_image_desc* desc,
                                            const deconv_options* opt, void* stream, void* workspace,
                                            size_t workspace_bytes) {
  if (!out) return DECONV_ERR_INVALID_ARG;
  *out = nullptr;
  STCHK(validate(batch, desc, opt));
  deconv_plan_s* p = new (std::nothrow) deconv_plan_s;
  if (!p) return DECONV_ERR_OOM;
  p->batch = batch;
  p->desc.assign(desc, desc + batch);
  for (auto& d : p->desc) p->max_height = std::max(p->max_height, (int)d.height);
  if (opt) p->opt = *opt; else deconv_options_default(&p->opt);
  p->stream = static_cast<hipStream_t>(stream);
  p->ls = p->stream;
  if (p->opt.use_graph && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete p;
    return DECONV_ERR_HIP;
  }
  Layout lay;
  build_layout(p, lay);
  if (workspace) {
    if (workspace_bytes < lay.total) { delete p; return DECONV_ERR_OOM; }
    p->ws = workspace;
  } else {
    if (hipMalloc(&p->ws, lay.total) != hipSuccess) { delete p; return DECONV_ERR_OOM; }
    p->own_ws = true;
    if (hipHostMalloc(reinterpret_cast<void**>(&p->hsum_host), sizeof(float2) * batch, hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&p->hsum_ev, hipEventDisableTiming) != hipSuccess) {
      deconv_plan_destroy(p);
      return DECONV_ERR_HIP;
    }
  }
  p->ws_bytes = lay.total;
  void* w = p->ws;
  p->d_meta = at<ImgMeta>(w, lay.off_meta);
  p->d_tiles = at<int4>(w, lay.off_tiles);
  p->yt = at<float>(w, lay.off_yt);
  p->dbuf[0] = at<float2>(w, lay.off_d0);
  p->dbuf[1] = at<float2>(w, lay.off_d1);
  p->v = at<float2>(w, lay.off_v);
  p->specA = at<float4>(w, lay.off_specA);
  p->specB = at<float4>(w, lay.off_specB);
  p->hh = at<float2>(w, lay.off_hh);
  p->tab = at<float>(w, lay.off_tab);
  p->tw = at<float2>(w, lay.off_tw);
  p->partials = at<double>(w, lay.off_part);
  p->done = at<int>(w, lay.off_done);
  p->nonfinite = at<int>(w, lay.off_nonf);
  p->iters_done = at<int>(w, lay.off_itd);
  p->stop_buf = at<int>(w, lay.off_stopbuf);
  p->res = at<double>(w, lay.off_res);
  p->mean = at<double>(w, lay.off_mean);
  p->goff = at<long long>(w, lay.off_goff);
  p->hoff = at<long long>(w, lay.off_hoff);
  p->hsum = at<float2>(w, lay.off_hsum);
  p->mu_cur = at<float>(w, lay.off_mu);
  p->dscale = at<float>(w, lay.off_dscale);
  p->d_small = at<int>(w, lay.off_small);
  p->npass = at<int>(w, lay.off_npass);
  p->hsep = at<float2>(w, lay.off_hsep);
  p->sep = at<int>(w, lay.off_sep);
  if (p->opt.ckpt_every > 0) {
    p->ck_yt = at<float>(w, lay.off_ck_yt);
    p->ck_v = at<float2>(w, lay.off_ck_v);
    p->ck_d = at<float2>(w, lay.off_ck_d);
    p->seg_u = at<float2>(w, lay.off_seg_u);
    p->seg_spec = at<float4>(w, lay.off_seg_spec);
    p->adj_a = at<float2>(w, lay.off_adj_a);
    p->adj_b = at<float2>(w, lay.off_adj_b);
    p->adj_z = at<float>(w, lay.off_adj_z);
    p->adj_y = at<float>(w, lay.off_adj_y);
    p->adj_S = at<double2>(w, lay.off_adj_S);
    p->adj_T = at<double2>(w, lay.off_adj_T);
    p->tw64 = at<double2>(w, lay.off_tw64);
    p->adj_lam = at<double>(w, lay.off_adj_lam);
    p->adj_vb = at<float2>(w, lay.off_adj_vb);
    p->adj_db = at<float2>(w, lay.off_adj_db);
    p->adj_mean = at<double>(w, lay.off_adj_mean);
  }

  // host-built tables
  const std::vector<int4>& tiles = p->h_tiles;
  std::vector<float2> tw(p->total_tw);
  std::vector<double2> tw64(p->total_tw);
  for (auto& kv : p->tw_off) {
    std::vector<float2> t;
    twiddles(kv.first, t);
    std::copy(t.begin(), t.end(), tw.begin() + kv.second);
    for (int k = 0; k < kv.first; ++k) {
      const double a = -2.0 * M_PI * (double)k / (double)kv.first;
      tw64[kv.second + k] = make_double2(cos(a), sin(a));
    }
  }
  if (p->tw64 && hipMemcpyAsync(p->tw64, tw64.data(), sizeof(double2) * tw64.size(), hipMemcpyHostToDevice,
                                 p->stream) != hipSuccess) {
    deconv_plan_destroy(p);
    return DECONV_ERR_HIP;
  }
  std::vector<float> tab(p->total_tab);
  std::vector<long long> goff(batch), hoff(batch);
  // BGS passes per image: the option's count, or with 0 b passes for a
  // (2b+1)^2 blur (Sec. III-B), at least one
  std::vector<int> npass(batch);
  p->max_pass = 1;
  for (int b = 0; b < batch; ++b) {
    npass[b] = p->opt.bgs_passes > 0 ? p->opt.bgs_passes : std::max(1, p->desc[b].ksize / 2);
    p->max_pass = std::max(p->max_pass, npass[b]);
  }
  for (int b = 0; b < batch; ++b) {
    const ImgMeta& m = p->meta[b];
    for (int k = 0; k < m.m; ++k) {
      double s = sin(M_PI * (double)k / (double)m.m);
      tab[m.tab + k] = (float)(4.0 * s * s);
    }
    for (int k = 0; k < m.nb * m.C; ++k) {
      double s = sin(M_PI * (double)k / (double)m.n);
      tab[m.tab + m.m + k] = (float)(4.0 * s * s);
    }
    goff[b] = 2 * m.sp;  // the setup grid (float2 units) lives in specB
    hoff[b] = p->hoff_h[b];
  }
  hipStream_t s = p->stream;
  auto fail = [&](deconv_status st) { deconv_plan_destroy(p); return st; };
  if (hipMemcpyAsync(p->d_meta, p->meta.data(), sizeof(ImgMeta) * batch, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->tab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->goff, goff.data(), sizeof(long long) * batch, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->hoff, hoff.data(), sizeof(long long) * batch, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->npass, npass.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s) != hipSuccess ||
      // padded spectrum entries are never written by the passes: clear once
      hipMemsetAsync(p->specA, 0, sizeof(float4) * p->total_sp, s) != hipSuccess ||
      hipMemsetAsync(p->specB, 0, sizeof(float4) * p->total_sp, s) != hipSuccess ||
      hipMemsetAsync(p->done, 0, sizeof(int) * batch, s) != hipSuccess ||
      // no blur yet: the autotuner's passes read the stored spectrum
      hipMemsetAsync(p->sep, 0, sizeof(int) * batch, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(DECONV_ERR_HIP);
  // the whole-image-in-LDS path takes the plan when every image has one and
  // the options need nothing it lacks (one pass, fixed penalty, grey images,
  // no checkpoints): always with opt.small_images = 1, and with 2 (the
  // default) when no side exceeds kSmallAutoSide (measured on MI355X against
  // the two-pass kernels: one image of side 32 / 48 / 64 / 72 2.7 / 1.9 /
  // 1.3 / 1.1x as fast, 64 images of 72^2 1.5x, 256 of 64^2 2.6x; one 96^2
  // image 0.6x)
  p->small = p->opt.small_images != 0 && p->opt.bgs_passes == 1 && !(p->opt.adapt_t > 0) &&
             p->opt.channels == 1 && p->opt.ckpt_every == 0;
  for (auto& d : p->desc)
    p->small = p->small && has_small_path(d.height, d.width) &&
               (p->opt.small_images == 1 || std::max(d.height, d.width) <= kSmallAutoSide);
  if (p->small) {
    std::vector<int> order(batch);
    for (int b = 0; b < batch; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int u, int v) { return p->desc[u].height < p->desc[v].height; });
    // one launch: of the image's side when all share it, else one that
    // dispatches on each image's side
    bool one_side = true;
    for (auto& d : p->desc) one_side = one_side && d.height == p->desc[0].height;
    p->small_groups.push_back({one_side ? p->desc[0].height : 0, 0, batch});
    if (hipMemcpy(p->d_small, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice) != hipSuccess)
      return fail(DECONV_ERR_HIP);
  }
  deconv_status st = p->small ? DECONV_OK : autotune(p);
  if (st != DECONV_OK) return fail(st);
  if (p->opt.use_graph && p->opt.batched) {
    // one side stream per extra launch of the longer pass (at most 7)
    const size_t n = std::min<size_t>(7, std::max(p->row_groups.size(), p->col_groups.size()) - 1);
    for (size_t k = 0; k < n; ++k) {
      hipStream_t ss = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&ss, hipStreamNonBlocking) != hipSuccess) return fail(DECONV_ERR_HIP);
      p->side.push_back(ss);
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail(DECONV_ERR_HIP);
      p->join_ev.push_back(ev);
    }
    if (n > 0 && hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess)
      return fail(DECONV_ERR_HIP);
  }
  *out = p;
  return DECONV_OK;
}

// ---------------------------------------------------------------------------
// run
// ---------------------------------------------------------------------------
// ids of the states plans hold: unique in the process, never 0
static std::atomic<uint64_t> g_run_id{0};
static uint64_t new_run_id() { return ++g_run_id; }

// H^ of every image, by direct sums over the taps (one launch for the batch)
// or, for kernels wider than kBlurMaxK, by 2-D FFTs of the embedded kernels
// in the grid in specB (free between calls: the column pass output is
// rebuilt by every prologue): full_out = the whole spectra (for
// deconv_blur_spectrum); pack = the half spectrum the passes read and the
// separable factors (deconv_blur_spectrum leaves them alone)
static bool singular_dc(float2 v) { return !(std::isfinite(v.x) && std::isfinite(v.y)) || (v.x == 0.f && v.y == 0.f); }

// With defer (and pinned memory), the DC terms are copied back without
// waiting: check_spectrum tests them once the caller has queued the rest of
// the run, so that the queue never drains between runs.
static deconv_status setup_spectrum(deconv_plan_s* p, const float* h, float* full_out, bool pack = true,
                                    bool defer = false) {
  hipStream_t s = p->stream;
  p->hsum_pending = false;
  const int B = p->batch;
  int maxk = 0, maxcol = 0, maxout = 0, maxm = 0;
  for (const ImgMeta& m : p->meta) {
    maxk = std::max(maxk, 2 * m.b + 1);
    maxcol = std::max(maxcol, m.nb * m.C);
    maxout = std::max(maxout, m.m + m.nb * m.C);
    maxm = std::max(maxm, m.m);
  }
  const int rowblk = (maxm + kBlurRows - 1) / kBlurRows;
  // the separable factors (and flags) of every image: the column pass reads
  // them, and the half spectrum of a separable blur is their product
  auto separable = [&]() -> deconv_status {
    hipLaunchKernelGGL(separable_psf_kernel, dim3((maxout + kNT - 1) / kNT, B), dim3(kNT), 0, s, p->d_meta, h,
                       p->hoff, p->tw, p->hsep, p->sep, p->opt.separable_blur);
    HIPCHK(hipGetLastError());
    return DECONV_OK;
  };
  if (maxk <= kBlurMaxK) {
    if (full_out) {
      int maxn = 0;
      for (const ImgMeta& m : p->meta) maxn = std::max(maxn, m.n);
      hipLaunchKernelGGL(blur_half_kernel, dim3((maxn + kBlurCols - 1) / kBlurCols, rowblk, B), dim3(kNT), 0, s,
                         p->d_meta, h, p->hoff, p->tw, p->hh, p->hsum, reinterpret_cast<float2*>(full_out),
                         nullptr, nullptr);
      HIPCHK(hipGetLastError());
    }
    if (pack) {
      STCHK(separable());
      hipLaunchKernelGGL(blur_half_kernel, dim3((maxcol + kBlurCols - 1) / kBlurCols, rowblk, B), dim3(kNT), 0, s,
                         p->d_meta, h, p->hoff, p->tw, p->hh, p->hsum, nullptr, p->hsep, p->sep);
      HIPCHK(hipGetLastError());
    }
  } else {
    // whole spectra by 2-D FFTs of the embedded kernels
    float2* grid = reinterpret_cast<float2*>(p->specB);
    int gx = 64;
    HIPCHK(hipMemsetAsync(grid, 0, sizeof(float4) * (size_t)p->total_sp, s));
    hipLaunchKernelGGL(embed_psf_kernel, dim3(B), dim3(kNT), 0, s, p->d_meta, h, p->hoff, grid, p->goff);
    HIPCHK(hipGetLastError());
    for (int b = 0; b < B; ++b) {
      const ImgMeta& m = p->meta[b];
      float2* g = grid + 2 * m.sp;
      HIPCHK(launch_fft_rows(m.n, g, m.m, p->tw + m.twr, 0, s));
      HIPCHK(launch_fft_cols(m.m, g, m.n, 1, p->tw + m.twc, 0, s));
      if (full_out)
        HIPCHK(hipMemcpyAsync(reinterpret_cast<float2*>(full_out) + m.px, g, sizeof(float2) * m.m * m.n,
                              hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(p->hsum + b, g, sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    if (pack) {
      hipLaunchKernelGGL(pack_half_kernel, dim3(gx, B), dim3(kNT), 0, s, p->d_meta, grid, p->goff, p->hh);
      HIPCHK(hipGetLastError());
      STCHK(separable());
    }
  }
  if (defer && p->hsum_host) {
    HIPCHK(hipMemcpyAsync(p->hsum_host, p->hsum, sizeof(float2) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(p->hsum_ev, s));
    p->hsum_pending = true;
    return DECONV_OK;
  }
  std::vector<float2> hs(B);
  HIPCHK(hipMemcpyAsync(hs.data(), p->hsum, sizeof(float2) * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b)
    if (singular_dc(hs[b])) return DECONV_ERR_SINGULAR;
  return DECONV_OK;
}

// the deferred DC-term test; a singular blur fails the call after the work
// queued on it has finished (its outputs are then undefined)
static deconv_status check_spectrum(deconv_plan_s* p) {
  if (!p->hsum_pending) return DECONV_OK;
  p->hsum_pending = false;
  HIPCHK(hipEventSynchronize(p->hsum_ev));
  for (int b = 0; b < p->batch; ++b)
    if (singular_dc(p->hsum_host[b])) {
      HIPCHK(hipStreamSynchronize(p->stream));
      return DECONV_ERR_SINGULAR;
    }
  return DECONV_OK;
}

// Non-temporal stores of the pass-to-pass spectra pay while the plan's
// working set stays in the last-level cache and cost once it spills to HBM
// (measured, both spectrum buffers together: one 1024^2 image, 17 MB: +2%;
// 2 x 1024^2 or 8 x 512^2, 34 MB: +5 to +8%; 4 x 1024^2, 67 MB: -6%;
// one 2048^2 image, 67 MB: -31%).
static int nt_spectra(const deconv_plan_s* p) {
  if (p->opt.spectra_hint != 0) return p->opt.spectra_hint == 2;
  return 2.0 * (double)p->total_sp * sizeof(float4) <= 40.0 * (1 << 20);
}

static RowArgs row_args(deconv_plan_s* p, const uint8_t* mask, const float* lam, const float* mu) {
  RowArgs a{};
  a.meta = p->d_meta;
  a.tiles = p->d_tiles;
  a.spec_in = p->specB;
  a.spec_out = p->specA;
  a.yt = p->yt;
  a.v = p->v;
  a.mask = mask;
  a.lam = lam;
  a.mu = mu;
  a.tw = p->tw;
  a.partials = p->partials;
  a.done = p->done;
  a.alpha = p->opt.alpha;
  a.nt_spec = nt_spectra(p);
  return a;
}

static ColArgs col_args(deconv_plan_s* p, const float* mu) {
  ColArgs a{};
  a.meta = p->d_meta;
  a.tiles = p->d_tiles;
  a.spec_in = p->specA;
  a.spec_out = p->specB;
  a.hh = p->hh;
  a.tab = p->tab;
  a.hsep = p->hsep;
  a.sep = p->sep;
  a.mu = mu;
  a.tw = p->tw;
  a.done = p->done;
  a.nt_spec = nt_spectra(p);
  return a;
}

static hipEvent_t take_event(deconv_plan_s* p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// With opt.profile (and outside a graph capture) a pass gets a start event on
// its first launch and a stop event on its last one.
struct PassTimer {
  deconv_plan_s* p;
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* dst;
  hipEvent_t a = nullptr, b = nullptr;
  PassTimer(deconv_plan_s* p_, std::vector<std::pair<hipEvent_t, hipEvent_t>>* d) : p(p_), dst(d) {
    if (p->opt.profile && p->ls == p->stream) {
      a = take_event(p);
      b = take_event(p);
      if (!a || !b) a = b = nullptr;
    }
  }
  hipEvent_t start(size_t idx) const { return idx == 0 ? a : nullptr; }
  hipEvent_t stop(size_t idx, size_t n) const { return idx + 1 == n ? b : nullptr; }
  void done() { if (a) dst->emplace_back(a, b); }
};

// the groups one pass launches: one per line length (batched) or per image
static const std::vector<Group> pass_groups(deconv_plan_s* p, bool rows) {
  if (p->opt.batched) return rows ? p->row_groups : p->col_groups;
  std::vector<Group> g;
  for (int b = 0; b < p->batch; ++b)
    for (auto& x : (rows ? p->row_img[b] : p->col_img[b])) g.push_back(x);
  return g;
}

// Streams of the launches of one pass.  While a graph is being captured and
// the pass has several launches (images of different lengths: independent
// work), launch k > 0 goes to a side stream that waits for the fork point,
// and the capture stream joins them all afterwards: the graph then holds the
// launches as parallel branches.  Otherwise everything goes to p->ls.
struct PassStreams {
  deconv_plan_s* p;
  size_t n;
  bool fork;
  PassStreams(deconv_plan_s* p_, size_t n_) : p(p_), n(n_) {
    fork = n > 1 && !p->side.empty() && p->ls == p->cap_stream && p->cap_stream != nullptr;
  }
  hipError_t begin() { return fork ? hipEventRecord(p->fork_ev, p->ls) : hipSuccess; }
  hipStream_t stream(size_t k) const { return (fork && k > 0) ? p->side[(k - 1) % p->side.size()] : p->ls; }
  hipError_t before(size_t k) {
    if (!fork || k == 0 || k > p->side.size()) return hipSuccess;
    return hipStreamWaitEvent(stream(k), p->fork_ev, 0);
  }
  hipError_t end() {
    if (!fork) return hipSuccess;
    const size_t m = std::min(n - 1, p->side.size());
    for (size_t q = 0; q < m; ++q) {
      hipError_t e = hipEventRecord(p->join_ev[q], p->side[q]);
      if (e == hipSuccess) e = hipStreamWaitEvent(p->ls, p->join_ev[q], 0);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// launch the row pass over every image (batched) or image by image
static deconv_status launch_rows(deconv_plan_s* p, RowArgs a) {
  PassTimer timer(p, &p->ev_row);
  const std::vector<Group>& gs = p->opt.batched ? p->row_groups : pass_groups(p, true);
  PassStreams ps(p, gs.size());
  HIPCHK(ps.begin());
  for (size_t k = 0; k < gs.size(); ++k) {
    a.tiles = p->d_tiles + gs[k].tile0;
    HIPCHK(ps.before(k));
    HIPCHK(launch_row(gs[k].L, gs[k].rt, gs[k].ntiles, gs[k].lds, ps.stream(k), a, timer.start(k),
                      timer.stop(k, gs.size()), p->wide_row));
  }
  HIPCHK(ps.end());
  timer.done();
  return DECONV_OK;
}

static deconv_status launch_cols(deconv_plan_s* p, ColArgs a) {
  PassTimer timer(p, &p->ev_col);
  const std::vector<Group>& gs = p->opt.batched ? p->col_groups : pass_groups(p, false);
  PassStreams ps(p, gs.size());
  HIPCHK(ps.begin());
  for (size_t k = 0; k < gs.size(); ++k) {
    a.tiles = p->d_tiles + gs[k].tile0;
    HIPCHK(ps.before(k));
    HIPCHK(launch_col(gs[k].L, gs[k].ntiles, gs[k].lds, ps.stream(k), a, timer.start(k), timer.stop(k, gs.size()),
                      p->wide_col && has_wide_col(gs[k].L)));
  }
  HIPCHK(ps.end());
  timer.done();
  return DECONV_OK;
}

// ---------------------------------------------------------------------------
// autotuner: per pass, one launch per line length or one launch for all
// lengths, whichever runs faster on this plan's own workspace
// ---------------------------------------------------------------------------
static std::string plan_signature(const deconv_plan_s* p) {
  std::vector<std::array<int, 5>> v;
  for (auto& d : p->desc) v.push_back({d.height, d.width, d.ksize, d.mask_kind, 0});
  std::sort(v.begin(), v.end());
  std::ostringstream os;
  os << "gfx950 nt" << kNTR << "/" << kNTC << " rows" << DCV_ROW_PIX << " cols" << DCV_COL_ELEMS << " |";
  for (size_t i = 0; i < v.size();) {
    size_t j = i;
    while (j < v.size() && v[j] == v[i]) ++j;
    os << " " << v[i][0] << "x" << v[i][1] << "k" << v[i][2] << "m" << v[i][3] << "*" << (j - i);
    i = j;
  }
  return os.str();
}

// One line per tuned batch signature: "signature<TAB>rs cs half wrow wcol"
// (launch shape of each pass, 0-2; row tile height class, wide row tiles and
// wide column tiles, each 0/1, or -1 for the plan's heuristic).  The last
// matching line wins; lines of the older two-field form are read too.
struct TuneChoice {
  int rs = 1, cs = 1, half = -1, wrow = -1, wcol = -1;
};

static bool cache_lookup(const char* path, const std::string& key, TuneChoice* out) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const size_t t1 = line.find('\t');
    if (t1 == std::string::npos || line.compare(0, t1, key) != 0 || t1 != key.size()) continue;
    TuneChoice c;
    const int n = sscanf(line.c_str() + t1 + 1, "%d %d %d %d %d", &c.rs, &c.cs, &c.half, &c.wrow, &c.wcol);
    if (n >= 2 && c.rs >= 0 && c.rs <= 2 && c.cs >= 0 && c.cs <= 2) {
      if (n < 5) c.half = c.wrow = c.wcol = -1;
      *out = c;
      found = true;
    }
  }
  return found;
}

static void cache_store(const char* path, const std::string& key, const TuneChoice& c) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << "\t" << c.rs << " " << c.cs << " " << c.half << " " << c.wrow << " " << c.wcol << "\n";
}

// rebuild the tile tables for the plan's knob choices and upload them
static deconv_status apply_tuning(deconv_plan_s* p, const TuneChoice& c) {
  p->tune_half = c.half;
  p->tune_wrow = c.wrow;
  p->tune_wcol = c.wcol;
  build_tiles(p, use_half_rt(p));
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipMemcpy(p->d_meta, p->meta.data(), sizeof(ImgMeta) * p->batch, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->d_tiles, p->h_tiles.data(), sizeof(int4) * p->h_tiles.size(), hipMemcpyHostToDevice));
  p->row_sched = c.rs;
  p->col_sched = c.cs;
  p->row_groups = p->row_sets[c.rs];
  p->col_groups = p->col_sets[c.cs];
  return DECONV_OK;
}

// The autotuner (schedule 0, batched plans): the launch shape of each pass
// (one launch per line length, one for all, hybrid) and the tile knobs the
// options leave open -- row tiles of the default or half height, 512 or 1024
// threads per half-height row tile, 256 or 512 threads per long column tile.
// Candidates are timed on whole iterations (column pass then row pass, plain
// iterations on zero data, on the plan's own workspace); the plan's size
// heuristics give the starting choice, and another wins only when it is at
// least 3% faster.  Decisions go to the tune cache when one is given.
static deconv_status autotune(deconv_plan_s* p) {
  if (p->opt.schedule != 0 || !p->opt.batched) return DECONV_OK;
  const bool multi_r = p->row_sets[0].size() > 1, multi_c = p->col_sets[0].size() > 1;
  // the heuristics' choice
  TuneChoice heur;
  const bool h_half = use_half_rt(p);
  heur.half = h_half ? 1 : 0;
  heur.wrow = p->wide_row ? 1 : 0;
  heur.wcol = p->wide_col ? 1 : 0;
  std::vector<std::pair<int, int>> rowc = {{heur.half, heur.wrow}};   // (half, wide rows)
  if (half_rt_allowed(p) && p->opt.row_tiles != 1) {
    std::vector<int> wr;
    if (p->opt.row_threads == 0) wr = {0, 1};
    else wr = {p->opt.row_threads == kNTRWide ? 1 : 0};
    if (p->opt.row_tiles == 0) rowc.push_back({0, 0});
    for (int w : wr) rowc.push_back({1, w});
  }
  std::vector<int> colc = {heur.wcol};
  bool long_cols = false;
  for (auto& d : p->desc) long_cols |= has_wide_col(d.height);
  if (long_cols && p->opt.col_threads == 0) colc = {heur.wcol, 1 - heur.wcol};
  if (!multi_r && !multi_c && rowc.size() < 2 && colc.size() < 2) return DECONV_OK;
  const std::string key = plan_signature(p);
  TuneChoice best = heur;
  if (cache_lookup(p->opt.tune_cache, key, &best)) return apply_tuning(p, best);
  hipStream_t s = p->stream;
  const size_t n = (size_t)p->total_px;
  HIPCHK(hipMemsetAsync(p->yt, 0, sizeof(float) * n, s));
  HIPCHK(hipMemsetAsync(p->v, 0, sizeof(float2) * n, s));
  HIPCHK(hipMemsetAsync(p->dbuf[0], 0, sizeof(float2) * n, s));
  HIPCHK(hipMemsetAsync(p->dbuf[1], 0, sizeof(float2) * n, s));
  // lambda = 0, mu = 1 and an all-unobserved mask: any finite data will do
  float* par = nullptr;
  uint8_t* msk = nullptr;
  HIPCHK(hipMalloc(&par, sizeof(float) * 2 * p->batch));
  if (hipMalloc(&msk, n) != hipSuccess) { (void)hipFree(par); return DECONV_ERR_OOM; }
  std::vector<float> hp(2 * p->batch, 0.f);
  for (int b = 0; b < p->batch; ++b) hp[p->batch + b] = 1.f;
  deconv_status st = DECONV_OK;
  if (hipMemcpy(par, hp.data(), sizeof(float) * hp.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(msk, 0, n, s) != hipSuccess) st = DECONV_ERR_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == DECONV_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = DECONV_ERR_HIP;
  // milliseconds of kReps iterations (after two untimed ones), best of two
  const int kReps = 10;
  auto time_iters = [&](double* ms_out) -> deconv_status {
    double best_ms = 1e300;
    for (int trial = 0; trial < 2; ++trial) {
      for (int r = 0; r < kReps + 2; ++r) {
        if (r == 2 && hipEventRecord(e0, s) != hipSuccess) return DECONV_ERR_HIP;
        ColArgs ca = col_args(p, par + p->batch);
        ca.done = nullptr;
        STCHK(launch_cols(p, ca));
        RowArgs ra = row_args(p, msk, par, par + p->batch);
        ra.mode = ROW_ITER;
        ra.d_in = p->dbuf[r & 1];
        ra.d_out = p->dbuf[1 - (r & 1)];
        ra.done = nullptr;
        STCHK(launch_rows(p, ra));
      }
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return DECONV_ERR_HIP;
      best_ms = std::min(best_ms, (double)ms);
    }
    *ms_out = best_ms;
    return DECONV_OK;
  };
  // the candidates one at a time, the other pass at its current best;
  // the first candidate timed is the heuristics' own
  double best_ms = 1e300;
  auto consider = [&](const TuneChoice& c) {
    if (st != DECONV_OK) return;
    st = apply_tuning(p, c);
    double ms = 0;
    if (st == DECONV_OK) st = time_iters(&ms);
    if (st == DECONV_OK && (best_ms == 1e300 || ms < 0.97 * best_ms)) {
      best_ms = ms;
      best = c;
    }
  };
  consider(heur);
  for (auto& rc : rowc)
    for (int k = multi_r ? 0 : 1; k <= (multi_r ? 2 : 1); ++k) {
      TuneChoice c = best;
      c.half = rc.first;
      c.wrow = rc.second;
      c.rs = k;
      consider(c);
    }
  for (int wc : colc)
    for (int k = multi_c ? 0 : 1; k <= (multi_c ? 2 : 1); ++k) {
      TuneChoice c = best;
      c.wcol = wc;
      c.cs = k;
      consider(c);
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(msk);
  (void)hipFree(par);
  if (st != DECONV_OK) return st;
  cache_store(p->opt.tune_cache, key, best);
  return apply_tuning(p, best);
}

extern "C" deconv_status deconv_plan_run_id(deconv_plan p, uint64_t* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  *out = p->have_state ? p->run_id : 0;
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_tiles(deconv_plan p, int32_t* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  out[0] = (!p->meta.empty() && p->meta[0].rt != rt_for(p->meta[0].n)) ? 2 : 1;
  out[1] = p->wide_row ? kNTRWide : kNTR;
  out[2] = p->wide_col ? kNTCWide : kNTC;
  out[3] = p->small ? 1 : 0;
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_separable(deconv_plan p, int32_t* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  HIPCHK(hipMemcpyAsync(out, p->sep, sizeof(int32_t) * p->batch, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_schedule(deconv_plan p, int32_t* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  out[0] = p->row_sched + 1;
  out[1] = p->col_sched + 1;
  return DECONV_OK;
}

// first spectra from the stored state (ytilde, v, d = dbuf[cur_d])
static deconv_status prologue_from_state(deconv_plan_s* p, const float* mu) {
  RowArgs a = row_args(p, nullptr, mu, mu);
  a.mode = ROW_STATE;
  a.d_in = p->dbuf[p->cur_d];
  a.d_out = p->dbuf[1 - p->cur_d];
  a.done = nullptr;
  STCHK(launch_rows(p, a));
  p->cur_d = 1 - p->cur_d;
  return DECONV_OK;
}

struct IterFlags {
  int check, store_v, store_x, last;
};

static IterFlags flags_for(const deconv_plan_s* p, int it, int iters) {
  const int K = p->opt.check_every;
  IterFlags f{};
  f.last = it == iters - 1;
  f.check = K > 0 && ((it + 1) % K == 0);
  // v is kept for the next check (it reads v^i); with tolerances, an image
  // may stop at any check, so every check also stores v and x to leave the
  // state of that iteration.  Without them only the last iteration stores x.
  const bool may_stop = f.check && (p->opt.tol_primal > 0 || p->opt.tol_dual > 0);
  f.store_v = f.last || may_stop || (K > 0 && (K == 1 || ((it + 2) % K == 0)));
  f.store_x = f.last || may_stop;
  return f;
}

// penalty the kernels read: the caller's, or the plan's adaptive copy
static const float* mu_in_use(const deconv_plan_s* p, const float* mu) {
  return p->opt.adapt_t > 0 ? p->mu_cur : mu;
}

// swaps of the double-buffered d per iteration (one more for the rescaling
// pass of the adaptive penalty)
static int d_swaps_per_iter(const deconv_plan_s* p) {
  return p->opt.adapt_t > 0 || p->opt.channels > 1 ? 2 : 1;
}

// One iteration: bgs_passes - 1 inner passes (column pass, then the row pass
// that redoes the z-step and transforms ytilde again), the last column pass
// and the row pass that finishes the iteration (+ residual reduction).  With
// the adaptive penalty the row pass stops after the dual update, the residual
// kernel updates mu and the factor of d (eq. (varying_penalty)), and a
// ROW_STATE pass starts the next x-step from the rescaled state.
static deconv_status launch_iteration(deconv_plan_s* p, const uint8_t* mask, const float* lam, const float* mu,
                                      IterFlags f, float* x_out, float2* u_out, float4* spec_store,
                                      int iters_since) {
  const bool adapt = p->opt.adapt_t > 0;
  const float* muk = mu_in_use(p, mu);
  for (int q = 1; q < p->max_pass; ++q) {
    // images with fewer passes than the plan's most skip the inner ones
    // they do not have: their spectra stay as they are, so the passes they
    // take are those of their own count
    ColArgs ci = col_args(p, muk);
    ci.npass = p->npass;
    ci.pass_q = q;
    STCHK(launch_cols(p, ci));
    RowArgs ra = row_args(p, mask, lam, muk);
    ra.mode = ROW_INNER;
    ra.npass = p->npass;
    ra.pass_q = q;
    STCHK(launch_rows(p, ra));
  }
  ColArgs ca = col_args(p, muk);
  ca.spec_store = spec_store;
  STCHK(launch_cols(p, ca));
  const bool colour = p->opt.channels > 1;
  const bool resid = f.check || adapt;
  RowArgs ra = row_args(p, mask, lam, muk);
  ra.mode = colour ? ROW_UONLY : ROW_ITER;
  ra.d_in = p->dbuf[p->cur_d];
  ra.d_out = p->dbuf[1 - p->cur_d];
  ra.check = resid;
  ra.store_v = f.store_v || adapt;
  ra.store_x = f.store_x;
  ra.last = f.last || adapt;
  ra.x_out = x_out;
  ra.u_out = u_out;
  STCHK(launch_rows(p, ra));
  if (colour) {
    // joint prox of each colour group: u (in d_out) -> v, d^{i+1}
    int ntile = 0;
    for (auto& m : p->meta) ntile = std::max(ntile, m.nrt);
    hipLaunchKernelGGL(group_prox_kernel, dim3(ntile, p->batch / p->opt.channels), dim3(kNTProx), 0, p->ls,
                       p->d_meta, lam, muk, p->dbuf[p->cur_d], p->dbuf[1 - p->cur_d], p->v, p->partials,
                       resid ? 1 : 0, p->done);
    HIPCHK(hipGetLastError());
  }
  p->cur_d = 1 - p->cur_d;
  if (resid) {
    hipLaunchKernelGGL(residual_kernel, dim3(p->batch), dim3(kNT), 0, p->ls, p->d_meta, p->partials, p->res,
                       p->done, p->nonfinite, p->iters_done, adapt ? 1 : iters_since, f.check,
                       p->opt.tol_primal, p->opt.tol_dual, p->opt.adapt_t, p->mu_cur, p->dscale, p->stop_buf,
                       p->cur_d);
    HIPCHK(hipGetLastError());
  }
  if (adapt || colour) {
    // next x-step from the stored state (d rescaled by the penalty update)
    RowArgs rs = row_args(p, mask, lam, muk);
    rs.mode = ROW_STATE;
    rs.d_in = p->dbuf[p->cur_d];
    rs.d_out = p->dbuf[1 - p->cur_d];
    rs.dscale = adapt ? p->dscale : nullptr;
    STCHK(launch_rows(p, rs));
    p->cur_d = 1 - p->cur_d;
  }
  return DECONV_OK;
}

// Quadratic warm start of z (eqs. (ini_x), (ini_z)): each step solves
// x = (H^T H + tau I)^{-1} H^T ytilde in the column pass and sets z = M_z H x
// in an inner row pass (z-step without over-relaxation).  Starts from the
// spectra of the initial state; v and d are untouched.
static deconv_status warm_start(deconv_plan_s* p, const uint8_t* mask, const float* lam, const float* mu) {
  for (int w = 0; w < p->opt.warm_iters; ++w) {
    ColArgs ca = col_args(p, mu);
    ca.warm = 1;
    ca.warm_tau = p->opt.warm_tau;
    STCHK(launch_cols(p, ca));
    RowArgs ra = row_args(p, mask, lam, mu);
    ra.mode = ROW_INNER;
    ra.alpha = 1.f;
    STCHK(launch_rows(p, ra));
  }
  return DECONV_OK;
}

static deconv_status copy_ckpt(deconv_plan_s* p, int slot, bool to_store) {
  const size_t n = (size_t)p->total_px;
  hipStream_t s = p->ls;
  float* yt = p->ck_yt + n * slot;
  float2* v = p->ck_v + n * slot;
  float2* d = p->ck_d + n * slot;
  if (to_store) {
    HIPCHK(hipMemcpyAsync(yt, p->yt, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(v, p->v, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d, p->dbuf[p->cur_d], sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  } else {
    HIPCHK(hipMemcpyAsync(p->yt, yt, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(p->v, v, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(p->dbuf[p->cur_d], d, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  }
  return DECONV_OK;
}

// iterations per replayed graph when residuals are never checked
constexpr int kGraphChunk = 10;
// without a stop test the host reads nothing between check periods, so one
// graph holds several (up to this many iterations): each graph launch costs
// the queue a gap of several microseconds
constexpr int kGraphIters = 250;

// iterate from the current spectra; handles checkpoints, graphs, stopping
static deconv_status iterate(deconv_plan_s* p, const uint8_t* mask, const float* lam, const float* mu,
                             int iters, float* x_out, bool record_ckpt) {
  hipStream_t s = p->stream;
  const int K = p->opt.check_every;
  const int ck = record_ckpt ? p->opt.ckpt_every : 0;
  const bool stopping = K > 0 && (p->opt.tol_primal > 0 || p->opt.tol_dual > 0);
  if (ck > 0) {
    STCHK(copy_ckpt(p, 0, true));
    p->nck = 1;
  }
  int it = 0;
  while (it < iters) {
    // graph replay of whole check periods (no checkpoint inside, not the
    // last); without checks, of chunks of kGraphChunk iterations; without a
    // stop test, of as many periods as fit in kGraphIters iterations
    const int G0 = K > 0 ? K : kGraphChunk;
    int G = G0;
    if (!stopping) {
      G = G0 * std::max(1, kGraphIters / G0);
      while (G > G0 && it + G >= iters) G -= G0;
    }
    if (p->opt.use_graph && ck == 0 && it % G0 == 0 && it + G < iters) {
      const int cur0 = p->cur_d;
      std::vector<uintptr_t> key = {(uintptr_t)G, (uintptr_t)cur0, (uintptr_t)mask, (uintptr_t)lam,
                                    (uintptr_t)mu, (uintptr_t)x_out};
      auto g = p->graphs.find(key);
      if (g == p->graphs.end()) {
        // capture on the private stream (the caller's may be the null
        // stream, which cannot be captured); the graph is replayed on the
        // caller's stream
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        p->ls = p->cap_stream;
        deconv_status st = DECONV_OK;
        for (int q = 0; q < G && st == DECONV_OK; ++q)
          st = launch_iteration(p, mask, lam, mu, flags_for(p, q, iters + G), x_out, nullptr, nullptr, K);
        hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
        p->ls = p->stream;
        p->cur_d = cur0;   // capturing ran nothing
        if (st != DECONV_OK) return st;
        if (e != hipSuccess) return DECONV_ERR_HIP;
        hipGraphExec_t exec;
        HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        g = p->graphs.emplace(key, exec).first;
      }
      HIPCHK(hipGraphLaunch(g->second, s));
      if ((G * d_swaps_per_iter(p)) % 2) p->cur_d = 1 - cur0;
      it += G;
      if (stopping) {
        std::vector<int> dn(p->batch);
        HIPCHK(hipMemcpyAsync(dn.data(), p->done, sizeof(int) * p->batch, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (std::all_of(dn.begin(), dn.end(), [](int v) { return v != 0; })) break;
      }
      continue;
    }
    IterFlags f = flags_for(p, it, iters);
    if (ck > 0 && ((it + 1) % ck == 0) && it + 1 < iters) f.store_v = 1;
    STCHK(launch_iteration(p, mask, lam, mu, f, x_out, nullptr, nullptr, K));
    ++it;
    if (ck > 0 && (it % ck == 0) && it < iters) {
      STCHK(copy_ckpt(p, it / ck, true));
      p->nck = it / ck + 1;
    }
    if (stopping && f.check) {
      std::vector<int> dn(p->batch);
      HIPCHK(hipMemcpyAsync(dn.data(), p->done, sizeof(int) * p->batch, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (std::all_of(dn.begin(), dn.end(), [](int v) { return v != 0; })) break;
    }
  }
  // Images that stopped early kept x, v and d of their stopping iteration;
  // their d sits in the buffer current then.  Bring it to the current one.
  if (stopping) {
    hipLaunchKernelGGL(stopped_d_kernel, dim3(64, p->batch), dim3(kNT), 0, s, p->d_meta, p->done, p->stop_buf,
                       p->cur_d, p->dbuf[0], p->dbuf[1]);
    HIPCHK(hipGetLastError());
  }
  return DECONV_OK;
}

// Iterations on the whole-image-in-LDS path: one launch per check period
// when a stop test needs the host between periods, else per kSmallIters
// iterations (several check periods; kSmallChunk without checks).  The
// kernel records the residuals of every check in its launch (each
// workgroup holds a whole image) and the stop decisions.  d stays in its
// buffer.
constexpr int kSmallChunk = 50;
constexpr int kSmallIters = 200;

static deconv_status iterate_small(deconv_plan_s* p, const uint8_t* mask, const float* lam, const float* mu,
                                   int iters, float* x_out) {
  hipStream_t s = p->stream;
  const int K = p->opt.check_every;
  const bool stopping = K > 0 && (p->opt.tol_primal > 0 || p->opt.tol_dual > 0);
  int it = 0;
  // launches start at check-period boundaries
  const int span = K > 0 ? (stopping ? K : K * std::max(1, kSmallIters / K)) : kSmallChunk;
  while (it < iters) {
    const int cnt = std::min(span, iters - it);
    SmallArgs a{};
    a.meta = p->d_meta;
    a.yt = p->yt;
    a.d = p->dbuf[p->cur_d];
    a.v = p->v;
    a.hh = p->hh;
    a.tab = p->tab;
    a.mask = mask;
    a.lam = lam;
    a.mu = mu;
    a.tw = p->tw;
    a.done = p->done;
    a.x_out = x_out;
    a.res = p->res;
    a.nonfinite = p->nonfinite;
    a.iters_done = p->iters_done;
    a.stop_buf = p->stop_buf;
    a.tol_p = p->opt.tol_primal;
    a.tol_d = p->opt.tol_dual;
    a.cur_d = p->cur_d;
    a.iters = cnt;
    a.check_every = K;
    a.stop_test = stopping;
    const bool checked = K > 0 && cnt % K == 0;   // the launch ends with a check
    a.store_x = it + cnt == iters || (checked && stopping);
    a.alpha = p->opt.alpha;
    PassTimer timer(p, &p->ev_row);
    for (size_t q = 0; q < p->small_groups.size(); ++q) {
      const auto& g = p->small_groups[q];
      a.imgs = p->d_small + g[1];
      HIPCHK(launch_small(g[0], g[0] > 0 ? g[0] : 0, g[2], s, a, timer.start(q), timer.stop(q, p->small_groups.size())));
    }
    timer.done();
    it += cnt;
    if (checked) {
      if (stopping) {
        std::vector<int> dn(p->batch);
        HIPCHK(hipMemcpyAsync(dn.data(), p->done, sizeof(int) * p->batch, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (std::all_of(dn.begin(), dn.end(), [](int v) { return v != 0; })) break;
      }
    }
  }
  return DECONV_OK;
}

static deconv_status finish(deconv_plan_s* p, int iters, float* ytilde_out, deconv_stats* stats,
                            const float* mu) {
  hipStream_t s = p->stream;
  if (ytilde_out)
    HIPCHK(hipMemcpyAsync(ytilde_out, p->yt, sizeof(float) * p->total_px, hipMemcpyDeviceToDevice, s));
  if (stats) {
    const int B = p->batch;
    std::vector<int> dn(B), itd(B), nf(B);
    std::vector<double> res(3 * B);
    std::vector<float> muh(B);
    HIPCHK(hipMemcpyAsync(muh.data(), mu, sizeof(float) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dn.data(), p->done, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(itd.data(), p->iters_done, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(nf.data(), p->nonfinite, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(res.data(), p->res, sizeof(double) * 3 * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    deconv_status ret = DECONV_OK;
    for (int b = 0; b < B; ++b) {
      stats[b].iters_done = dn[b] ? itd[b] : iters;
      stats[b].r_primal = res[3 * b];
      stats[b].r_dual = res[3 * b + 1];
      stats[b].r_z = res[3 * b + 2];
      stats[b].status = nf[b] ? DECONV_ERR_NONFINITE : DECONV_OK;
      stats[b].mu = muh[b];
      if (nf[b]) ret = DECONV_ERR_NONFINITE;
    }
    return ret;
  }
  return DECONV_OK;
}

static deconv_status reset_counters(deconv_plan_s* p) {
  // done, nonfinite, iters_done, stop_buf and res lie back to back in the
  // workspace (build_layout): one fill
  const long long words = (reinterpret_cast<const char*>(p->res + 3 * p->batch) -
                           reinterpret_cast<const char*>(p->done)) / 4;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)std::min<long long>((words + kNT - 1) / kNT, 64)), dim3(kNT),
                     0, p->stream, reinterpret_cast<unsigned*>(p->done), words);
  HIPCHK(hipGetLastError());
  return DECONV_OK;
}

static bool needs_mask(const deconv_plan_s* p) {
  for (auto& d : p->desc)
    if (d.mask_kind == DECONV_MASK_EXPLICIT) return true;
  return false;
}

extern "C" deconv_status deconv_admm_run(deconv_plan p, const float* y, const uint8_t* mask, const float* h,
                                         const float* lambda, const float* mu, int32_t iters, float* x_out,
                                         float* ytilde_out, deconv_stats* stats) {
  if (!p || !y || !h || !lambda || !mu || !x_out || iters < 1) return DECONV_ERR_INVALID_ARG;
  if (needs_mask(p) && !mask) return DECONV_ERR_INVALID_ARG;
  const bool ckpt = p->opt.ckpt_every > 0;
  if (ckpt && iters > p->opt.max_iters) return DECONV_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  p->have_state = false;
  p->ck_valid = false;
  p->run_id = 0;
  p->mask = mask;
  STCHK(setup_spectrum(p, h, nullptr, true, true));
  STCHK(reset_counters(p));
  hipLaunchKernelGGL(observed_sum_kernel, dim3(kMeanBlocks, p->batch), dim3(kNT), 0, s, p->d_meta, y, mask,
                     p->mean);
  HIPCHK(hipGetLastError());
  p->cur_d = 0;
  hipLaunchKernelGGL(init_state_kernel, dim3(p->max_height, p->batch), dim3(kNT), 0, s, p->d_meta, y, mask,
                     p->mean, kMeanBlocks, p->yt, p->v, p->dbuf[0]);
  HIPCHK(hipGetLastError());
  if (p->opt.adapt_t > 0) {
    HIPCHK(hipMemcpyAsync(p->mu_cur, mu, sizeof(float) * p->batch, hipMemcpyDeviceToDevice, s));
    p->mu_valid = true;
  }
  // (the whole-image-in-LDS kernel starts from the state itself; the
  // spectra of the prologue serve the two-pass kernels and the warm start)
  if (!p->small || p->opt.warm_iters > 0) STCHK(prologue_from_state(p, mu_in_use(p, mu)));
  if (p->opt.warm_iters > 0) STCHK(warm_start(p, mask, lambda, mu));
  if (p->small) STCHK(iterate_small(p, mask, lambda, mu, iters, x_out));
  else STCHK(iterate(p, mask, lambda, mu, iters, x_out, ckpt));
  STCHK(check_spectrum(p));
  p->have_state = true;
  p->last_iters = iters;
  p->ck_valid = ckpt;
  p->run_id = new_run_id();
  p->ck_run_id = ckpt ? p->run_id : 0;
  return finish(p, iters, ytilde_out, stats, mu_in_use(p, mu));
}

extern "C" deconv_status deconv_admm_continue(deconv_plan p, const float* lambda, const float* mu, int32_t iters,
                                              float* x_out, float* ytilde_out, deconv_stats* stats) {
  if (!p || !lambda || !mu || !x_out || iters < 1) return DECONV_ERR_INVALID_ARG;
  if (!p->have_state) return DECONV_ERR_STATE;
  if (needs_mask(p) && !p->mask) return DECONV_ERR_STATE;
  p->ck_valid = false;
  p->run_id = new_run_id();
  STCHK(reset_counters(p));
  // the adaptive penalty goes on from the last adapted mu, for which d is
  // scaled; only a state without one (imported) starts from the caller's
  if (p->opt.adapt_t > 0 && !p->mu_valid) {
    HIPCHK(hipMemcpyAsync(p->mu_cur, mu, sizeof(float) * p->batch, hipMemcpyDeviceToDevice, p->stream));
    p->mu_valid = true;
  }
  if (!p->small) STCHK(prologue_from_state(p, mu_in_use(p, mu)));
  if (p->small) STCHK(iterate_small(p, p->mask, lambda, mu, iters, x_out));
  else STCHK(iterate(p, p->mask, lambda, mu, iters, x_out, false));
  return finish(p, iters, ytilde_out, stats, mu_in_use(p, mu));
}

extern "C" deconv_status deconv_state_export(deconv_plan p, float* ytilde, float* v, float* d) {
  if (!p || !ytilde || !v || !d) return DECONV_ERR_INVALID_ARG;
  if (!p->have_state) return DECONV_ERR_STATE;
  hipStream_t s = p->stream;
  const size_t n = (size_t)p->total_px;
  HIPCHK(hipMemcpyAsync(ytilde, p->yt, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(v, p->v, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(d, p->dbuf[p->cur_d], sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  return DECONV_OK;
}

extern "C" deconv_status deconv_state_import(deconv_plan p, const uint8_t* mask, const float* h,
                                             const float* ytilde, const float* v, const float* d) {
  if (!p || !h || !ytilde || !v || !d) return DECONV_ERR_INVALID_ARG;
  if (needs_mask(p) && !mask) return DECONV_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  p->mask = mask;
  const size_t n = (size_t)p->total_px;
  STCHK(setup_spectrum(p, h, nullptr));
  HIPCHK(hipMemcpyAsync(p->yt, ytilde, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(p->v, v, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  p->cur_d = 0;
  HIPCHK(hipMemcpyAsync(p->dbuf[0], d, sizeof(float2) * n, hipMemcpyDeviceToDevice, s));
  p->have_state = true;
  p->ck_valid = false;
  p->mu_valid = false;
  p->run_id = new_run_id();
  return DECONV_OK;
}

extern "C" deconv_status deconv_blur_spectrum(deconv_plan p, const float* h, float* spectrum_out) {
  if (!p || !h || !spectrum_out) return DECONV_ERR_INVALID_ARG;
  deconv_status st = setup_spectrum(p, h, spectrum_out, false);
  if (st != DECONV_OK) return st;
  HIPCHK(hipStreamSynchronize(p->stream));
  return DECONV_OK;
}

extern "C" deconv_status deconv_fft2(int32_t count, int32_t height, int32_t width, float* data, int32_t inverse,
                                     void* stream) {
  if (count < 1 || !data) return DECONV_ERR_INVALID_ARG;
  if (!supported_len(height) || !supported_len(width)) return DECONV_ERR_UNSUPPORTED_SIZE;
  if ((int)fftrow_lds_bytes(width) > max_lds_bytes() || (int)fftcol_lds_bytes(height) > max_lds_bytes())
    return DECONV_ERR_UNSUPPORTED_SIZE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float2* twr = cached_twiddles(width);
  const float2* twc = cached_twiddles(height);
  if (!twr || !twc) return DECONV_ERR_HIP;
  float2* g = reinterpret_cast<float2*>(data);
  HIPCHK(launch_fft_rows(width, g, (long long)count * height, twr, inverse ? 1 : 0, s));
  HIPCHK(launch_fft_cols(height, g, width, count, twc, inverse ? 1 : 0, s));
  return DECONV_OK;
}

#include "backward_host.inc"

static deconv_status pass_times(deconv_plan_s* p, double* out, bool reverse) {
  HIPCHK(hipStreamSynchronize(p->stream));
  double ms[2] = {0.0, 0.0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* lists[2] = {reverse ? &p->ev_brow : &p->ev_row,
                                                              reverse ? &p->ev_bcol : &p->ev_col};
  for (int k = 0; k < 2; ++k) {
    for (auto& e : *lists[k]) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
      ms[k] += t;
      p->ev_pool.push_back(e.first);
      p->ev_pool.push_back(e.second);
    }
    out[2 * k] = ms[k];
    out[2 * k + 1] = (double)lists[k]->size();
    lists[k]->clear();
  }
  return DECONV_OK;
}

extern "C" deconv_status deconv_plan_kernel_times(deconv_plan p, double* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  return pass_times(p, out, false);
}

extern "C" deconv_status deconv_plan_bwd_kernel_times(deconv_plan p, double* out) {
  if (!p || !out) return DECONV_ERR_INVALID_ARG;
  return pass_times(p, out, true);
}

extern "C" const char* deconv_status_str(deconv_status s) {
  switch (s) {
    case DECONV_OK: return "ok";
    case DECONV_ERR_INVALID_ARG: return "invalid argument";
    case DECONV_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case DECONV_ERR_SINGULAR: return "blur has zero DC gain (sum(h) == 0)";
    case DECONV_ERR_NONFINITE: return "non-finite values in the iteration";
    case DECONV_ERR_NO_CHECKPOINTS: return "backward needs a checkpointed forward run";
    case DECONV_ERR_HIP: return "HIP runtime error";
    case DECONV_ERR_OOM: return "out of memory / workspace too small";
    case DECONV_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}
