// deconv_admm_run_static (include/deconv.h): a whole run whose workspace is a
// file-scope device array instead of a device allocation, for callers that
// cannot allocate.  Built on the public entry points only.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>

#include "../../include/deconv.h"

#define HIPCHK(expr)                                                      \
  do {                                                                    \
    if ((expr) != hipSuccess) return DECONV_ERR_HIP;                      \
  } while (0)

#define STCHK(expr)                                \
  do {                                             \
    deconv_status s_ = (expr);                     \
    if (s_ != DECONV_OK) return s_;                \
  } while (0)

// The workspace: one copy per GPU, held until the process ends.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device -> address of its copy of scratch

// Address of the current device's copy of scratch, looked up once per device
// (with that device current).  Host code passes this address to kernels and
// copies, never the array's own name.
static deconv_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return DECONV_OK;
}

extern "C" deconv_status deconv_admm_run_static(int32_t batch, const deconv_image_desc* desc,
                                                const deconv_options* opt, void* stream, const float* y,
                                                const uint8_t* mask, const float* h, const float* lambda,
                                                const float* mu, int32_t iters, float* x_out, float* ytilde_out,
                                                deconv_stats* stats) {
  deconv_options o;
  if (opt) o = *opt;
  else deconv_options_default(&o);
  // no reverse pass (the plan ends with the call); no graphs, events or
  // autotuning (they allocate)
  if (o.ckpt_every != 0) return DECONV_ERR_INVALID_ARG;
  o.use_graph = 0;
  o.profile = 0;
  o.tune_cache = nullptr;
  if (o.schedule == 0) o.schedule = 3;
  size_t need = 0;
  STCHK(deconv_plan_workspace_size(batch, desc, &o, &need));
  if (need > kStaticScratchBytes) {
    fprintf(stderr, "deconv_admm_run_static: the batch needs %zu bytes of workspace, more than the %zu of the "
            "static array\n", need, kStaticScratchBytes);
    return DECONV_ERR_OOM;
  }
  void* ws = nullptr;
  STCHK(scratch_address(&ws));
  deconv_plan p = nullptr;
  STCHK(deconv_plan_create(&p, batch, desc, &o, stream, ws, kStaticScratchBytes));
  const deconv_status st = deconv_admm_run(p, y, mask, h, lambda, mu, iters, x_out, ytilde_out, stats);
  deconv_plan_destroy(p);
  return st;
}
