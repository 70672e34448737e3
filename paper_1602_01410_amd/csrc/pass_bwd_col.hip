// Instantiations and launcher of one pass (see launch.hpp).
#include "launch.hpp"

namespace dcv {

hipError_t launch_bwd_col(int L, int grid, size_t lds, hipStream_t s, BwdColArgs a, hipEvent_t e0, hipEvent_t e1) {
  void* args[] = {&a};
  if (L <= 0) return launch_lds(bwd_col_kernel_multi<DCV_LEN_ARGS>, grid, lds, s, args, kNTC, e0, e1);
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(bwd_col_kernel<n>, grid, lds, s, args, kNTC, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
