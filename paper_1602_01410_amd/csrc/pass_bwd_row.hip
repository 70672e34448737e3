// Instantiations and launcher of one pass (see launch.hpp).
#include "launch.hpp"

namespace dcv {

hipError_t launch_bwd_row(int L, int grid, size_t lds, hipStream_t s, BwdRowArgs a, hipEvent_t e0, hipEvent_t e1) {
  void* args[] = {&a};
  if (L <= 0) return launch_lds(bwd_row_kernel_multi<DCV_LEN_ARGS>, grid, lds, s, args, kNTR, e0, e1);
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(bwd_row_kernel<n>, grid, lds, s, args, kNTR, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
