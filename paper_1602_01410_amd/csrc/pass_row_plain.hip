// Instantiations of the row pass for plain iterations (see launch.hpp).
#include "launch.hpp"

namespace dcv {

hipError_t launch_row_plain(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0, hipEvent_t e1) {
  void* args[] = {&a};
  if (L == 0) return launch_lds(row_kernel_multi<true, DCV_LEN_ARGS>, grid, lds, s, args, kNTR, e0, e1);
  if (rt > 0 && L > 0 && rt != rt_for(L)) {
    switch (L) {
#define DCV_CASE(n) \
  case n: return rt == rt_half(n) ? launch_lds(row_kernel<n, true, rt_half(n)>, grid, lds, s, args, kNTR, e0, e1) \
                                  : hipErrorInvalidValue;
      DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
    }
    return hipErrorInvalidValue;
  }
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(row_kernel<n, true>, grid, lds, s, args, kNTR, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
