// Instantiations and launcher of one pass (see launch.hpp).
#include "launch.hpp"

namespace dcv {

size_t row_lds_bytes(int L, int rt) {
  switch (L) {
#define DCV_CASE(n) case n: return row_lds_elems(n, rt) * sizeof(float2);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return 0;
}

hipError_t launch_row(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0, hipEvent_t e1) {
  const bool plain = a.mode == ROW_ITER && !a.check && !a.store_v && !a.store_x && !a.u_out && !a.last;
  if (plain) return launch_row_plain(L, rt, grid, lds, s, a, e0, e1);
  void* args[] = {&a};
  if (L == 0) return launch_lds(row_kernel_multi<false, DCV_LEN_ARGS>, grid, lds, s, args, kNTR, e0, e1);
  if (rt > 0 && L > 0 && rt != rt_for(L)) {
    switch (L) {
#define DCV_CASE(n) \
  case n: return rt == rt_half(n) ? launch_lds(row_kernel<n, false, rt_half(n)>, grid, lds, s, args, kNTR, e0, e1) \
                                  : hipErrorInvalidValue;
      DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
    }
    return hipErrorInvalidValue;
  }
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(row_kernel<n, false>, grid, lds, s, args, kNTR, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
