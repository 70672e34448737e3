// Instantiations and launcher of one pass (see launch.hpp).
#include "launch.hpp"

namespace dcv {

size_t col_lds_bytes(int L) {
  switch (L) {
#define DCV_CASE(n) case n: return col_lds_elems(n) * sizeof(float2);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return 0;
}

hipError_t launch_col(int L, int grid, size_t lds, hipStream_t s, ColArgs a, hipEvent_t e0, hipEvent_t e1,
                      bool wide) {
  void* args[] = {&a};
  if (wide) {
    switch (L) {
#define DCV_CASE(n) case n: return launch_lds(col_kernel<n, kNTCWide>, grid, lds, s, args, kNTCWide, e0, e1);
      DCV_FOR_EACH_WIDE_COL_LEN(DCV_CASE)
#undef DCV_CASE
    }
  }
  if (L < 0 && -L <= kShortLenMax)
    return launch_lds(col_kernel_multi<DCV_SHORT_LEN_ARGS>, grid, lds, s, args, kNTC, e0, e1);
  if (L <= 0) return launch_lds(col_kernel_multi<DCV_LEN_ARGS>, grid, lds, s, args, kNTC, e0, e1);
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(col_kernel<n>, grid, lds, s, args, kNTC, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
