// Row-pass launcher and its generic instantiation (see launch.hpp).
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

template hipError_t launch_row_variant<RV_GENERIC>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                   hipEvent_t, bool);

hipError_t launch_row(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0, hipEvent_t e1,
                      bool wide) {
  switch (row_variant(a)) {
    case RV_PLAIN: return launch_row_variant<RV_PLAIN>(L, rt, grid, lds, s, a, e0, e1, wide);
    case RV_STOREV: return launch_row_variant<RV_STOREV>(L, rt, grid, lds, s, a, e0, e1, wide);
    case RV_CHECK: return launch_row_variant<RV_CHECK>(L, rt, grid, lds, s, a, e0, e1, wide);
    default: return launch_row_variant<RV_GENERIC>(L, rt, grid, lds, s, a, e0, e1, false);
  }
}

}  // namespace dcv
