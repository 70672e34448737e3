// Row-pass instantiations for the iteration before a residual check (v
// stored) and for the check itself (see launch.hpp).
#include "launch.hpp"

namespace dcv {

template hipError_t launch_row_variant<RV_STOREV>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                  hipEvent_t, bool);
template hipError_t launch_row_variant<RV_CHECK>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                 hipEvent_t, bool);

}  // namespace dcv
