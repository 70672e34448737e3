// Row-pass instantiations for plain iterations (see launch.hpp).
#include "launch.hpp"

namespace dcv {

template hipError_t launch_row_variant<RV_PLAIN>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                 hipEvent_t, bool);

}  // namespace dcv
