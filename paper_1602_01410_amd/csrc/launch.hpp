// Host-side launchers of the row and column passes, one translation unit
// each (pass_*.hip) so that their many length instantiations compile in
// parallel.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "backward.hpp"
#include "kernels.hpp"

// every supported line length: 2^a 3^c, a >= 1, c <= 2, 8 <= L <= 2048
#define DCV_FOR_EACH_LEN(X)                                                                    \
  X(8) X(12) X(16) X(18) X(24) X(32) X(36) X(48) X(64) X(72) X(96) X(128) X(144) X(192)   \
  X(256) X(288) X(384) X(512) X(576) X(768) X(1024) X(1152) X(1536) X(2048)

#define DCV_LEN_ARGS                                                                            \
  8, 12, 16, 18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256, 288, 384, 512, 576, 768, 1024, 1152, \
      1536, 2048

namespace dcv {

inline bool supported_len(int L) {
  switch (L) {
#define DCV_CASE(n) case n: return true;
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return false;
}

// Launch with dynamic LDS.  With events, they are attached to the dispatch
// itself (hipExtLaunchKernel), so they time the kernel and not the gap
// before it.
template <typename K>
inline hipError_t launch_lds(K kernel, int grid, size_t lds, hipStream_t s, void** args, int nt,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (e0 || e1)
    return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(grid), dim3(nt), args, lds, s, e0, e1, 0);
  return hipLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(grid), dim3(nt), args, lds, s);
}

// L = 0 launches the kernel that dispatches on each tile's length.
// launch_row picks the plain-iteration instantiation when the arguments ask
// for no residuals and no stores of v, x or u.
size_t row_lds_bytes(int L, int rt = 0);
size_t col_lds_bytes(int L);
// rt: rows per tile of the group (0 or rt_for(L): the default; rt_half(L) for
// the lengths of DCV_FOR_EACH_HALF_RT_LEN)
hipError_t launch_row(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_row_plain(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0,
                            hipEvent_t e1);
hipError_t launch_col(int L, int grid, size_t lds, hipStream_t s, ColArgs a, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_bwd_row(int L, int grid, size_t lds, hipStream_t s, BwdRowArgs a);
hipError_t launch_bwd_col(int L, int grid, size_t lds, hipStream_t s, BwdColArgs a);

}  // namespace dcv
