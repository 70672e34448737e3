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

// the lengths up to kShortLenMax: a multi-length launch whose lengths are all
// short dispatches over these only (fewer registers than the full list)
#define DCV_SHORT_LEN_ARGS 8, 12, 16, 18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256, 288

namespace dcv {

constexpr int kShortLenMax = 288;

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

// L <= 0 launches a kernel that dispatches on each tile's length; -L is the
// longest length among the tiles (0: unknown, any length).
// launch_row picks the row-pass variant the arguments need (row_variant).
size_t row_lds_bytes(int L, int rt = 0);
size_t col_lds_bytes(int L);
// rt: rows per tile of the group (0 or rt_for(L): the default; rt_half(L) for
// the lengths of DCV_FOR_EACH_HALF_RT_LEN)
// wide: kNTRWide threads per half-height tile (plans with few tiles), for
// the RV_PLAIN and RV_STOREV variants
hipError_t launch_row(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr, bool wide = false);
// one row-pass variant (RV_*): instantiated in its own translation unit
template <int V>
hipError_t launch_row_variant(int L, int rt, int grid, size_t lds, hipStream_t s, RowArgs a, hipEvent_t e0,
                              hipEvent_t e1, bool wide) {
  void* args[] = {&a};
  // the check variant holds more registers: at 1024 threads one workgroup per
  // compute unit would fit, so it keeps kNTR
  if constexpr (V == RV_PLAIN || V == RV_STOREV) {
    if (wide && rt > 0 && rt != rt_for(L)) {
      switch (L) {
#define DCV_CASE(n)                                                                                        \
  case n: return rt == rt_half(n) ? launch_lds(row_kernel<n, V, rt_half(n), kNTRWide>, grid, lds, s, args, \
                                               kNTRWide, e0, e1)                                           \
                                  : hipErrorInvalidValue;
        DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
      }
      return hipErrorInvalidValue;
    }
  }
  if (L < 0 && -L <= kShortLenMax)
    return launch_lds(row_kernel_multi<V, DCV_SHORT_LEN_ARGS>, grid, lds, s, args, kNTR, e0, e1);
  if (L <= 0) return launch_lds(row_kernel_multi<V, DCV_LEN_ARGS>, grid, lds, s, args, kNTR, e0, e1);
  if (rt > 0 && rt != rt_for(L)) {
    switch (L) {
#define DCV_CASE(n) \
  case n: return rt == rt_half(n) ? launch_lds(row_kernel<n, V, rt_half(n)>, grid, lds, s, args, kNTR, e0, e1) \
                                  : hipErrorInvalidValue;
      DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
    }
    return hipErrorInvalidValue;
  }
  switch (L) {
#define DCV_CASE(n) case n: return launch_lds(row_kernel<n, V>, grid, lds, s, args, kNTR, e0, e1);
    DCV_FOR_EACH_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return hipErrorInvalidValue;
}
extern template hipError_t launch_row_variant<RV_PLAIN>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                        hipEvent_t, bool);
extern template hipError_t launch_row_variant<RV_STOREV>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                         hipEvent_t, bool);
extern template hipError_t launch_row_variant<RV_CHECK>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                        hipEvent_t, bool);
extern template hipError_t launch_row_variant<RV_GENERIC>(int, int, int, size_t, hipStream_t, RowArgs, hipEvent_t,
                                                          hipEvent_t, bool);
// wide: kNTCWide threads per column tile where the length has that
// instantiation (has_wide_col), for plans with few tiles
#define DCV_FOR_EACH_WIDE_COL_LEN(X) X(512) X(576) X(768) X(1024) X(1152) X(1536) X(2048)
inline bool has_wide_col(int L) {
  switch (L) {
#define DCV_CASE(n) case n: return true;
    DCV_FOR_EACH_WIDE_COL_LEN(DCV_CASE)
#undef DCV_CASE
  }
  return false;
}
hipError_t launch_col(int L, int grid, size_t lds, hipStream_t s, ColArgs a, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr, bool wide = false);
// whole-image-in-LDS path (small.hpp): square images of a few sides
struct SmallArgs;
bool has_small_path(int M, int N);
// largest side that the default option (small_images = 2) sends to the
// whole-image-in-LDS path
constexpr int kSmallAutoSide = 72;
hipError_t launch_small(int M, int N, int grid, hipStream_t s, SmallArgs a, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_bwd_row(int L, int grid, size_t lds, hipStream_t s, BwdRowArgs a, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t launch_bwd_col(int L, int grid, size_t lds, hipStream_t s, BwdColArgs a, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);

}  // namespace dcv
