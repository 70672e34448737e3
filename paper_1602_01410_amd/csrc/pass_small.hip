// Instantiations and launcher of the whole-image-in-LDS path (small.hpp).
#include <algorithm>

#include "launch.hpp"
#include "small.hpp"

namespace dcv {

#define DCV_FOR_EACH_SMALL_SIDE(X) X(32) X(48) X(64) X(72) X(96)
#define DCV_SMALL_SIDE_ARGS 32, 48, 64, 72, 96

bool has_small_path(int M, int N) {
  if (M != N) return false;
  switch (M) {
#define DCV_CASE(n) case n: return SmallShape<n, n>::lds_bytes <= 160 * 1024;
    DCV_FOR_EACH_SMALL_SIDE(DCV_CASE)
#undef DCV_CASE
  }
  return false;
}

template <int M, int N>
static hipError_t launch_small_mn(int grid, hipStream_t s, SmallArgs a, hipEvent_t e0, hipEvent_t e1) {
  static bool attr = false;
  const size_t lds = SmallShape<M, N>::lds_bytes;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(small_kernel<M, N>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  void* args[] = {&a};
  return launch_lds(small_kernel<M, N>, grid, lds, s, args, kNTS, e0, e1);
}

hipError_t launch_small(int M, int N, int grid, hipStream_t s, SmallArgs a, hipEvent_t e0, hipEvent_t e1) {
  if (M <= 0) {
    // images of several sides: one launch, LDS for the largest (-M)
    static bool attr = false;
    size_t lds = 0;
#define DCV_CASE(n) lds = std::max(lds, SmallShape<n, n>::lds_bytes);
    DCV_FOR_EACH_SMALL_SIDE(DCV_CASE)
#undef DCV_CASE
    const auto k = small_kernel_multi<DCV_SMALL_SIDE_ARGS>;
    if (!attr) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr = true;
    }
    void* args[] = {&a};
    return launch_lds(k, grid, lds, s, args, kNTS, e0, e1);
  }
  if (M == N) {
    switch (M) {
#define DCV_CASE(n) case n: return launch_small_mn<n, n>(grid, s, a, e0, e1);
      DCV_FOR_EACH_SMALL_SIDE(DCV_CASE)
#undef DCV_CASE
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace dcv
