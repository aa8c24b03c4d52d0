// The autotuner's other builds of the lean tile-relative force kernel
// without the potential on j-tiles of 256 records: FP32 window of 16, 32 or
// 64 pairs and an occupancy of 2 to 5 waves per SIMD (the default, 32 and
// 4, is built with the other kernels in force.hip; the 128-record tiles in
// force_tuned_t128.hip).  Compiled on its own so that the library's sources
// build in parallel.
#include "force_impl.h"

namespace nb {

template <int FW, int WPE>
static void launch_tr(const ForceLaunch& L) {
  hipLaunchKernelGGL((force_kernel<kTR, false, true, false, true, FW, WPE>), dim3(L.grid), dim3(kForceThreads), 0,
                     L.st, L.s, L.act, L.par, L.target_items);
}

hipError_t launch_force_tuned(const ForceLaunch& L) {
  if (L.tile == 128) return launch_force_tuned_t128(L);
  switch (L.window * 10 + L.waves) {
    case 162: launch_tr<16, 2>(L); break;
    case 163: launch_tr<16, 3>(L); break;
    case 164: launch_tr<16, 4>(L); break;
    case 322: launch_tr<32, 2>(L); break;
    case 323: launch_tr<32, 3>(L); break;
    case 642: launch_tr<64, 2>(L); break;
    case 643: launch_tr<64, 3>(L); break;
    case 644: launch_tr<64, 4>(L); break;
    case 165: launch_tr<16, 5>(L); break;
    case 325: launch_tr<32, 5>(L); break;
    case 645: launch_tr<64, 5>(L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nb
