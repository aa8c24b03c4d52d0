// The autotuner's builds of the lean tile-relative force kernel without the
// potential on j-tiles of 128 records: FP32 window of 16 or 32 pairs and an
// occupancy of 2 to 5 waves per SIMD (a 64-pair window on these tiles
// spills kilobytes of registers and is not built).  Compiled on its own so
// that the library's sources build in parallel.
#include "force_impl.h"

namespace nb {

template <int FW, int WPE>
static void launch_tr128(const ForceLaunch& L) {
  hipLaunchKernelGGL((force_kernel<kTR, false, true, false, true, FW, WPE, 128>), dim3(L.grid),
                     dim3(kForceThreads), 0, L.st, L.s, L.act, L.par, L.target_items);
}

hipError_t launch_force_tuned_t128(const ForceLaunch& L) {
  switch (L.window * 10 + L.waves) {
    case 162: launch_tr128<16, 2>(L); break;
    case 163: launch_tr128<16, 3>(L); break;
    case 164: launch_tr128<16, 4>(L); break;
    case 165: launch_tr128<16, 5>(L); break;
    case 322: launch_tr128<32, 2>(L); break;
    case 323: launch_tr128<32, 3>(L); break;
    case 324: launch_tr128<32, 4>(L); break;
    case 325: launch_tr128<32, 5>(L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nb
