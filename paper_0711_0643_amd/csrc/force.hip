// Launchers of the force kernel (the kernel itself: force_impl.h).  The
// autotuner's other builds of the lean tile-relative kernel are compiled in
// force_tuned.hip.
#include "force_impl.h"

namespace nb {

// WPE: waves per SIMD the kernel is built for (SPLIT: 4, else 3).  Every
// default build needs no scratch memory: a kernel that does costs several
// microseconds more per launch, which dominates the small blocks.
template <int MODE, bool NEAR, bool SPLIT, bool LEAN = false, int WPE = (SPLIT ? 4 : 3)>
static void launch_mode(const ForceLaunch& L, bool pot) {
  if (pot)
    hipLaunchKernelGGL((force_kernel<MODE, true, NEAR, SPLIT, LEAN, 32, WPE>), dim3(L.grid), dim3(kForceThreads), 0,
                       L.st, L.s, L.act, L.par, L.target_items);
  else
    hipLaunchKernelGGL((force_kernel<MODE, false, NEAR, SPLIT, LEAN, 32, WPE>), dim3(L.grid), dim3(kForceThreads), 0,
                       L.st, L.s, L.act, L.par, L.target_items);
}

template <bool SPLIT>
static hipError_t launch_family(const ForceLaunch& L, int mode, bool pot, bool near) {
  switch (mode) {
    case kF64: launch_mode<kF64, false, SPLIT>(L, pot); break;
    case kDS:
      if (near) launch_mode<kDS, true, SPLIT>(L, pot);
      else launch_mode<kDS, false, SPLIT>(L, pot);
      break;
    case kMX64:
      if (near) launch_mode<kMX64, true, SPLIT>(L, pot);
      else launch_mode<kMX64, false, SPLIT>(L, pot);
      break;
    case kTR:
      if (SPLIT) {
        // every split layout runs the FP64 arithmetic in this mode
        launch_mode<kF64, false, true>(L, pot);
      } else if (near && L.lean) {
        // the default builds that need no scratch memory: 4 waves per SIMD
        // without the potential, 3 with it
        if (!pot && (L.window != 32 || L.waves != 4 || L.tile != kTile)) return launch_force_tuned(L);
        if (pot)
          hipLaunchKernelGGL((force_kernel<kTR, true, true, false, true, 32, 3>), dim3(L.grid), dim3(kForceThreads), 0,
                             L.st, L.s, L.act, L.par, L.target_items);
        else
          hipLaunchKernelGGL((force_kernel<kTR, false, true, false, true, 32, 4>), dim3(L.grid), dim3(kForceThreads), 0,
                             L.st, L.s, L.act, L.par, L.target_items);
      } else if (near) {
        launch_mode<kTR, true, false>(L, pot);
      } else {
        launch_mode<kTR, false, false>(L, pot);
      }
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_force(const DevState& s, int mode, bool pot, bool near, bool split, bool lean, const int32_t* act,
                        int grid, int par, int64_t target_items, hipStream_t st, int window, int waves, int tile) {
  const ForceLaunch L{s, act, grid, par, lean, target_items, st, window, waves, tile};
  return split ? launch_family<true>(L, mode, pot, near) : launch_family<false>(L, mode, pot, near);
}

}  // namespace nb
