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

// The builds with the fused predictor (PIF): FP64 in both families, and the
// default lean tile-relative build (whose j-split layouts run FP64); the
// host switches the predictor on only where one of these runs.
template <int MODE, bool POT, bool SPLIT, bool LEAN, int WPE>
static void launch_pif(const ForceLaunch& L) {
  hipLaunchKernelGGL((force_kernel<MODE, POT, MODE == kTR, SPLIT, LEAN, 32, WPE, kTile, true>), dim3(L.grid),
                     dim3(kForceThreads), 0, L.st, L.s, L.act, L.par, L.target_items);
}

static hipError_t launch_family_pif(const ForceLaunch& L, int mode, bool pot, bool near, bool split) {
  const bool tr_split = mode == kTR && split;
  if (mode == kF64 || tr_split) {
    if (split) {
      if (pot) launch_pif<kF64, true, true, false, 4>(L);
      else launch_pif<kF64, false, true, false, 4>(L);
    } else {
      if (pot) launch_pif<kF64, true, false, false, 3>(L);
      else launch_pif<kF64, false, false, false, 3>(L);
    }
  } else if (mode == kTR && near && L.lean && (pot || (L.window == 32 && L.waves == 4 && L.tile == kTile))) {
    if (pot) launch_pif<kTR, true, false, true, 3>(L);
    else launch_pif<kTR, false, false, true, 4>(L);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool has_pif_build(int mode, bool pot, bool near, bool split, bool lean, int window, int waves, int tile) {
  const bool lean_default = near && lean && (pot || (window == 32 && waves == 4 && tile == kTile));
  return mode == kF64 || (mode == kTR && (split || lean_default));
}

hipError_t launch_force(const DevState& s, int mode, bool pot, bool near, bool split, bool lean, const int32_t* act,
                        int grid, int par, int64_t target_items, hipStream_t st, int window, int waves, int tile,
                        bool pif) {
  const ForceLaunch L{s, act, grid, par, lean, target_items, st, window, waves, tile};
  if (pif) return launch_family_pif(L, mode, pot, near, split);
  return split ? launch_family<true>(L, mode, pot, near) : launch_family<false>(L, mode, pot, near);
}

}  // namespace nb
