// Perturber lists (Sect. 3.1, "Parallelizing the perturber list"): for each
// listed particle i, the particles j != i of its cluster whose force on i
// exceeds a threshold, in the order a serial sweep over the particles
// identifies them (ascending particle id), at most max_pert of them.  The
// paper broadcasts every processor's candidates and sorts them into that
// order; here the predicted positions and masses are first staged in id
// order, then one wavefront sweeps the whole cluster for its i in id order
// and compacts the passing ids in place, so the order comes out directly.
// The test m_j / R^2 > threshold is taken in FP64 with R^2 formed as
// ((dx dx + dy dy) + dz dz) + eps^2, every operation rounded (no fused
// multiply-add), so a list is the same bit for bit on any machine that
// rounds as IEEE does.
#include "kernels.h"

namespace nb {

namespace {

constexpr int kPertThreads = 256;
constexpr int kPertPer = 4;  // consecutive ids per lane per round

__device__ __forceinline__ double softened_r2(double dx, double dy, double dz, double eps2) {
#pragma clang fp contract(off)
  return dx * dx + dy * dy + dz * dz + eps2;
}

// Predicted positions and masses in particle-id order (s.pid), so that the
// sweeps below read them coalesced in the order they test them.
__global__ void __launch_bounds__(256) stage_by_id_kernel(DevState s) {
  const int64_t n = s.n;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const int64_t sj = s.slot_of[j];
    s.pid[j] = s.xp[sj];
    s.pid[n + j] = s.xp[n + sj];
    s.pid[2 * n + j] = s.xp[2 * n + sj];
    s.pid[3 * n + j] = s.m[sj];
  }
}

// One wavefront per active entry q (grid-stride over entries, four per
// workgroup).  Each round covers 64 * kPertPer consecutive ids, lane l the
// kPertPer ids from l * kPertPer on; an exclusive scan of the lanes' pass
// counts (shuffles only: no barrier, no LDS) gives every passing id its
// place, so the list fills in ascending order.
__global__ void __launch_bounds__(kPertThreads)
perturbers_kernel(DevState s, const int32_t* __restrict__ ids, const int64_t* __restrict__ aoff, int64_t n_active,
                  const double* __restrict__ thr, int32_t cap, int32_t* __restrict__ lists,
                  int32_t* __restrict__ counts) {
  constexpr int kWaves = kPertThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = s.n;
  const double* X = s.pid;
  const double* Y = s.pid + n;
  const double* Z = s.pid + 2 * n;
  const double* M = s.pid + 3 * n;
  for (int64_t q = (int64_t)blockIdx.x * kWaves + wave; q < n_active; q += (int64_t)gridDim.x * kWaves) {
    // cluster of entry q: the last c with aoff[c] <= q
    int lo = 0, hi = s.nc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (aoff[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const int64_t b = s.coff[c], e = s.coff[c + 1];
    const int64_t id = ids[q];
    int32_t found = 0;
    if (id >= b && id < e) {
      const double xi = X[id], yi = Y[id], zi = Z[id];
      const double eps2 = s.eps[c] * s.eps[c];
      const double t = thr[c];
      for (int64_t j0 = b; j0 < e; j0 += 64 * kPertPer) {
        const int64_t jb = j0 + (int64_t)lane * kPertPer;
        unsigned bits = 0;
#pragma unroll
        for (int u = 0; u < kPertPer; ++u) {
          const int64_t j = jb + u;
          if (j < e && j != id) {
            const double r2 = softened_r2(X[j] - xi, Y[j] - yi, Z[j] - zi, eps2);
            if (M[j] / r2 > t) bits |= 1u << u;
          }
        }
        const int cnt = __popc(bits);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int up = __shfl_up(incl, o);
          if (lane >= o) incl += up;
        }
        int at = found + incl - cnt;
#pragma unroll
        for (int u = 0; u < kPertPer; ++u) {
          if ((bits >> u) & 1u) {
            if (at < cap) lists[q * cap + at] = (int32_t)(jb + u);
            ++at;
          }
        }
        found += __shfl(incl, 63);
      }
    } else if (lane == 0) {
      __hip_atomic_fetch_or(s.status, (int32_t)ST_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int k = (found < cap ? found : cap) + lane; k < cap; k += 64) lists[q * cap + k] = -1;
    if (lane == 0) counts[q] = found;
  }
}

}  // namespace

hipError_t launch_perturbers(const DevState& s, const int32_t* ids, const int64_t* aoff, int64_t n_active,
                             const double* thr, int32_t cap, int32_t* lists, int32_t* counts, hipStream_t st) {
  const int64_t sg = (s.n + 255) / 256;
  hipLaunchKernelGGL(stage_by_id_kernel, dim3((unsigned)(sg < 65536 ? sg : 65536)), dim3(256), 0, st, s);
  const int64_t wgs = (n_active + kPertThreads / 64 - 1) / (kPertThreads / 64);
  const int64_t grid = wgs < 65536 ? wgs : 65536;
  hipLaunchKernelGGL(perturbers_kernel, dim3((unsigned)grid), dim3(kPertThreads), 0, st, s, ids, aoff, n_active, thr,
                     cap, lists, counts);
  return hipGetLastError();
}

}  // namespace nb
