// Perturber lists (Sect. 3.1, "Parallelizing the perturber list"): for each
// listed particle i, the particles j != i of its cluster whose force on i
// exceeds a threshold, in the order a serial sweep over the particles
// identifies them (ascending particle id), at most max_pert of them.  The
// paper broadcasts every processor's candidates and sorts them into that
// order; here the predicted positions and masses are first staged in id
// order, then each listed i sweeps its whole cluster in id order (through
// LDS tiles shared by a group of i's) and places the passing ids in order as
// they are found, so the order comes out directly.
// The test m_j / R^2 > threshold is taken in FP64 with R^2 formed as
// ((dx dx + dy dy) + dz dz) + eps^2, every operation rounded (no fused
// multiply-add), so a list is the same bit for bit on any machine that
// rounds as IEEE does.
#include "kernels.h"

namespace nb {

namespace {

constexpr int kPertThreads = 256;
constexpr int kPertGroup = 16;    // listed particles per workgroup
constexpr int kPertRound = 1024;  // j-ids per LDS round

__device__ __forceinline__ double softened_r2(double dx, double dy, double dz, double eps2) {
#pragma clang fp contract(off)
  return dx * dx + dy * dy + dz * dz + eps2;
}

// fl(m / r2) > t without the division where its outcome is certain.  With
// t and p = fl(t r2) well inside the normal range, m > fl(p (1 + 2^-40))
// gives m / r2 > t (1 + 2^-40 - 3u) exactly, so the rounded quotient
// exceeds t; m < fl(p (1 - 2^-40)) gives a rounded quotient below t
// (u = 2^-53, every rounding a relative error of at most u there).
// Otherwise (|m / (t r2) - 1| within about 2^-40, t not positive, anything
// out of range, NaN) the rounded quotient itself decides, as the
// definition states.
// t_ok: t within (2^-1000, 2^1000), the same for the whole cluster.  Nearly
// every pair fails with certainty, so that side is tested first and the
// rest runs only where some lane of the wavefront needs it.
__device__ __forceinline__ bool above_threshold(double m, double r2, double t, bool t_ok) {
#pragma clang fp contract(off)
  const double p = t * r2;
  const bool ok = t_ok && p > 0x1p-1000 && p < 0x1p1000;
  bool pass = false;
  if (!(ok && m < p * (1.0 - 0x1p-40))) {  // not a certain failure
    pass = ok && m > p * (1.0 + 0x1p-40);
    if (!pass) pass = m / r2 > t;
  }
  return pass;
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

// One workgroup per group of kPertGroup consecutive entries (grid-stride),
// taken cluster by cluster (entries are cluster-major, so a group meets few
// clusters); each wavefront holds kPertGroup / 4 of them.  The cluster's
// id-ordered j-data pass through LDS in rounds of kPertRound ids, read by
// every wavefront of the group.  Lane l reads ids u * 64 + l of the round
// (consecutive lanes, consecutive LDS words) and tests each against all of
// its wavefront's entries; a ballot per id and entry places the passing ids
// in ascending order.
__global__ void __launch_bounds__(kPertThreads)
perturbers_kernel(DevState s, const int32_t* __restrict__ ids, const int64_t* __restrict__ aoff, int64_t n_active,
                  const double* __restrict__ thr, int32_t cap, int32_t* __restrict__ lists,
                  int32_t* __restrict__ counts) {
  constexpr int kWaves = kPertThreads / 64;
  constexpr int kPerWave = kPertGroup / kWaves;
  __shared__ double tX[kPertRound], tY[kPertRound], tZ[kPertRound], tM[kPertRound];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t n = s.n;
  const double* X = s.pid;
  const double* Y = s.pid + n;
  const double* Z = s.pid + 2 * n;
  const double* M = s.pid + 3 * n;
  for (int64_t g0 = (int64_t)blockIdx.x * kPertGroup; g0 < n_active; g0 += (int64_t)gridDim.x * kPertGroup) {
    const int64_t g1 = g0 + kPertGroup < n_active ? g0 + kPertGroup : n_active;
    for (int64_t qs = g0; qs < g1;) {  // the clusters met by the group, in order (uniform)
      int lo = 0, hi = s.nc - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (aoff[mid] <= qs) lo = mid; else hi = mid - 1;
      }
      const int c = lo;
      const int64_t b = s.coff[c], e = s.coff[c + 1];
      const int64_t qe = aoff[c + 1] < g1 ? aoff[c + 1] : g1;
      if (qe <= qs) {
        // offsets that end before n_active or do not ascend: the rest of the
        // group belongs to no cluster; reported, empty lists, loop ends
        for (int64_t r = qs * cap + tid; r < g1 * cap; r += kPertThreads) lists[r] = -1;
        for (int64_t r = qs + tid; r < g1; r += kPertThreads) counts[r] = 0;
        if (tid == 0)
          __hip_atomic_fetch_or(s.status, (int32_t)ST_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      const double eps2 = s.eps[c] * s.eps[c];
      const double t = thr[c];
      const bool t_ok = t > 0x1p-1000 && t < 0x1p1000;
      // this wavefront's entries of the cluster
      int64_t q[kPerWave], id[kPerWave];
      bool on[kPerWave];
      double xi[kPerWave], yi[kPerWave], zi[kPerWave];
      int32_t found[kPerWave];
#pragma unroll
      for (int k = 0; k < kPerWave; ++k) {
        q[k] = qs + wave * kPerWave + k;
        id[k] = -1;
        on[k] = false;
        xi[k] = yi[k] = zi[k] = 0.0;
        found[k] = 0;
        if (q[k] < qe) {
          id[k] = ids[q[k]];
          on[k] = id[k] >= b && id[k] < e;
          if (on[k]) {
            xi[k] = X[id[k]];
            yi[k] = Y[id[k]];
            zi[k] = Z[id[k]];
          } else if (lane == 0) {
            __hip_atomic_fetch_or(s.status, (int32_t)ST_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      for (int64_t j0 = b; j0 < e; j0 += kPertRound) {
        __syncthreads();  // the previous round is consumed
        for (int k = tid; k < kPertRound; k += kPertThreads) {
          const int64_t j = j0 + k;
          const bool in = j < e;
          tX[k] = in ? X[j] : 0.0;
          tY[k] = in ? Y[j] : 0.0;
          tZ[k] = in ? Z[j] : 0.0;
          tM[k] = in ? M[j] : 0.0;
        }
        __syncthreads();
        for (int u = 0; u < kPertRound / 64; ++u) {
          // each LDS record is read once and tested against every entry of
          // the wavefront
          const int l = u * 64 + lane;
          const int64_t j = j0 + l;
          const double xj = tX[l], yj = tY[l], zj = tZ[l], mj = tM[l];
          // the tests of all entries first (padding past the cluster and the
          // entry itself may give inf or NaN there; the conditions drop
          // them); a division runs only for the rare pair whose outcome the
          // product test leaves open
          bool pass[kPerWave];
#pragma unroll
          for (int k = 0; k < kPerWave; ++k) {
            const double r2 = softened_r2(xj - xi[k], yj - yi[k], zj - zi[k], eps2);
            pass[k] = on[k] & (j < e) & (j != id[k]) & above_threshold(mj, r2, t, t_ok);
          }
          // most ids pass for none of the wavefront's entries: one ballot
          // over all of them skips the per-entry placement (every entry's
          // mask would be empty)
          bool any_pass = false;
#pragma unroll
          for (int k = 0; k < kPerWave; ++k) any_pass |= pass[k];
          if (__ballot(any_pass) == 0) continue;
#pragma unroll
          for (int k = 0; k < kPerWave; ++k) {
            if (!on[k]) continue;  // uniform within the wavefront
            const uint64_t mask = __ballot(pass[k]);
            const int at = found[k] + __popcll(mask & below);
            if (pass[k] && at < cap) lists[q[k] * cap + at] = (int32_t)j;
            found[k] += __popcll(mask);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kPerWave; ++k) {
        if (q[k] < qe) {
          for (int m = (found[k] < cap ? found[k] : cap) + lane; m < cap; m += 64) lists[q[k] * cap + m] = -1;
          if (lane == 0) counts[q[k]] = found[k];
        }
      }
      qs = qe;
    }
  }
}

}  // namespace

hipError_t launch_perturbers(const DevState& s, const int32_t* ids, const int64_t* aoff, int64_t n_active,
                             const double* thr, int32_t cap, int32_t* lists, int32_t* counts, hipStream_t st) {
  const int64_t sg = (s.n + 255) / 256;
  hipLaunchKernelGGL(stage_by_id_kernel, dim3((unsigned)(sg < 65536 ? sg : 65536)), dim3(256), 0, st, s);
  const int64_t wgs = (n_active + kPertGroup - 1) / kPertGroup;
  const int64_t grid = wgs < 65536 ? wgs : 65536;
  hipLaunchKernelGGL(perturbers_kernel, dim3((unsigned)grid), dim3(kPertThreads), 0, st, s, ids, aoff, n_active, thr,
                     cap, lists, counts);
  return hipGetLastError();
}

}  // namespace nb
