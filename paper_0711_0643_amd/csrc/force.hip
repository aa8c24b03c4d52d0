// Pairwise acceleration, jerk and potential on the active block
// (Sect. 2.1, Eq. Force; jerk and potential by direct summation).
//
// One launch processes every work item of the current plan.  A work item is
// (cluster c, i-chunk, j-slice): up to 256/JL active particles of c against
// one contiguous slice of c's particles.  The workgroup stages the slice in
// LDS tiles of kTile j-records (coalesced SoA reads from HBM), and every
// wavefront sweeps each tile: with JL = 1 all 64 lanes of a wave read the same
// record (an LDS broadcast) and each lane owns one i; with JL > 1 the j's of a
// tile are further split over JL lanes per i and the lane partials are
// combined in LDS in a fixed order.  Each item writes FP64 partial sums to
// its own rows; slices are added later in slice order, so results do not
// depend on scheduling (the paper's j-parallel partition, Sect. 3, carried
// out across lanes and workgroups of one GPU).
//
// Arithmetic modes:
//   kF64  : everything in FP64; 1/sqrt from v_rsq_f64 plus one third-order
//           Newton step.
//   kDS   : positions as FP32 hi/lo pairs, differenced as
//           (hi_j - hi_i) + (lo_j - lo_i); pair terms in FP32; partial sums
//           over windows of at most 32 j in FP32, then added to FP64 totals.
//   kMX64 : as kDS but the position difference is formed in FP64 from the
//           predicted FP64 positions and rounded once to FP32.
// The self pair (j == i) and the zero padding of a ragged last tile are
// removed by zeroing 1/R, only on tiles where a lane's own i or the padding
// can occur (a wave-uniform test), so full tiles run unmasked.
#include "common.h"
#include "kernels.h"

namespace nb {

struct alignas(16) RecF64 {
  double x, y, z, m, vx, vy, vz, pad;
};
struct alignas(16) RecDS {
  float hx, hy, hz, m, lx, ly, lz, p0, vx, vy, vz, p1;
};
struct alignas(16) RecMX {
  double x, y, z;
  float m, vx, vy, vz;
};

template <int MODE> struct ModeT;
template <> struct ModeT<kF64> {
  using Rec = RecF64;
  struct I { double x, y, z, vx, vy, vz; };
};
template <> struct ModeT<kDS> {
  using Rec = RecDS;
  struct I { float hx, hy, hz, lx, ly, lz, vx, vy, vz; };
};
template <> struct ModeT<kMX64> {
  using Rec = RecMX;
  struct I { double x, y, z; float vx, vy, vz; };
};

constexpr int kLdsBytes = kTile * 64;  // the largest record is 64 B
static_assert(kForceThreads * 7 * 8 <= kLdsBytes, "reduction buffer must fit the tile buffer");

template <int MODE>
__device__ __forceinline__ typename ModeT<MODE>::Rec load_rec(const DevState& s, int64_t j) {
  const int64_t n = s.n;
  typename ModeT<MODE>::Rec r;
  if constexpr (MODE == kF64) {
    r.x = s.xp[j]; r.y = s.xp[n + j]; r.z = s.xp[2 * n + j];
    r.m = s.m[j];
    r.vx = s.vp[j]; r.vy = s.vp[n + j]; r.vz = s.vp[2 * n + j];
    r.pad = 0.0;
  } else if constexpr (MODE == kDS) {
    const float* jr = s.jr;
    r.hx = jr[JR_HX * n + j]; r.hy = jr[JR_HY * n + j]; r.hz = jr[JR_HZ * n + j];
    r.m = jr[JR_M * n + j];
    r.lx = jr[JR_LX * n + j]; r.ly = jr[JR_LY * n + j]; r.lz = jr[JR_LZ * n + j];
    r.p0 = 0.f;
    r.vx = jr[JR_VX * n + j]; r.vy = jr[JR_VY * n + j]; r.vz = jr[JR_VZ * n + j];
    r.p1 = 0.f;
  } else {
    const float* jr = s.jr;
    r.x = s.xp[j]; r.y = s.xp[n + j]; r.z = s.xp[2 * n + j];
    r.m = jr[JR_M * n + j];
    r.vx = jr[JR_VX * n + j]; r.vy = jr[JR_VY * n + j]; r.vz = jr[JR_VZ * n + j];
  }
  return r;
}

template <int MODE>
__device__ __forceinline__ typename ModeT<MODE>::Rec zero_rec() {
  typename ModeT<MODE>::Rec r;
  __builtin_memset(&r, 0, sizeof(r));
  return r;
}

template <int MODE>
__device__ __forceinline__ typename ModeT<MODE>::I load_i(const DevState& s, int64_t i) {
  const int64_t n = s.n;
  typename ModeT<MODE>::I d;
  if constexpr (MODE == kF64) {
    d.x = s.xp[i]; d.y = s.xp[n + i]; d.z = s.xp[2 * n + i];
    d.vx = s.vp[i]; d.vy = s.vp[n + i]; d.vz = s.vp[2 * n + i];
  } else if constexpr (MODE == kDS) {
    const float* jr = s.jr;
    d.hx = jr[JR_HX * n + i]; d.hy = jr[JR_HY * n + i]; d.hz = jr[JR_HZ * n + i];
    d.lx = jr[JR_LX * n + i]; d.ly = jr[JR_LY * n + i]; d.lz = jr[JR_LZ * n + i];
    d.vx = jr[JR_VX * n + i]; d.vy = jr[JR_VY * n + i]; d.vz = jr[JR_VZ * n + i];
  } else {
    const float* jr = s.jr;
    d.x = s.xp[i]; d.y = s.xp[n + i]; d.z = s.xp[2 * n + i];
    d.vx = jr[JR_VX * n + i]; d.vy = jr[JR_VY * n + i]; d.vz = jr[JR_VZ * n + i];
  }
  return d;
}

// 1/sqrt(r2) in FP64: hardware estimate, then y <- y + y e (1/2 + 3e/8) with
// e = 1 - r2 y^2 (third-order Newton-type step for r2^(-1/2)).
__device__ __forceinline__ double rsqrt_f64(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  const double t = r2 * y;
  const double e = __builtin_fma(-t, y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(0.375, e, 0.5), y);
}

// Accumulators: FP64 totals plus (mixed modes) an FP32 window.
struct Acc64 { double v[7]; };
struct Acc32 { float v[7]; };

// One pair interaction in FP64, added straight into the totals.
template <bool MASK>
__device__ __forceinline__ void pair_f64(const ModeT<kF64>::I& I, const RecF64& J, double eps2,
                                         bool drop, Acc64& A) {
  const double dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
  const double dvx = J.vx - I.vx, dvy = J.vy - I.vy, dvz = J.vz - I.vz;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
  double rinv = rsqrt_f64(r2);
  if (MASK) rinv = drop ? 0.0 : rinv;
  const double rinv2 = rinv * rinv;
  const double mr = J.m * rinv;
  const double mr3 = mr * rinv2;
  const double rv = __builtin_fma(dz, dvz, __builtin_fma(dy, dvy, dx * dvx));
  const double al = (-3.0 * rinv2) * rv;
  A.v[0] = __builtin_fma(mr3, dx, A.v[0]);
  A.v[1] = __builtin_fma(mr3, dy, A.v[1]);
  A.v[2] = __builtin_fma(mr3, dz, A.v[2]);
  A.v[3] = __builtin_fma(mr3, __builtin_fma(al, dx, dvx), A.v[3]);
  A.v[4] = __builtin_fma(mr3, __builtin_fma(al, dy, dvy), A.v[4]);
  A.v[5] = __builtin_fma(mr3, __builtin_fma(al, dz, dvz), A.v[5]);
  A.v[6] -= mr;
}

// The FP32 part shared by the mixed modes, given the FP32 differences.
template <bool MASK>
__device__ __forceinline__ void pair_f32(float dx, float dy, float dz, float dvx, float dvy,
                                         float dvz, float m, float eps2, bool drop, Acc32& A) {
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
  float rinv = __builtin_amdgcn_rsqf(r2);
  if (MASK) rinv = drop ? 0.f : rinv;
  const float rinv2 = rinv * rinv;
  const float mr = m * rinv;
  const float mr3 = mr * rinv2;
  const float rv = __builtin_fmaf(dz, dvz, __builtin_fmaf(dy, dvy, dx * dvx));
  const float al = (-3.f * rinv2) * rv;
  A.v[0] = __builtin_fmaf(mr3, dx, A.v[0]);
  A.v[1] = __builtin_fmaf(mr3, dy, A.v[1]);
  A.v[2] = __builtin_fmaf(mr3, dz, A.v[2]);
  A.v[3] = __builtin_fmaf(mr3, __builtin_fmaf(al, dx, dvx), A.v[3]);
  A.v[4] = __builtin_fmaf(mr3, __builtin_fmaf(al, dy, dvy), A.v[4]);
  A.v[5] = __builtin_fmaf(mr3, __builtin_fmaf(al, dz, dvz), A.v[5]);
  A.v[6] -= mr;
}

template <bool MASK>
__device__ __forceinline__ void pair_ds(const ModeT<kDS>::I& I, const RecDS& J, float eps2, bool drop,
                                        Acc32& A) {
  const float dx = (J.hx - I.hx) + (J.lx - I.lx);
  const float dy = (J.hy - I.hy) + (J.ly - I.ly);
  const float dz = (J.hz - I.hz) + (J.lz - I.lz);
  pair_f32<MASK>(dx, dy, dz, J.vx - I.vx, J.vy - I.vy, J.vz - I.vz, J.m, eps2, drop, A);
}

template <bool MASK>
__device__ __forceinline__ void pair_mx(const ModeT<kMX64>::I& I, const RecMX& J, float eps2, bool drop,
                                        Acc32& A) {
  const float dx = (float)(J.x - I.x);
  const float dy = (float)(J.y - I.y);
  const float dz = (float)(J.z - I.z);
  pair_f32<MASK>(dx, dy, dz, J.vx - I.vx, J.vy - I.vy, J.vz - I.vz, J.m, eps2, drop, A);
}

// Sweep this lane's share of one LDS tile.  jl0: first tile-local j of the
// lane; PER: j per lane per tile; the global index of tile entry u is
// tile_j0 + u.  MASK drops the lane's own i and entries at or past j_end.
template <int MODE, int PER, bool MASK>
__device__ __forceinline__ void sweep_tile(const typename ModeT<MODE>::Rec* tile, int jl0,
                                           int64_t tile_j0, int64_t j_end, int64_t i_glob,
                                           const typename ModeT<MODE>::I& I, double eps2d, float eps2f,
                                           Acc64& A) {
  if constexpr (MODE == kF64) {
#pragma unroll 8
    for (int u = 0; u < PER; ++u) {
      const int jl = jl0 + u;
      const int64_t jg = tile_j0 + jl;
      const bool drop = MASK && (jg == i_glob || jg >= j_end);
      pair_f64<MASK>(I, tile[jl], eps2d, drop, A);
    }
  } else {
    constexpr int F = PER < 32 ? PER : 32;  // FP32 window, then flush to FP64
    for (int w = 0; w < PER; w += F) {
      Acc32 B;
#pragma unroll
      for (int d = 0; d < 7; ++d) B.v[d] = 0.f;
#pragma unroll
      for (int u = 0; u < F; ++u) {
        const int jl = jl0 + w + u;
        const int64_t jg = tile_j0 + jl;
        const bool drop = MASK && (jg == i_glob || jg >= j_end);
        if constexpr (MODE == kDS)
          pair_ds<MASK>(I, tile[jl], eps2f, drop, B);
        else
          pair_mx<MASK>(I, tile[jl], eps2f, drop, B);
      }
#pragma unroll
      for (int d = 0; d < 7; ++d) A.v[d] += (double)B.v[d];
    }
  }
}

// Locate the cluster that owns work item `item` (plans are ordered by
// cluster; item_off is ascending).
__device__ __forceinline__ int find_cluster(const Plan* plan, int nc, int64_t item) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plan[mid].item_off <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int MODE, int JL>
__device__ void run_item(const DevState& s, const int32_t* __restrict__ act, const Plan& P, int c,
                         int64_t local_item, unsigned char* lds) {
  constexpr int IWG = kForceThreads / JL;
  constexpr int PER = kTile / JL;
  using Rec = typename ModeT<MODE>::Rec;
  using IT = typename ModeT<MODE>::I;
  Rec* tile = reinterpret_cast<Rec*>(lds);

  const int tid = threadIdx.x;
  const int il = tid % IWG;
  const int jl = tid / IWG;
  const int chunk = (int)(local_item / P.slices);
  const int slice = (int)(local_item % P.slices);
  const int64_t c_begin = s.coff[c], c_end = s.coff[c + 1];
  const int q_local = chunk * IWG + il;  // entry of the cluster's active list
  const bool listed = q_local < P.n_act;
  bool valid = listed;
  int64_t i_glob = c_begin;
  if (valid) {
    i_glob = act[P.act_off + q_local];
    if (i_glob < c_begin || i_glob >= c_end) {
      __hip_atomic_fetch_or(s.status, (int32_t)ST_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      valid = false;
      i_glob = c_begin;
    }
  }
  const IT I = load_i<MODE>(s, i_glob);
  const double eps = s.eps[c];
  const double eps2d = eps * eps;
  const float eps2f = (float)eps2d;

  Acc64 A;
#pragma unroll
  for (int d = 0; d < 7; ++d) A.v[d] = 0.0;

  const int64_t j_begin = c_begin + (int64_t)slice * P.slice_len;
  int64_t j_end = j_begin + P.slice_len;
  if (j_end > c_end) j_end = c_end;

  for (int64_t j0 = j_begin; j0 < j_end; j0 += kTile) {
    __syncthreads();  // previous tile fully consumed
    for (int r = tid; r < kTile; r += kForceThreads) {
      const int64_t j = j0 + r;
      tile[r] = (j < j_end) ? load_rec<MODE>(s, j) : zero_rec<MODE>();
    }
    __syncthreads();
    const bool mine = valid && i_glob >= j0 && i_glob < j0 + kTile;
    const bool need_mask = (j0 + kTile > j_end) || __any(mine);
    if (need_mask)
      sweep_tile<MODE, PER, true>(tile, jl * PER, j0, j_end, i_glob, I, eps2d, eps2f, A);
    else
      sweep_tile<MODE, PER, false>(tile, jl * PER, j0, j_end, i_glob, I, eps2d, eps2f, A);
  }

  const int64_t rows_cap = s.rows_cap;
  const int64_t row0 = P.slot_base + (int64_t)slice * P.n_act;
  if (!valid) {  // unlisted lane, or an index outside its cluster: contributes zeros
#pragma unroll
    for (int d = 0; d < 7; ++d) A.v[d] = 0.0;
  }
  if constexpr (JL == 1) {
    if (listed) {
#pragma unroll
      for (int d = 0; d < 7; ++d) s.part[d * rows_cap + row0 + q_local] = A.v[d];
    }
  } else {
    // combine the JL lane partials of each i in ascending lane order
    __syncthreads();
    double* red = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int d = 0; d < 7; ++d) red[(d * JL + jl) * IWG + il] = A.v[d];
    __syncthreads();
    if (tid < IWG) {
      const int q2 = chunk * IWG + tid;
      if (q2 < P.n_act) {
#pragma unroll
        for (int d = 0; d < 7; ++d) {
          double sum = 0.0;
          for (int l = 0; l < JL; ++l) sum += red[(d * JL + l) * IWG + tid];
          s.part[d * rows_cap + row0 + q2] = sum;
        }
      }
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(kForceThreads) force_kernel(DevState s, const int32_t* __restrict__ act) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  const int64_t total = s.ctl->total_items;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int c = find_cluster(s.plan, s.nc, item);
    const Plan P = s.plan[c];
    const int64_t local = item - P.item_off;
    switch (P.variant) {
      case 0: run_item<MODE, 1>(s, act, P, c, local, lds); break;
      case 1: run_item<MODE, 4>(s, act, P, c, local, lds); break;
      case 2: run_item<MODE, 16>(s, act, P, c, local, lds); break;
      default: run_item<MODE, 64>(s, act, P, c, local, lds); break;
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

hipError_t launch_force(const DevState& s, int mode, const int32_t* act, int grid, hipStream_t st) {
  switch (mode) {
    case kF64: hipLaunchKernelGGL(force_kernel<kF64>, dim3(grid), dim3(kForceThreads), 0, st, s, act); break;
    case kDS: hipLaunchKernelGGL(force_kernel<kDS>, dim3(grid), dim3(kForceThreads), 0, st, s, act); break;
    default: hipLaunchKernelGGL(force_kernel<kMX64>, dim3(grid), dim3(kForceThreads), 0, st, s, act); break;
  }
  return hipGetLastError();
}

}  // namespace nb
