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
//           The hardware 1/sqrt (v_rsq_f32) is accurate to < 1 ulp but its
//           error has a small nonzero mean; summed over N terms that mean
//           does not average out, and where the pair terms cancel (|a| much
//           smaller than the sum of |terms|) it dominates the error.  The
//           library measures that mean relative error b once on the device
//           (rsq_bias_kernel) and the FP64 flush multiplies the window by
//           (1 - 3b) for the R^-3 terms and (1 - b) for the potential.
//   kMX64 : as kDS but the position difference is formed in FP64 from the
//           predicted FP64 positions and rounded once to FP32.
//   kTR   : tile-relative FP32 (layouts with one lane per i; the j-split
//           layouts of small blocks form the position difference in FP64
//           from the tile's FP64 copy instead).  Slots are sorted along a Morton curve, so
//           the kTile j of a tile are close in space; the predictor records
//           each tile's frame (bounding-box centres of the predicted
//           positions and velocities).  The tile loader converts every j to
//           FP32 coordinates relative to that frame (one FP64 subtraction
//           per j and workgroup), each lane converts its i once per tile,
//           and the pair difference is a single FP32 subtraction.  Its
//           error, u (|x_i - o| + |x_j - o|), is that of a few ulps of the
//           pair distance except for pairs much closer than the tile's
//           size; those are the pairs the near test below sends to FP64.
// The self pair (j == i) and the zero padding of a ragged last tile are
// removed by zeroing 1/R, only on tiles where a lane's own i or the padding
// can occur (a wave-uniform test), so full tiles run unmasked.
//
// Near pairs (mixed modes).  One FP32 pair term carries a few u = 2^-24 of
// relative error, which limits the relative error of a sum only when the
// term is small against the sum.  No pair stays in FP32 when its
// acceleration term may exceed near_tau |a_i| or its jerk term may exceed
// near_tau_k |k_i| (|a_i|, |k_i| from the last step).  A jerk term is at
// most 2 m_j |v_j - v_i| / R^3 (the matrix I - 3 r r^T / R^2 has norm 2),
// and |v_j - v_i| <= |v_i - v_c| + W for the tile's velocity centre v_c and
// radius W.
#pragma once

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
// kTR: FP32 position and velocity relative to the tile frame, FP32 mass.
struct alignas(16) RecTR {
  float x, y, z, m, vx, vy, vz, p0;
};
// kTR: the FP64 predicted state of a tile entry, for its near pairs.
struct RecP64 {
  double x, y, z, vx, vy, vz;
};
struct NoI64 {};

template <int MODE> struct ModeT;
// Rec: the LDS record of one j; I: what a lane keeps of one i for the pair
// arithmetic; I64 (kTR): the i's FP64 predicted state, from which I is
// formed anew for every tile.
template <> struct ModeT<kF64> {
  using Rec = RecF64;
  struct I { double x, y, z, vx, vy, vz; };
  using I64 = NoI64;
};
template <> struct ModeT<kDS> {
  using Rec = RecDS;
  struct I { float hx, hy, hz, lx, ly, lz, vx, vy, vz; };
  using I64 = NoI64;
};
template <> struct ModeT<kMX64> {
  using Rec = RecMX;
  struct I { double x, y, z; float vx, vy, vz; };
  using I64 = NoI64;
};
template <> struct ModeT<kTR> {
  using Rec = RecTR;
  struct I { float x, y, z, vx, vy, vz; };
  using I64 = RecP64;
};

// LDS per workgroup: one tile of records (at most 64 B each), or for kTR
// the 32 B records followed by their 48 B FP64 copies.
constexpr int kLdsBytes = kTile * 80;
static_assert(kTile * (sizeof(RecTR) + sizeof(RecP64)) <= kLdsBytes, "kTR tile must fit");
static_assert(kTile * sizeof(RecF64) <= kLdsBytes, "FP64 tile must fit");
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
    static_assert(MODE == kMX64, "kTR records are formed by the tile loader");
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
  } else if constexpr (MODE == kMX64) {
    const float* jr = s.jr;
    d.x = s.xp[i]; d.y = s.xp[n + i]; d.z = s.xp[2 * n + i];
    d.vx = jr[JR_VX * n + i]; d.vy = jr[JR_VY * n + i]; d.vz = jr[JR_VZ * n + i];
  } else {
    d.x = d.y = d.z = d.vx = d.vy = d.vz = 0.f;  // formed per tile from the FP64 state
  }
  return d;
}

__device__ __forceinline__ RecP64 load_p64(const DevState& s, int64_t i) {
  const int64_t n = s.n;
  RecP64 r;
  r.x = s.xp[i]; r.y = s.xp[n + i]; r.z = s.xp[2 * n + i];
  r.vx = s.vp[i]; r.vy = s.vp[n + i]; r.vz = s.vp[2 * n + i];
  return r;
}

// FP64 j-record of the fused predictor: particle j predicted to tp from its
// state, with the arithmetic of the selection's predictor.
__device__ __forceinline__ RecF64 predict_rec(const DevState& s, int64_t j, double tp) {
  const int64_t n = s.n;
  const double h = tp - s.t[j];
  double p[3], q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t o = d * n + j;
    hermite_predict(s.x[o], s.v[o], s.a[o], s.k[o], h, p[d], q[d]);
  }
  RecF64 r;
  r.x = p[0]; r.y = p[1]; r.z = p[2];
  r.m = s.m[j];
  r.vx = q[0]; r.vy = q[1]; r.vz = q[2];
  r.pad = 0.0;
  return r;
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
template <bool MASK, bool POT>
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
  if (POT) A.v[6] -= mr;
}

// FP32 differences of one pair (mixed modes) and R^2.
struct Diff32 { float dx, dy, dz, dvx, dvy, dvz, r2; };

template <int MODE>
__device__ __forceinline__ Diff32 diff32(const typename ModeT<MODE>::I& I, const typename ModeT<MODE>::Rec& J,
                                         float eps2) {
  Diff32 d;
  if constexpr (MODE == kDS) {
    d.dx = (J.hx - I.hx) + (J.lx - I.lx);
    d.dy = (J.hy - I.hy) + (J.ly - I.ly);
    d.dz = (J.hz - I.hz) + (J.lz - I.lz);
  } else if constexpr (MODE == kTR) {
    d.dx = J.x - I.x;
    d.dy = J.y - I.y;
    d.dz = J.z - I.z;
  } else {
    d.dx = (float)(J.x - I.x);
    d.dy = (float)(J.y - I.y);
    d.dz = (float)(J.z - I.z);
  }
  d.dvx = J.vx - I.vx;
  d.dvy = J.vy - I.vy;
  d.dvz = J.vz - I.vz;
  d.r2 = __builtin_fmaf(d.dz, d.dz, __builtin_fmaf(d.dy, d.dy, __builtin_fmaf(d.dx, d.dx, eps2)));
  return d;
}

// kTR in the layouts that split j over lanes (small blocks, often small
// clusters, where a tile spans much of the cluster): the position
// difference is formed in FP64 from the tile's FP64 copy and the i's FP64
// position and rounded once; velocities stay tile-relative FP32.
__device__ __forceinline__ Diff32 diff32_tr64(const RecTR& J, const RecP64& Jp, const ModeT<kTR>::I& I,
                                              const double* xi, float eps2f) {
  Diff32 d;
  d.dx = (float)(Jp.x - xi[0]);
  d.dy = (float)(Jp.y - xi[1]);
  d.dz = (float)(Jp.z - xi[2]);
  d.dvx = J.vx - I.vx;
  d.dvy = J.vy - I.vy;
  d.dvz = J.vz - I.vz;
  d.r2 = __builtin_fmaf(d.dz, d.dz, __builtin_fmaf(d.dy, d.dy, __builtin_fmaf(d.dx, d.dx, eps2f)));
  return d;
}

// Weight of an FP32 pair in the per-pair near scheme: 1 when its term
// (t = m_j / R^2 for the acceleration, m_j / R^3 for the jerk) is below the
// per-i threshold g, 0 above it (the pair then goes to FP64).  Branch-free:
// (g - t) * 2^40 clamped to [0, 1], one FMA from gB = g * 2^40 and a clamp,
// so the first pass and the FP64 re-scan get the same weight bit for bit;
// the re-scan adds (1 - weight) of the pair in FP64, so the split is exact
// even in the (measure-zero) fractional case.
constexpr float kNearScale = 1099511627776.0f;  // 2^40

__device__ __forceinline__ float near_weight(float t, float gB) {
  return __builtin_amdgcn_fmed3f(__builtin_fmaf(-t, kNearScale, gB), 0.f, 1.f);
}

// Near weight of a pair from its m_j / R^2 (t) and m_j / R^3 (t3): the
// acceleration threshold gB and the jerk threshold gkB (both times 2^40).
__device__ __forceinline__ float near_weight2(float t, float t3, float gB, float gkB) {
  return fminf(near_weight(t, gB), near_weight(t3, gkB));
}

// The rest of an FP32 pair, accumulated into the FP32 window.  ZERO: drop
// the pair when `drop` is set.  WEIGHT: scale it by its near weight and keep
// the smallest weight of the window in *wmin.
template <bool ZERO, bool POT, bool WEIGHT>
__device__ __forceinline__ void finish_f32(const Diff32& d, float m, bool drop, float gB, float gkB, float* wmin,
                                           Acc32& A) {
  float rinv = __builtin_amdgcn_rsqf(d.r2);
  if (ZERO) rinv = drop ? 0.f : rinv;
  const float rinv2 = rinv * rinv;
  float mr, mr3;
  if (WEIGHT) {
    const float t = m * rinv2;  // m_j / R^2
    const float t3 = t * rinv;  // m_j / R^3
    const float w = near_weight2(t, t3, gB, gkB);
    *wmin = fminf(*wmin, w);
    mr3 = t3 * w;
    mr = POT ? m * rinv * w : 0.f;
  } else {
    mr = m * rinv;
    mr3 = mr * rinv2;
  }
  const float rv = __builtin_fmaf(d.dz, d.dvz, __builtin_fmaf(d.dy, d.dvy, d.dx * d.dvx));
  const float al = (-3.f * rinv2) * rv;
  A.v[0] = __builtin_fmaf(mr3, d.dx, A.v[0]);
  A.v[1] = __builtin_fmaf(mr3, d.dy, A.v[1]);
  A.v[2] = __builtin_fmaf(mr3, d.dz, A.v[2]);
  A.v[3] = __builtin_fmaf(mr3, __builtin_fmaf(al, d.dx, d.dvx), A.v[3]);
  A.v[4] = __builtin_fmaf(mr3, __builtin_fmaf(al, d.dy, d.dvy), A.v[4]);
  A.v[5] = __builtin_fmaf(mr3, __builtin_fmaf(al, d.dz, d.dvz), A.v[5]);
  if (POT) A.v[6] -= mr;
}

// Near weight of a pair recomputed for the FP64 re-scan, with exactly the
// operations of the first pass.
__device__ __forceinline__ float near_weight_again(const Diff32& d, float m, float gB, float gkB) {
  const float rinv = __builtin_amdgcn_rsqf(d.r2);
  const float t = m * (rinv * rinv);
  return near_weight2(t, t * rinv, gB, gkB);
}

// A pair of a mixed mode evaluated in FP64 from the same record: the
// double-single position hi + lo is exact in FP64, velocities and mass are
// the record's FP32 values widened.  Added straight into the FP64 totals.
template <int MODE, bool POT>
__device__ __forceinline__ void pair_mixed64(const typename ModeT<MODE>::I& I, const typename ModeT<MODE>::Rec& J,
                                             double eps2, double share, Acc64& A) {
  double dx, dy, dz;
  if constexpr (MODE == kDS) {
    dx = ((double)J.hx + (double)J.lx) - ((double)I.hx + (double)I.lx);
    dy = ((double)J.hy + (double)J.ly) - ((double)I.hy + (double)I.ly);
    dz = ((double)J.hz + (double)J.lz) - ((double)I.hz + (double)I.lz);
  } else {
    dx = J.x - I.x;
    dy = J.y - I.y;
    dz = J.z - I.z;
  }
  const double dvx = (double)J.vx - (double)I.vx;
  const double dvy = (double)J.vy - (double)I.vy;
  const double dvz = (double)J.vz - (double)I.vz;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
  const double rinv = rsqrt_f64(r2);
  const double rinv2 = rinv * rinv;
  const double mr = share * (double)J.m * rinv;
  const double mr3 = mr * rinv2;
  const double rv = __builtin_fma(dz, dvz, __builtin_fma(dy, dvy, dx * dvx));
  const double al = (-3.0 * rinv2) * rv;
  A.v[0] = __builtin_fma(mr3, dx, A.v[0]);
  A.v[1] = __builtin_fma(mr3, dy, A.v[1]);
  A.v[2] = __builtin_fma(mr3, dz, A.v[2]);
  A.v[3] = __builtin_fma(mr3, __builtin_fma(al, dx, dvx), A.v[3]);
  A.v[4] = __builtin_fma(mr3, __builtin_fma(al, dy, dvy), A.v[4]);
  A.v[5] = __builtin_fma(mr3, __builtin_fma(al, dz, dvz), A.v[5]);
  if (POT) A.v[6] -= mr;
}

// A kTR pair in FP64 from the FP64 predicted states (the mass is the
// record's FP32 value widened), added straight into the FP64 totals.
template <bool POT>
__device__ __forceinline__ void pair_tr64(const RecP64& Fi, const RecP64& Fj, float m, double eps2, double share,
                                          Acc64& A) {
  const double dx = Fj.x - Fi.x, dy = Fj.y - Fi.y, dz = Fj.z - Fi.z;
  const double dvx = Fj.vx - Fi.vx, dvy = Fj.vy - Fi.vy, dvz = Fj.vz - Fi.vz;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
  const double rinv = rsqrt_f64(r2);
  const double rinv2 = rinv * rinv;
  const double mr = share * (double)m * rinv;
  const double mr3 = mr * rinv2;
  const double rv = __builtin_fma(dz, dvz, __builtin_fma(dy, dvy, dx * dvx));
  const double al = (-3.0 * rinv2) * rv;
  A.v[0] = __builtin_fma(mr3, dx, A.v[0]);
  A.v[1] = __builtin_fma(mr3, dy, A.v[1]);
  A.v[2] = __builtin_fma(mr3, dz, A.v[2]);
  A.v[3] = __builtin_fma(mr3, __builtin_fma(al, dx, dvx), A.v[3]);
  A.v[4] = __builtin_fma(mr3, __builtin_fma(al, dy, dvy), A.v[4]);
  A.v[5] = __builtin_fma(mr3, __builtin_fma(al, dz, dvz), A.v[5]);
  if (POT) A.v[6] -= mr;
}

// FP64 pass over the near windows of one tile, after the FP32 sweep (the
// tile is still in LDS).  Bit p * NW + k of `flags` marks window k (F
// entries from jl0 + k F) of i-particle p.  WIN (window test): the window's
// FP32 sum was left out, so every pair of it except the dropped ones (own j,
// padding) is added in FP64.  Otherwise (per-pair weights): each pair whose
// near weight w is below 1 adds (1 - w) of its FP64 value; w is recomputed
// with exactly the operations of the FP32 pass.  Each lane walks its own
// windows in ascending order, so the sums do not depend on the other lanes.
// Kept inline (no call, whose register saves would go through scratch
// memory) and unrolled by 4 so that the LDS reads of consecutive pairs
// overlap: at this point the FP32 window state is dead, so the FP64
// temporaries fit beside the totals.
template <int MODE, int F, int NW, int IPT, bool POT, bool WIN>
__device__ __forceinline__ void near_windows_f64(const DevState& s, const typename ModeT<MODE>::Rec* tile,
                                                 const RecP64* tile64, int jl0, const int* own, int jend,
                                                 const int64_t* i_glob, const typename ModeT<MODE>::I* I,
                                                 const float* gB, const float* gkB, double eps2d, float eps2f,
                                                 uint32_t flags, Acc64* A) {
#pragma unroll
  for (int p = 0; p < IPT; ++p) {
    uint32_t f = (flags >> (p * NW)) & ((1u << NW) - 1u);
    RecP64 Fi{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == kTR) {
      if (f) Fi = load_p64(s, i_glob[p]);  // the i's FP64 state (rarely needed: not kept in registers)
    }
    while (f) {
      const int jw = jl0 + __builtin_ctz(f) * F;
      f &= f - 1u;
#pragma unroll 4
      for (int u = 0; u < F; ++u) {
        const int jl = jw + u;
        if (jl == own[p] || jl >= jend) continue;
        const typename ModeT<MODE>::Rec J = tile[jl];
        double share = 1.0;
        if constexpr (!WIN) {
          Diff32 D;
          if constexpr (MODE == kTR)
            D = diff32_tr64(J, tile64[jl], I[p], &Fi.x, eps2f);
          else
            D = diff32<MODE>(I[p], J, eps2f);
          const float wt = near_weight_again(D, J.m, gB[p], gkB[p]);
          if (!(wt < 1.f)) continue;
          share = 1.0 - (double)wt;
        }
        if constexpr (MODE == kTR)
          pair_tr64<POT>(Fi, tile64[jl], J.m, eps2d, share, A[p]);
        else
          pair_mixed64<MODE, POT>(I[p], J, eps2d, share, A[p]);
      }
    }
  }
}

// kTR with the window test: a window flagged "mid" may hold a pair much
// closer than its tile is large.  Tile-relative FP32 coordinates carry an
// error of about u (|x_i - o| + |x_j - o|), so for such a pair they lose
// too much of the pair distance although its term is too small for the
// near test.  The window is summed again in FP32 with the position
// difference formed in FP64 (the tile's FP64 copy and the i's FP64
// position, rounded once) and flushed with the same bias factors; its
// first FP32 sum was left out.  Each lane walks its own windows in order.
template <int F, int NW, int IPT, bool POT>
__device__ __forceinline__ void mid_windows(const DevState& s, const RecTR* tile, const RecP64* tile64, int jl0,
                                            const int* own, int jend, const int64_t* i_glob,
                                            const ModeT<kTR>::I* I, float eps2f, double ca, double cp,
                                            uint32_t mflags, Acc64* A) {
#pragma unroll
  for (int p = 0; p < IPT; ++p) {
    uint32_t f = (mflags >> (p * NW)) & ((1u << NW) - 1u);
    double xi[3] = {0.0, 0.0, 0.0};
    if (f) {
      const int64_t n = s.n, i = i_glob[p];
      xi[0] = s.xp[i];
      xi[1] = s.xp[n + i];
      xi[2] = s.xp[2 * n + i];
    }
    while (f) {
      const int jw = jl0 + __builtin_ctz(f) * F;
      f &= f - 1u;
      Acc32 B;
#pragma unroll
      for (int d = 0; d < 7; ++d) B.v[d] = 0.f;
      float wdummy = 1.f;
#pragma unroll 8
      for (int u = 0; u < F; ++u) {
        const int jl = jw + u;
        const bool drop = jl == own[p] || jl >= jend;
        const RecTR J = tile[jl];
        finish_f32<true, POT, false>(diff32_tr64(J, tile64[jl], I[p], xi, eps2f), J.m, drop, 0.f, 0.f, &wdummy, B);
      }
#pragma unroll
      for (int d = 0; d < 6; ++d) A[p].v[d] = __builtin_fma((double)B.v[d], ca, A[p].v[d]);
      if (POT) A[p].v[6] = __builtin_fma((double)B.v[6], cp, A[p].v[6]);
    }
  }
}

// Sweep this lane's share of one LDS tile for its IPT i-particles.  jl0:
// first tile-local j of the lane; PER: j per lane per tile; the global index
// of tile entry u is the tile start + u.  Each j-record is read from LDS once and
// used for all IPT particles.  MASK drops the particle's own j and entries at
// or past j_end.
//
// NEAR (mixed modes): a single FP32 term carries a few u of error, which
// limits the relative force only when that term is comparable to the whole
// sum, i.e. for a close neighbour with m_j / R^2 > g = tau |a_i| (|a_i| from
// the last step).  No such pair stays in FP32; two ways to find them:
//  * window test (layouts with one lane per i, large blocks): each lane keeps
//    the smallest R^2 of its window (one min per pair); when
//    m_max / R^2_min > g (m_max: largest mass of the window's 32-entry group,
//    wmax[]) the window may hold a near pair: its FP32 sum is left out and
//    the whole window is summed in FP64 instead (a near term would also
//    spoil the rounding of the FP32 sum).
//  * per-pair weights (layouts that split j over lanes, small blocks, where
//    clusters are often small and near pairs common): each pair gets weight
//    0 or 1 in the FP32 window, and the weight-0 pairs are added in FP64.
// The FP64 work runs after the tile's FP32 sweep (near_windows_f64), in a
// wave-uniform branch taken only when some lane marked a window.
// Near thresholds per i: with the window test (one lane per i) gsel = g =
// near_tau |a_i| and ksel = the R^2 below which a window may hold a jerk
// term above near_tau_k |k_i|; with per-pair weights gsel = g * 2^40 and
// ksel = (near_tau_k |k_i| / (2 v)) * 2^40, the m_j / R^3 above which a
// jerk term may exceed it (v bounds |v_j - v_i| over the tile).
template <int MODE, int PER, int IPT, bool MASK, bool POT, bool NEAR, bool LEANW = false, int FW = 32, int TJ = kTile>
__device__ __forceinline__ void sweep_tile(const DevState& s, const typename ModeT<MODE>::Rec* tile,
                                           const RecP64* tile64, const float* wmax, int jl0, const int* own,
                                           int jend, const int64_t* i_glob, const typename ModeT<MODE>::I* I,
                                           const double (*xi64)[3], const float* gsel, const float* ksel,
                                           const float* mthr, double eps2d, float eps2f, double ca, double cp,
                                           Acc64* A) {
  if constexpr (MODE == kF64) {
#pragma unroll 8
    for (int u = 0; u < PER; ++u) {
      const int jl = jl0 + u;
      const RecF64 J = tile[jl];
#pragma unroll
      for (int p = 0; p < IPT; ++p) {
        const bool drop = MASK && (jl == own[p] || jl >= jend);
        pair_f64<MASK, POT>(I[p], J, eps2d, drop, A[p]);
      }
    }
  } else {
    constexpr bool WIN = NEAR && PER == TJ;  // window test
    constexpr bool WGT = NEAR && !WIN;          // per-pair weights
    constexpr int F = PER < FW ? PER : FW;      // FP32 window, then flush to FP64
    constexpr int NW = PER / F;                 // windows per tile
    constexpr bool MID = WIN && MODE == kTR;    // mid windows (kTR, window test)
    static_assert(IPT * NW <= 32, "near flags must fit 32 bits");
    // near windows of this tile: bit p * NW + window; mid windows: the same
    // bits shifted by 32
    uint64_t flags = 0;
    for (int w = 0; w < PER; w += F) {
      Acc32 B[IPT];
      float r2min[IPT];
      float wmin = 1.f;  // smallest near weight met by this lane in the window
#pragma unroll
      for (int p = 0; p < IPT; ++p) {
        r2min[p] = INFINITY;
#pragma unroll
        for (int d = 0; d < 7; ++d) B[p].v[d] = 0.f;
      }
      // per-pair weights carry more temporaries per pair: a partial unroll
      // keeps the j-split layouts within their register budget
#pragma unroll(WGT ? 8 : F)
      for (int u = 0; u < F; ++u) {
        const int jl = jl0 + w + u;
        const typename ModeT<MODE>::Rec J = tile[jl];
#pragma unroll
        for (int p = 0; p < IPT; ++p) {
          Diff32 D;
          if constexpr (MODE == kTR && PER != TJ)
            D = diff32_tr64(J, tile64[jl], I[p], xi64[p], eps2f);
          else
            D = diff32<MODE>(I[p], J, eps2f);
          const bool drop = MASK && (jl == own[p] || jl >= jend);
          if (WIN) r2min[p] = __builtin_fminf(r2min[p], (MASK && drop) ? INFINITY : D.r2);
          finish_f32<MASK, POT, WGT>(D, J.m, drop, gsel[p], ksel[p], &wmin, B[p]);
        }
      }
      // flush: the FP32 window times the factor that removes the mean bias
      // of the hardware reciprocal square root (ca for terms in R^-3, cp for
      // R^-1); a window that may hold a near pair (window test) is left out
      // here and summed in FP64 after the sweep
#pragma unroll
      for (int p = 0; p < IPT; ++p) {
        double fa = ca, fp = cp;
        if constexpr (WIN) {
          bool cand = (wmax[(jl0 + w) / F] > gsel[p] * r2min[p]) || (r2min[p] < ksel[p]);
          // lean sweep (no masked variant): the window holding the i's own
          // entry is always summed again in FP64, which skips that entry
          if constexpr (LEANW) cand = cand || (unsigned)(own[p] - (jl0 + w)) < (unsigned)F;
          flags |= (uint64_t)cand << (p * NW + w / F);
          bool redo = cand;
          if constexpr (MID) {
            const bool mid = !cand && r2min[p] < mthr[p];
            flags |= (uint64_t)mid << (32 + p * NW + w / F);
            redo = cand || mid;
          }
          fa = redo ? 0.0 : ca;
          fp = redo ? 0.0 : cp;
        }
        if constexpr (WGT) flags |= (uint64_t)(wmin < 1.f) << (p * NW + w / F);
#pragma unroll
        for (int d = 0; d < 6; ++d) A[p].v[d] = __builtin_fma((double)B[p].v[d], fa, A[p].v[d]);
        if (POT) A[p].v[6] = __builtin_fma((double)B[p].v[6], fp, A[p].v[6]);
      }
    }
    if constexpr (NEAR) {
      if (__any(flags != 0u)) {
        near_windows_f64<MODE, F, NW, IPT, POT, WIN>(s, tile, tile64, jl0, own, jend, i_glob, I, gsel, ksel, eps2d,
                                                     eps2f, (uint32_t)flags, A);
        if constexpr (MID)
          mid_windows<F, NW, IPT, POT>(s, tile, tile64, jl0, own, jend, i_glob, I, eps2f, ca, cp,
                                       (uint32_t)(flags >> 32), A);
      }
    }
  }
}

// Cluster of work item `item`: the last cluster whose item_off <= item
// (plans are in cluster order, item_off ascending).
__device__ __forceinline__ int find_cluster(const Plan* plan, int nc, int64_t item) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plan[mid].item_off <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One work item.  Layout: JL lanes per i-slot, IPT i-particles per lane
// (IPT > 1 only with JL = 1); the chunk holds IWG = IPT * 256 / JL entries of
// the cluster's active list.
// LEAN (kTR with the near test, every softening large enough that the self
// pair stays finite in FP32): the one-lane-per-i layouts have no masked
// sweep.  The self pair has a zero position and velocity difference, so it
// adds exactly nothing to a and k, and its window is always redone in FP64
// (which skips it); padding records sit at 1e15, where every term is zero.
// Without the masked copy of the sweep the kernel needs far fewer registers.
template <int MODE, int JL, int IPT, bool POT, bool NEAR, bool LEAN = false, int FW = 32, int TJ = kTile,
          bool PIF = false>
__device__ void run_item(const DevState& s, const int32_t* __restrict__ act, const Plan& P, int c,
                         int64_t local_item, unsigned char* lds, float* wmax) {
  static_assert(JL == 1 || IPT == 1, "several i per lane only with one lane per i");
  constexpr int SLOTS = kForceThreads / JL;  // i-slots per pass
  constexpr int IWG = SLOTS * IPT;
  constexpr int PER = TJ / JL;
  constexpr bool FRAME = MODE == kTR || (NEAR && MODE != kF64);  // reads the tile frames
  constexpr bool LEANW = LEAN && JL == 1 && NEAR && MODE == kTR;
  constexpr float kPad = LEANW ? 1e15f : 0.f;  // position of padding records
  using Rec = typename ModeT<MODE>::Rec;
  using IT = typename ModeT<MODE>::I;
  constexpr bool WIN = NEAR && PER == TJ;  // window test (else per-pair weights)
  Rec* tile = reinterpret_cast<Rec*>(lds);
  RecP64* tile64 = reinterpret_cast<RecP64*>(lds + kTile * sizeof(RecTR));  // kTR only

  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // opaque here: nothing derived from it is hoisted out of the item loop
  const int il = tid % SLOTS;
  const int jl = tid / SLOTS;
  const int chunk = (int)(local_item / P.slices);
  const int slice = (int)(local_item % P.slices);
  const int64_t c_begin = s.coff[c], c_end = s.coff[c + 1];

  int q_local[IPT];
  bool listed[IPT], valid[IPT];
  int64_t i_glob[IPT];
  IT I[IPT];
  Acc64 A[IPT];
#pragma unroll
  for (int p = 0; p < IPT; ++p) {
    q_local[p] = chunk * IWG + p * SLOTS + il;  // entry of the cluster's active list
    listed[p] = q_local[p] < P.n_act;
    valid[p] = listed[p];
    i_glob[p] = c_begin;
    if (valid[p]) {
      i_glob[p] = act[P.act_off + q_local[p]];
      if (i_glob[p] < c_begin || i_glob[p] >= c_end) {
        __hip_atomic_fetch_or(s.status, (int32_t)ST_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        valid[p] = false;
        i_glob[p] = c_begin;
      }
    }
    I[p] = load_i<MODE>(s, i_glob[p]);
#pragma unroll
    for (int d = 0; d < 7; ++d) A[p].v[d] = 0.0;
  }
  const double eps = s.eps[c];
  const double eps2d = eps * eps;
  const float eps2f = (float)eps2d;
  const double ca = s.ctl->rsq_scale3, cp = s.ctl->rsq_scale1;
  // near-pair thresholds from the last step: g = tau |a_i| (times 2^40 for
  // the per-pair weights), gk = tau_k |k_i|; infinity (no test) while
  // unknown or zero
  float gsel[IPT], gk[IPT];
  const float tau_a = (float)s.ctl->near_tau, tau_k = (float)s.ctl->near_tau_k, tau_m = (float)s.ctl->mid_tau;
#pragma unroll
  for (int p = 0; p < IPT; ++p) {
    gsel[p] = INFINITY;
    gk[p] = INFINITY;
    if (NEAR) {
      const int64_t n = s.n, i = i_glob[p];
      const double ax = s.a[i], ay = s.a[n + i], az = s.a[2 * n + i];
      const double gi = s.ctl->near_tau * sqrt(ax * ax + ay * ay + az * az);
      if (gi > 0.0 && gi < 1e30) gsel[p] = (float)gi;
      const double kx = s.k[i], ky = s.k[n + i], kz = s.k[2 * n + i];
      const double gki = s.ctl->near_tau_k * sqrt(kx * kx + ky * ky + kz * kz);
      if (gki > 0.0 && gki < 1e30) gk[p] = (float)gki;
      if (!WIN) gsel[p] = gsel[p] * kNearScale;
    }
  }

  const int64_t j_begin = c_begin + (int64_t)slice * P.slice_len;
  int64_t j_end = j_begin + P.slice_len;
  if (j_end > c_end) j_end = c_end;
  // PIF builds (launched only while the fused predictor is on, the device
  // flag the selection reads being set from the same host test): the FP64
  // records of a block that takes it (j-split layouts) are predicted here to
  // the cluster's prediction time.  The flag is not read here: a load on
  // this path delays the tile's loads by a memory round trip.
  bool fused = false;
  double tp = 0.0;
  if constexpr (PIF && MODE == kF64 && JL > 1) {
    fused = fused_prediction(1, P.variant, P.chunks);
    tp = s.tpred[c];
  }
  // the frames must have been formed at the cluster's prediction time (the
  // selection forms them only for blocks that read them, all of a cluster's
  // or none): checked on the item's first tile, off the sweep's registers
  if constexpr (FRAME) {
    if (tid == 0 && j_begin < j_end &&
        s.tmeta[(int64_t)(s.cl_ch[c] + (int)((j_begin - c_begin) / kTile)) * kTileMeta + TM_T] != s.tpred[c])
      __hip_atomic_fetch_or(s.status, (int32_t)ST_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  for (int64_t j0 = j_begin; j0 < j_end; j0 += TJ) {
    // frame of this tile (selection chunk), the same for every thread
    double fo[3] = {0.0, 0.0, 0.0}, fv[3] = {0.0, 0.0, 0.0};
    float f_w = 0.f, f_mmax = 0.f, f_d = 0.f;
    if constexpr (FRAME) {
      const double* f = s.tmeta + (int64_t)(s.cl_ch[c] + (int)((j0 - c_begin) / kTile)) * kTileMeta;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        fo[d] = f[TM_OX + d];
        fv[d] = f[TM_VX + d];
      }
      f_w = (float)f[TM_W];
      f_mmax = (float)f[TM_MMAX];
      f_d = (float)f[TM_D];
    }
    __syncthreads();  // previous tile fully consumed
    // at most one record per thread; a tile lies inside one selection chunk
    // (slices start at multiples of kTile), whose frame it uses
    static_assert(TJ <= kForceThreads && kTile % TJ == 0, "tile of at most one record per thread");
    {
      const int64_t j = j0 + tid;
      const bool loads = tid < TJ && j < j_end;
      float mrec;
      if constexpr (MODE == kTR) {
        RecTR r = zero_rec<kTR>();
        r.x = r.y = r.z = kPad;
        RecP64 q{(double)kPad, (double)kPad, (double)kPad, 0.0, 0.0, 0.0};
        if (loads) {
          q = load_p64(s, j);
          r.x = (float)(q.x - fo[0]);
          r.y = (float)(q.y - fo[1]);
          r.z = (float)(q.z - fo[2]);
          r.vx = (float)(q.vx - fv[0]);
          r.vy = (float)(q.vy - fv[1]);
          r.vz = (float)(q.vz - fv[2]);
          r.m = s.jr[JR_M * s.n + j];
        }
        tile[tid] = r;
        tile64[tid] = q;
        mrec = r.m;
      } else {
        Rec rec;
        if constexpr (PIF && MODE == kF64 && JL > 1) {
          rec = zero_rec<MODE>();
          if (loads) rec = fused ? predict_rec(s, j, tp) : load_rec<MODE>(s, j);
        } else {
          rec = loads ? load_rec<MODE>(s, j) : zero_rec<MODE>();
        }
        tile[tid] = rec;
        mrec = (float)rec.m;
      }
      if (NEAR && JL == 1) {  // largest mass of each window of FW entries (padding has m = 0)
        float mm = mrec;
#pragma unroll
        for (int o = FW / 2; o >= 1; o >>= 1) mm = fmaxf(mm, __shfl_xor(mm, o, FW));
        if (tid % FW == 0) wmax[tid / FW] = mm;
      }
    }
    // per i and tile: kTR coordinates relative to the frame (from the FP64
    // state, reloaded rather than kept), and the jerk threshold (a jerk term
    // is at most 2 m_j (|v_i - v_c| + W) / R^3): the window test flags
    // R^2 < (2 m_max v / gk)^(2/3), the per-pair weights m_j / R^3 > gk / (2 v)
    float ksel[IPT], mthr[IPT];
    double xi64[IPT][3];  // kTR j-split layouts: the i's FP64 position
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
      float vrel[3];
      xi64[p][0] = xi64[p][1] = xi64[p][2] = 0.0;
      if constexpr (MODE == kTR) {
        const RecP64 F = load_p64(s, i_glob[p]);
        if constexpr (JL > 1) {
          xi64[p][0] = F.x;
          xi64[p][1] = F.y;
          xi64[p][2] = F.z;
        }
        I[p].x = (float)(F.x - fo[0]);
        I[p].y = (float)(F.y - fo[1]);
        I[p].z = (float)(F.z - fo[2]);
        I[p].vx = (float)(F.vx - fv[0]);
        I[p].vy = (float)(F.vy - fv[1]);
        I[p].vz = (float)(F.vz - fv[2]);
        vrel[0] = I[p].vx; vrel[1] = I[p].vy; vrel[2] = I[p].vz;
      } else if constexpr (MODE == kF64) {
        vrel[0] = vrel[1] = vrel[2] = 0.f;
      } else {
        vrel[0] = I[p].vx - (float)fv[0];
        vrel[1] = I[p].vy - (float)fv[1];
        vrel[2] = I[p].vz - (float)fv[2];
      }
      ksel[p] = WIN ? 0.f : INFINITY;
      mthr[p] = 0.f;
      if constexpr (NEAR && MODE != kF64) {
        const float vmax = sqrtf(vrel[0] * vrel[0] + vrel[1] * vrel[1] + vrel[2] * vrel[2]) + f_w;
        if (gk[p] < INFINITY) {
          if constexpr (WIN) {
            const float c2 = 2.f * f_mmax * vmax;
            if (c2 > 0.f) ksel[p] = exp2f((2.f / 3.f) * log2f(c2 / gk[p]));
          } else {
            if (vmax > 0.f) ksel[p] = gk[p] / (2.f * vmax) * kNearScale;
          }
        }
        if constexpr (WIN && MODE == kTR) {
          // mid test: a pair of distance R in this tile has a relative error
          // of about (L / R) u with L = |x_i - o| + D; redo the window when
          // its term times L / R may exceed mid_tau |a_i| (acceleration) or
          // mid_tau |k_i| (jerk):  R^3 < m L / (mid_tau |a|) or
          // R^4 < 2 m v L / (mid_tau |k|)
          const float L = sqrtf(I[p].x * I[p].x + I[p].y * I[p].y + I[p].z * I[p].z) + f_d;
          const float ca_ = f_mmax * L * tau_a / tau_m;
          if (gsel[p] < INFINITY && ca_ > 0.f) mthr[p] = exp2f((2.f / 3.f) * log2f(ca_ / gsel[p]));
          const float ck_ = 2.f * f_mmax * vmax * L * tau_k / tau_m;
          if (gk[p] < INFINITY && ck_ > 0.f) mthr[p] = fmaxf(mthr[p], sqrtf(ck_ / gk[p]));
        }
      }
    }
    __syncthreads();
    // tile-local index of each i's own entry (-1: not in this tile) and the
    // tile-local end of the slice: masking compares 32-bit tile indices
    int own[IPT];
    bool mine = false;
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
      const int64_t d = i_glob[p] - j0;
      own[p] = (valid[p] && d >= 0 && d < TJ) ? (int)d : -1;
      mine |= own[p] >= 0;
    }
    const int jend = (int)(j_end - j0 < TJ ? j_end - j0 : TJ);
    const bool need_mask = !LEANW && (jend < TJ || __any(mine));
    if constexpr (LEANW)
      sweep_tile<MODE, PER, IPT, false, POT, NEAR, true, FW, TJ>(s, tile, tile64, wmax, jl * PER, own, jend, i_glob, I,
                                                             xi64, gsel, ksel, mthr, eps2d, eps2f, ca, cp, A);
    else if (need_mask)
      sweep_tile<MODE, PER, IPT, true, POT, NEAR, false, FW, TJ>(s, tile, tile64, wmax, jl * PER, own, jend, i_glob, I,
                                                             xi64, gsel, ksel, mthr, eps2d, eps2f, ca, cp, A);
    else
      sweep_tile<MODE, PER, IPT, false, POT, NEAR, false, FW, TJ>(s, tile, tile64, wmax, jl * PER, own, jend, i_glob, I,
                                                              xi64, gsel, ksel, mthr, eps2d, eps2f, ca, cp, A);
  }
  // PIF builds: the other FP64 records are the stored prediction, which the
  // selection left complete unless it decided this block fused, so the
  // first tile's chunk must carry the cluster's prediction time (checked
  // after the sweep, off the latency of its first tile)
  if constexpr (PIF && MODE == kF64) {
    if (!fused && tid == 0 && j_begin < j_end &&
        s.tpstamp[s.cl_ch[c] + (int)((j_begin - c_begin) / kTile)] != s.tpred[c])
      __hip_atomic_fetch_or(s.status, (int32_t)ST_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  const int64_t rows_cap = s.rows_cap;
  const int64_t row0 = P.slot_base + (int64_t)slice * P.n_act;
#pragma unroll
  for (int p = 0; p < IPT; ++p) {
    if (!valid[p]) {  // unlisted slot, or an index outside its cluster: contributes zeros
#pragma unroll
      for (int d = 0; d < 7; ++d) A[p].v[d] = 0.0;
    }
  }
  if constexpr (JL == 1) {
#pragma unroll
    for (int p = 0; p < IPT; ++p) {
      if (listed[p]) {
#pragma unroll
        for (int d = 0; d < (POT ? 7 : 6); ++d) s.part[d * rows_cap + row0 + q_local[p]] = A[p].v[d];
      }
    }
  } else {
    // combine the JL lane partials of each i in ascending lane order
    __syncthreads();
    double* red = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int d = 0; d < 7; ++d) red[(d * JL + jl) * SLOTS + il] = A[0].v[d];
    __syncthreads();
    if (tid < SLOTS) {
      const int q2 = chunk * IWG + tid;
      if (q2 < P.n_act) {
#pragma unroll
        for (int d = 0; d < (POT ? 7 : 6); ++d) {
          double sum = 0.0;
          for (int l = 0; l < JL; ++l) sum += red[(d * JL + l) * SLOTS + tid];
          s.part[d * rows_cap + row0 + q2] = sum;
        }
      }
    }
  }
}

// POT: also sum the potential (partial row 6); without it row 6 is not written.
// NEAR: FP64 evaluation of near pairs in the mixed modes.
// SPLIT: only the layouts that split j over lanes (2, 3, 4).  They need at
// most 128 VGPRs, so this kernel runs 4 waves per SIMD, against 3 (at most
// 168 VGPRs, which the two-i-per-lane layout needs) for the kernel with
// every layout.  The host launches it when no cluster can reach a
// one-lane-per-i layout (its size is below that layout's threshold); a work
// item of such a layout here is an inconsistency: it is reported and
// skipped.  Without the pinned occupancy the near-pair variants of the full
// kernel grow past 168 VGPRs and drop to 2 waves.
// par >= 0 with a single cluster (the step pipeline): the plan follows from
// that step parity's selection count (plan_single); otherwise it is read
// from s.plan.
// FW: the FP32 window (16, 32 or 64 pairs); WPE: the occupancy the
// compiler is held to (waves per SIMD); TJ: j-records per LDS tile (128 or
// 256; a 128-record tile uses half the threads to load and half a selection
// chunk's frame); PIF: the fused predictor (launched only by the step
// pipeline, and only while it is on).  Builds other than FW = 32, TJ = 256
// with the default occupancy are made only of the lean tile-relative kernel
// without the potential (the autotuner's candidates).
template <int MODE, bool POT, bool NEAR, bool SPLIT, bool LEAN, int FW = 32, int WPE = (SPLIT ? 4 : 3),
          int TJ = kTile, bool PIF = false>
__global__ void __launch_bounds__(kForceThreads) __attribute__((amdgpu_waves_per_eu(WPE)))
force_kernel(DevState s, const int32_t* __restrict__ act, int par, int64_t target_items) {
  static_assert(FW == 16 || FW == 32 || FW == 64, "FP32 window of 16, 32 or 64 pairs");
  static_assert(TJ == 128 || TJ == kTile, "j-tiles of 128 or 256 records");
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  __shared__ float wmax[kTile / 16];
  __shared__ int64_t offs_sh[kLdsClusters];
  const bool single = par >= 0 && s.nc == 1;
  // batches of up to kLdsClusters: the item offsets in LDS for the lookup
  const bool lds_lookup = !single && s.nc > 1 && s.nc <= kLdsClusters;
  if (lds_lookup) {
    for (int k = threadIdx.x; k < s.nc; k += kForceThreads) offs_sh[k] = s.offs[k];
    __syncthreads();
  }
  Plan P1{};
  int64_t total;
  if (single) {
    P1 = plan_single(s, par, target_items);
    total = (int64_t)P1.chunks * P1.slices;
  } else {
    total = s.ctl->total_items;
  }
  // the tile-relative mode runs the FP64 arithmetic in the layouts that
  // split j over lanes (SM: the split-layout mode)
  constexpr int SM = MODE == kTR ? kF64 : MODE;
  constexpr bool SNEAR = NEAR && SM != kF64;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int c = single ? 0 : lds_lookup ? last_at_or_below(offs_sh, s.nc, item) : find_cluster(s.plan, s.nc, item);
    const Plan P = single ? P1 : s.plan[c];
    const int64_t local = item - P.item_off;
    if constexpr (SPLIT) {
      switch (P.variant) {
        case 2: run_item<SM, 4, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 3: run_item<SM, 16, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 4: run_item<SM, 64, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        default:
          if (threadIdx.x == 0)
            __hip_atomic_fetch_or(s.status, (int32_t)ST_STATE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
      }
    } else if constexpr (MODE == kTR) {
      // the tile-relative format has no two-i-per-lane build (its registers
      // spill, and a kernel that needs scratch memory costs microseconds
      // per launch): the host plans it with that layout's threshold above
      // any block size, so layout 0 never occurs here
      switch (P.variant) {
        case 1: run_item<MODE, 1, 1, POT, NEAR, LEAN, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 2: run_item<SM, 4, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 3: run_item<SM, 16, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        default: run_item<SM, 64, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
      }
    } else {
      switch (P.variant) {
        case 0: run_item<MODE, 1, 2, POT, NEAR, LEAN, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 1: run_item<MODE, 1, 1, POT, NEAR, LEAN, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 2: run_item<SM, 4, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        case 3: run_item<SM, 16, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
        default: run_item<SM, 64, 1, POT, SNEAR, false, FW, TJ, PIF>(s, act, P, c, local, lds, wmax); break;
      }
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

struct ForceLaunch {
  const DevState& s;
  const int32_t* act;
  int grid, par;
  bool lean;
  int64_t target_items;
  hipStream_t st;
  int window, waves, tile;  // FP32 window, occupancy and j-tile of the lean tile-relative kernel
};

// The lean tile-relative kernel without the potential in one of the
// autotuner's other builds (window 16, 32 or 64; 2 to 5 waves per SIMD;
// j-tiles of 256 or 128 records, the latter with windows of 16 or 32; not
// the default 32 / 4 / 256):
// force_tuned.hip and force_tuned_t128.hip.
hipError_t launch_force_tuned(const ForceLaunch& L);
hipError_t launch_force_tuned_t128(const ForceLaunch& L);

}  // namespace nb
