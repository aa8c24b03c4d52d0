// Block-step kernels around the force pass (Sect. 2.1 item list):
// selection of the block, Hermite prediction, planning of the force work,
// reduction of slice partials, Hermite correction with Aarseth's step
// criterion and power-of-two quantisation, start-up and energy.
// All FP64.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace nb {

__device__ __forceinline__ void set_status(const DevState& s, int32_t bit) {
  __hip_atomic_fetch_or(s.status, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// (smallest value, how many have it) of two such pairs.  A NaN never counts.
__device__ __forceinline__ void min_count(double& v, int32_t& n, double ov, int32_t on) {
  const double m = fmin(v, ov);
  n = (v == m ? n : 0) + (ov == m ? on : 0);
  v = m;
}

// The workgroup's smallest v and the number of its threads' counts n at
// that value; every thread gets both.  The waves are combined in a fixed
// order (the count is exact in any order).
__device__ __forceinline__ double block_min_count(double v, int32_t& n, double* buf, int32_t* nbuf) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) min_count(v, n, __shfl_xor(v, o), __shfl_xor(n, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    buf[threadIdx.x >> 6] = v;
    nbuf[threadIdx.x >> 6] = n;
  }
  __syncthreads();
  double r = buf[0];
  int32_t rn = nbuf[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) min_count(r, rn, buf[w], nbuf[w]);
  n = rn;
  return r;
}

// ---------------------------------------------------------------------------
// Hermite predictor (Sect. 2.1, predictor equations) for particle i to time
// tp.  Writes what the force pass of `mode` and the corrector read:
//   kF64: x_p, v_p (FP64);
//   kMX64: x_p, the FP32 velocity of the j-record, and v_p only for members
//          of the block (the corrector's particles);
//   kDS: as kMX64 plus the FP32 pair hi = fl32(x_p), lo = fl32(x_p - hi);
//   kTR: x_p, v_p (FP64) of every particle (the force pass forms FP32
//        coordinates relative to each tile's frame from them);
//   kAllRecords (predict entry point, start-up, energy): everything,
//          including the FP32 mass of the j-record (constant otherwise).
constexpr int kAllRecords = -1;
// Inputs of the predictor for particle i: t and x, v, a, k.
struct PredIn {
  double t, x[3], v[3], a[3], k[3];
};

__device__ __forceinline__ PredIn load_pred(const DevState& s, int64_t i) {
  PredIn in;
  const int64_t n = s.n;
  in.t = s.t[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t o = d * n + i;
    in.x[d] = s.x[o];
    in.v[d] = s.v[o];
    in.a[d] = s.a[o];
    in.k[d] = s.k[o];
  }
  return in;
}

// The predicted position and velocity are also returned in xo, vo.
__device__ __forceinline__ void predict_from(const DevState& s, int64_t i, const PredIn& in, double tp, int mode,
                                             bool member, double xo[3], double vo[3]) {
  const int64_t n = s.n;
  const double h = tp - in.t;
  const bool all = mode == kAllRecords;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t o = d * n + i;
    double xp, vp;
    hermite_predict(in.x[d], in.v[d], in.a[d], in.k[d], h, xp, vp);
    xo[d] = xp;
    vo[d] = vp;
    s.xp[o] = xp;
    if (all || mode == kF64 || mode == kTR || member) s.vp[o] = vp;
    if (all || mode == kDS || mode == kMX64) s.jr[(JR_VX + d) * n + i] = (float)vp;
    if (all || mode == kDS) {
      const float hi = (float)xp;
      s.jr[(JR_HX + d) * n + i] = hi;
      s.jr[(JR_LX + d) * n + i] = (float)(xp - (double)hi);
    }
  }
  if (all) s.jr[JR_M * n + i] = (float)s.m[i];
}

// Frame of selection chunk ch (= LDS tile) from the predicted positions and
// velocities of its particles (`have`: this thread holds one), for the
// mixed modes: bounding-box centres of positions and velocities, the
// half-diagonals of the velocity and position boxes, the largest mass and
// the prediction time tp (the force pass checks that a frame it reads was
// formed at its cluster's prediction time).  Called by every thread of the
// workgroup; min / max are exact, so the frame does not depend on the
// reduction order.
__device__ __forceinline__ void tile_frame(const DevState& s, int ch, bool have, const double xp[3], const double vp[3],
                                           double m, double tp) {
  __shared__ double red[kSelThreads / 64][13];
  const int tid = threadIdx.x;
  double lo[6], hi[6], mm = have ? m : 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = have ? xp[d] : INFINITY;
    hi[d] = have ? xp[d] : -INFINITY;
    lo[3 + d] = have ? vp[d] : INFINITY;
    hi[3 + d] = have ? vp[d] : -INFINITY;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
    }
    mm = fmax(mm, __shfl_xor(mm, off));
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      red[tid >> 6][d] = lo[d];
      red[tid >> 6][6 + d] = hi[d];
    }
    red[tid >> 6][12] = mm;
  }
  __syncthreads();
  // 13 threads combine the wave results of one quantity each, in parallel
  if (tid < 13) {
    double r = red[0][tid];
    for (int w = 1; w < kSelThreads / 64; ++w) r = tid < 6 ? fmin(r, red[w][tid]) : fmax(r, red[w][tid]);
    red[0][tid] = r;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      lo[d] = red[0][d];
      hi[d] = red[0][6 + d];
    }
    mm = red[0][12];
    double* f = s.tmeta + (int64_t)ch * kTileMeta;
    double w2 = 0.0, d2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      f[TM_OX + d] = 0.5 * (lo[d] + hi[d]);
      f[TM_VX + d] = 0.5 * (lo[3 + d] + hi[3 + d]);
      const double e = hi[3 + d] - lo[3 + d], ex = hi[d] - lo[d];
      w2 += e * e;
      d2 += ex * ex;
    }
    f[TM_W] = 0.5 * sqrt(w2);
    f[TM_MMAX] = mm;
    f[TM_D] = 0.5 * sqrt(d2);
    f[TM_T] = tp;
  }
}

// Full prediction, one workgroup per selection chunk: every particle of
// every cluster to s.tpred of its cluster, every record field, and the
// chunk's tile frame.
__global__ void __launch_bounds__(kSelThreads) predict_all_kernel(DevState s) {
  const int ch = blockIdx.x;
  const int64_t i = s.ch_begin[ch] + threadIdx.x;
  const bool have = i < s.ch_begin[ch + 1];
  double xp[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};
  double m = 0.0;
  const double tp = s.tpred[s.ch_cluster[ch]];
  if (have) {
    predict_from(s, i, load_pred(s, i), tp, kAllRecords, true, xp, vp);
    m = s.m[i];
  }
  tile_frame(s, ch, have, xp, vp, m, tp);
  if (threadIdx.x == 0) s.tpstamp[ch] = tp;
}

hipError_t launch_predict_all(const DevState& s, hipStream_t st) {
  static_assert(kSelChunk == kSelThreads, "one particle per thread");
  hipLaunchKernelGGL(predict_all_kernel, dim3(s.nch), dim3(kSelThreads), 0, st, s);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) map_active_kernel(DevState s, const int32_t* __restrict__ ids,
                                                         int64_t n_active) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_active) return;
  const int32_t id = ids[q];
  s.ulist[q] = (id >= 0 && id < s.n) ? s.slot_of[id] : -1;
}

hipError_t launch_map_active(const DevState& s, const int32_t* ids, int64_t n_active, hipStream_t st) {
  if (n_active <= 0) return hipSuccess;
  hipLaunchKernelGGL(map_active_kernel, dim3((unsigned)((n_active + 255) / 256)), dim3(256), 0, st, s, ids,
                     n_active);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) identity_kernel(DevState s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s.n; i += (int64_t)gridDim.x * blockDim.x)
    s.act[i] = (int32_t)i;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t <= s.nc) s.aoff[t] = s.coff[t];
}

hipError_t launch_identity(const DevState& s, hipStream_t st) {
  int64_t g = (s.n + 255) / 256;
  const int64_t gc = (s.nc + 1 + 255) / 256;
  if (g < gc) g = gc;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)(g < 65535 ? g : 65535)), dim3(256), 0, st, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work plan of a force pass (one workgroup).  For every cluster: the i x j
// layout variant from its block size, the number of i-chunks, and the number
// of j-slices, chosen from the cluster's own block size and particle count
// only (so a cluster's sums come out bit-identical whether it is planned
// alone or inside a batch): as many slices as bring the cluster alone to
// about target_items work items, at most one per LDS tile and at most what
// the partial-row budget of the cluster allows.  Offsets of items and
// partial rows are exclusive prefix sums in cluster order.
__device__ __forceinline__ int64_t wg_exclusive_scan(int64_t v, int64_t* buf, int64_t* total) {
  // 256 threads: inclusive scan inside each wave by shuffles, then the wave
  // totals through LDS (buf[0..3])
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) buf[wave] = x;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int64_t t = buf[w];
    before += w < wave ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();  // buf is reused by the next scan
  return before + x - v;
}

__device__ __forceinline__ bool bad_range(const int64_t* aoff, const int64_t* coff, int c, int64_t bound) {
  const int64_t a0 = aoff[c], a1 = aoff[c + 1];
  return a0 < 0 || a1 < a0 || a1 > bound || a1 - a0 > coff[c + 1] - coff[c];
}

// The plan of one cluster, apart from its offsets (items, rows, units).
__device__ __forceinline__ void plan_row(const DevState& s, const int64_t* __restrict__ aoff, int64_t n_act_bound,
                                         int64_t target_items, int count_stats, const int32_t* counts,
                                         const int32_t* vmin_all, int c, Plan& P) {
  const int64_t nn = s.coff[c + 1] - s.coff[c];
  int64_t na;
  if (counts) {
    na = __hip_atomic_load(&counts[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    na = aoff[c + 1] - aoff[c];
    if (bad_range(aoff, s.coff, c, n_act_bound)) na = 0;
  }
  plan_layout(na, nn, target_items, vmin_all, P);
  if (count_stats && na > 0) {  // block-step counters (one writer per cluster)
    s.inter[c] += (double)na * (double)nn;
    s.steps[c] += 1;
  }
  if (counts) {
    P.act_off = s.coff[c];
  } else {  // clamped so that a corrupt offset cannot steer reads out of the list
    P.act_off = aoff[c] < 0 ? 0 : aoff[c] > n_act_bound ? n_act_bound : aoff[c];
  }
}


// The plan, computed by one workgroup of 256 threads.
// counts != NULL (step pipeline): cluster c's block is counts[c] entries of
// the active list starting at coff[c] (its own segment); aoff is unused.
__device__ void plan_body(const DevState& s, const int64_t* __restrict__ aoff, int64_t n_act_bound,
                          int64_t target_items, int count_stats, const int32_t* counts) {
  __shared__ int64_t sbuf[256];
  const int tid = threadIdx.x;
  const int nc = s.nc;
  const int per = (nc + 255) / 256;
  const int c0 = tid * per < nc ? tid * per : nc;
  const int c1 = c0 + per < nc ? c0 + per : nc;
  int32_t vmin[2 * (kNumVariants - 1) + 1];  // large-cluster, small-cluster thresholds, size cut
  load_thresholds(s.ctl, vmin);

  if (!counts) {
    bool bad = (tid == 0) && (aoff[0] != 0);
    for (int c = c0; c < c1; ++c)
      if (bad_range(aoff, s.coff, c, n_act_bound)) bad = true;
    if (bad) set_status(s, ST_INDEX);
  }

  int64_t my_items = 0, my_rows = 0, my_red = 0;
  for (int c = c0; c < c1; ++c) {
    Plan& P = s.plan[c];
    plan_row(s, aoff, n_act_bound, target_items, count_stats, counts, vmin, c, P);
    const int64_t chunks = P.chunks, S = P.slices, na = P.n_act;
    my_items += chunks * S;
    my_rows += S * na;
    my_red += plan_units(P);
  }
  __syncthreads();
  int64_t tot_items, tot_rows, tot_red;
  int64_t bi = wg_exclusive_scan(my_items, sbuf, &tot_items);
  int64_t br = wg_exclusive_scan(my_rows, sbuf, &tot_rows);
  int64_t bu = wg_exclusive_scan(my_red, sbuf, &tot_red);
  for (int c = c0; c < c1; ++c) {
    Plan& P = s.plan[c];
    P.item_off = bi;
    P.slot_base = br;
    P.red_off = bu;
    s.offs[c] = bi;
    s.offs[nc + c] = bu;
    bi += (int64_t)P.chunks * P.slices;
    br += (int64_t)P.slices * P.n_act;
    bu += plan_units(P);
  }
  if (tid == 0) {
    if (tot_rows > s.rows_cap) {  // cannot happen with the bounds of the plan; refuse the pass
      set_status(s, ST_INDEX);
      tot_items = 0;
      tot_red = 0;
    }
    s.ctl->total_items = tot_items;
    s.ctl->total_rows = tot_rows;
    s.ctl->total_red = tot_red;
  }
}

// The plan for at most 64 clusters: one wave, one cluster per lane, the
// offsets by wave shuffles (no barriers).
__device__ __forceinline__ int64_t wave_exclusive_scan(int64_t v, int64_t* total) {
  const int lane = threadIdx.x;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63);
  return x - v;
}

__device__ void plan_small(const DevState& s, const int64_t* __restrict__ aoff, int64_t n_act_bound,
                           int64_t target_items, int count_stats, const int32_t* counts) {
  const int c = threadIdx.x;
  const int nc = s.nc;
  int32_t vmin[2 * (kNumVariants - 1) + 1];  // large-cluster, small-cluster thresholds, size cut
  load_thresholds(s.ctl, vmin);
  if (!counts) {
    bool bad = (c == 0) && (aoff[0] != 0);
    if (c < nc && bad_range(aoff, s.coff, c, n_act_bound)) bad = true;
    if (bad) set_status(s, ST_INDEX);
  }
  Plan P{};
  if (c < nc) plan_row(s, aoff, n_act_bound, target_items, count_stats, counts, vmin, c, P);
  int64_t tot_items, tot_rows, tot_red;
  P.item_off = wave_exclusive_scan(c < nc ? (int64_t)P.chunks * P.slices : 0, &tot_items);
  P.slot_base = wave_exclusive_scan(c < nc ? (int64_t)P.slices * P.n_act : 0, &tot_rows);
  P.red_off = wave_exclusive_scan(c < nc ? plan_units(P) : 0, &tot_red);
  if (c < nc) {
    s.plan[c] = P;
    s.offs[c] = P.item_off;
    s.offs[nc + c] = P.red_off;
  }
  if (c == 0) {
    if (tot_rows > s.rows_cap) {  // cannot happen with the bounds of the plan; refuse the pass
      set_status(s, ST_INDEX);
      tot_items = 0;
      tot_red = 0;
    }
    s.ctl->total_items = tot_items;
    s.ctl->total_rows = tot_rows;
    s.ctl->total_red = tot_red;
  }
}

__global__ void __launch_bounds__(64) plan_small_kernel(DevState s, const int64_t* __restrict__ aoff,
                                                        int64_t n_act_bound, int64_t target_items, int count_stats,
                                                        int32_t* counts) {
  plan_small(s, aoff, n_act_bound, target_items, count_stats, counts);
  // step pipeline: this half of the counters is read; clear it for the step
  // after next, which counts into it again
  if (counts && (int)threadIdx.x < s.nc) counts[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) plan_kernel(DevState s, const int64_t* __restrict__ aoff,
                                                   int64_t n_act_bound, int64_t target_items, int count_stats) {
  plan_body(s, aoff, n_act_bound, target_items, count_stats, nullptr);
}

hipError_t launch_plan(const DevState& s, const int64_t* aoff, int64_t n_act_bound, int64_t target_items,
                       hipStream_t st, int count_stats) {
  if (s.nc <= 64)
    hipLaunchKernelGGL(plan_small_kernel, dim3(1), dim3(64), 0, st, s, aoff, n_act_bound, target_items, count_stats,
                       (int32_t*)nullptr);
  else
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(256), 0, st, s, aoff, n_act_bound, target_items, count_stats);
  return hipGetLastError();
}

// The stored state of particle i that its corrector reads: t, dt, a, k (the
// values from the start of its step) and the predicted x_p, v_p.
struct CorrIn {
  double t, dt, a0[3], k0[3], xp[3], vp[3];
};

__device__ __forceinline__ CorrIn load_corr(const DevState& s, int64_t i) {
  CorrIn in;
  const int64_t n = s.n;
  in.t = s.t[i];
  in.dt = s.dt[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t o = d * n + i;
    in.a0[d] = s.a[o];
    in.k0[d] = s.k[o];
    in.xp[d] = s.xp[o];
    in.vp[d] = s.vp[o];
  }
  return in;
}

// Sum of the slice partials of every active entry (the across-processor sum
// of the paper's j-parallel scheme, Sect. 3).  Work unit = 256/TP entries of
// one cluster, TP = lanes per entry (the cluster's slice count rounded up to a
// power of two, at most 256).  Lane l adds slices l, l + TP, ... in order;
// the lane sums of each wave are combined by a fixed binary tree of shuffles,
// and for TP > 64 the TP / 64 wave sums by a fixed tree in LDS.  TP and
// the order depend only on the cluster's own plan, so the bits of a cluster
// do not depend on the rest of the batch.  Outputs: acc[d * stride + q],
// jerk[d * stride + q], pot[q] (pot may be NULL); entries at or past the
// active count are skipped.  STEP: the sums go straight to the corrector.
__device__ __forceinline__ double correct_one(const DevState& s, const Ctl& ctl, int c, int64_t i, bool first,
                                              const double a1[3], const double k1[3], const CorrIn& in);

// Cluster of reduce unit u: the last cluster whose red_off <= u.
__device__ __forceinline__ int cluster_of_unit(const Plan* plan, int nc, int64_t u) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plan[mid].red_off <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The reduce work units [blockIdx.x, units) in steps of gridDim.x.  SINGLE:
// the only cluster's plan is P1 (step pipeline); otherwise from s.plan.
template <bool STEP, bool SINGLE, bool COUNT>
__device__ __forceinline__ void reduce_units(const DevState& s, int64_t units, const Plan& P1, int64_t n_active,
                                             double* acc, double* jerk, double* pot, int64_t stride,
                                             double* wave_min, int32_t* wave_cnt, double (*wave_sum)[256 / 64],
                                             int64_t* offs_sh) {
  const int tid = threadIdx.x;
  const int64_t rows_cap = s.rows_cap;
  // batches of up to kLdsClusters: the unit offsets in LDS for the lookup
  const bool lds_lookup = !SINGLE && s.nc > 1 && s.nc <= kLdsClusters;
  if (lds_lookup) {
    for (int k = tid; k < s.nc; k += 256) offs_sh[k] = s.offs[s.nc + k];
    __syncthreads();
  }
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int c = SINGLE ? 0 : lds_lookup ? last_at_or_below(offs_sh, s.nc, u) : cluster_of_unit(s.plan, s.nc, u);
    const Plan P = SINGLE ? P1 : s.plan[c];
    const int tp = P.red_tp;
    const int epw = 256 / tp;
    const int lane = tid % tp;
    const int64_t e = (u - P.red_off) * epw + tid / tp;  // entry within the cluster
    const bool live = e < P.n_act;
    const int64_t q = P.act_off + e;
    // STEP: the corrector's inputs are loaded first, so that their latency
    // overlaps that of the slice partials
    const bool corrects = STEP && live && lane == 0 && q < n_active;
    int64_t i = 0;
    CorrIn cin{};
    if (corrects) {
      i = s.act[q];
      cin = load_corr(s, i);
    }
    double v[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) v[d] = 0.0;
    if (live) {
      const int64_t r0 = P.slot_base + e;
      for (int sl = lane; sl < P.slices; sl += tp) {
        const int64_t r = r0 + (int64_t)sl * P.n_act;
#pragma unroll
        for (int d = 0; d < 6; ++d) v[d] += s.part[d * rows_cap + r];
        if (pot) v[6] += s.part[6 * rows_cap + r];
      }
    }
    // lane l of a group of wtp = min(tp, 64) lanes adds lane l + off,
    // off = wtp/2 ... 1; a group lies inside one wave
    const int wtp = tp < 64 ? tp : 64;
    const int wl = tid & (wtp - 1);
    for (int off = wtp >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int d = 0; d < 7; ++d) {
        const double o = __shfl_down(v[d], off);
        if (wl < off) v[d] += o;
      }
    }
    if (tp > 64) {  // the entry spans tp / 64 waves (tp is the same for the whole block)
      if ((tid & 63) == 0) {
#pragma unroll
        for (int d = 0; d < 7; ++d) wave_sum[d][tid >> 6] = v[d];
      }
      __syncthreads();
      if (lane == 0) {
        const int w = tid >> 6;
#pragma unroll
        for (int d = 0; d < 7; ++d)
          v[d] = tp == 128 ? wave_sum[d][w] + wave_sum[d][w + 1]
                           : (wave_sum[d][0] + wave_sum[d][1]) + (wave_sum[d][2] + wave_sum[d][3]);
      }
    }
    double t_next = INFINITY;  // STEP: new t + dt of the corrected particle
    if (live && lane == 0 && q < n_active) {
      if constexpr (STEP) {  // step pipeline: correct the particle right here
        double a1[3], k1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          a1[d] = v[d];
          k1[d] = v[3 + d];
        }
        if (pot) s.pot[i] = v[6];
        t_next = correct_one(s, *s.ctl, c, i, e == 0, a1, k1, cin);
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          acc[d * stride + q] = v[d];
          jerk[d * stride + q] = v[3 + d];
        }
        if (pot) pot[q] = v[6];
      }
    }
    if constexpr (STEP) {
      // smallest new t + dt of the unit (and, when the selection counts
      // block sizes, how many of its particles have it), for the next block
      // selection
      int32_t cnt = t_next < INFINITY ? 1 : 0;
      if constexpr (COUNT) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) min_count(t_next, cnt, __shfl_xor(t_next, o), __shfl_xor(cnt, o));
      } else {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) t_next = fmin(t_next, __shfl_xor(t_next, o));
      }
      if ((tid & 63) == 0) {
        wave_min[tid >> 6] = t_next;
        wave_cnt[tid >> 6] = cnt;
      }
      __syncthreads();
      if (tid == 0) {
        double m = wave_min[0];
        int32_t k = wave_cnt[0];
        for (int w = 1; w < 4; ++w) min_count(m, k, wave_min[w], wave_cnt[w]);
        s.umin[u] = m;
        if (COUNT) s.ucnt[u] = k;
      }
    }
    __syncthreads();  // wave_min and wave_sum are reused by the next unit
  }
}

template <bool STEP, bool COUNT = false>
__global__ void __launch_bounds__(256) reduce_kernel(DevState s, const int64_t* __restrict__ aoff,
                                                     int64_t n_bound, int n_from_aoff, double* acc, double* jerk,
                                                     double* pot, int64_t stride, int par, int64_t target_items) {
  __shared__ double wave_min[256 / 64];
  __shared__ int32_t wave_cnt[256 / 64];
  __shared__ double wave_sum[7][256 / 64];
  __shared__ int64_t offs_sh[kLdsClusters];
  const int tid = threadIdx.x;
  const int64_t n_active = n_from_aoff ? aoff[s.nc] : n_bound;
  // step pipeline with one cluster: the plan follows from this step's count
  const bool single = STEP && s.nc == 1;
  Plan P1{};
  int64_t units;
  if (single) {
    P1 = plan_single(s, par, target_items);
    units = plan_units(P1);
  } else {
    units = s.ctl->total_red;
  }
  if (single && blockIdx.x == 0 && tid == 0) {
    // the previous step's count is read by now (force and reduction of that
    // step, this step's selection): clear it for the next step's selection,
    // which counts into that half; then the block-step counters
    s.acount[par ^ 1] = 0;
    if (P1.n_act > 0) {
      s.inter[0] += (double)P1.n_act * (double)s.n;
      s.steps[0] += 1;
    }
  }
  if constexpr (STEP) {
    if (single) {
      reduce_units<true, true, COUNT>(s, units, P1, n_active, acc, jerk, pot, stride, wave_min, wave_cnt, wave_sum,
                                      offs_sh);
      return;
    }
  }
  reduce_units<STEP, false, COUNT>(s, units, P1, n_active, acc, jerk, pot, stride, wave_min, wave_cnt, wave_sum,
                                   offs_sh);
}


// Entries listed past the clusters' active counts (n_active larger than the
// active offsets say) get zeros and the index status bit.
__global__ void __launch_bounds__(256) reduce_tail_kernel(DevState s, const int64_t* __restrict__ aoff,
                                                          int64_t n_active, double* acc, double* jerk,
                                                          double* pot) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_active) return;
  const int64_t listed = aoff[s.nc];
  if (aoff[0] == 0 && q < listed) return;
  set_status(s, ST_INDEX);
#pragma unroll
  for (int d = 0; d < 3; ++d) acc[d * n_active + q] = jerk[d * n_active + q] = 0.0;
  if (pot) pot[q] = 0.0;
}

hipError_t launch_reduce(const DevState& s, const int64_t* aoff, int64_t n_active, double* acc,
                         double* jerk, double* pot, hipStream_t st) {
  const int64_t g = (n_active + 255) / 256;
  hipLaunchKernelGGL(reduce_tail_kernel, dim3((unsigned)g), dim3(256), 0, st, s, aoff, n_active, acc, jerk, pot);
  hipLaunchKernelGGL(reduce_kernel<false>, dim3(kReduceGrid), dim3(256), 0, st, s, aoff, n_active, 0, acc, jerk,
                     pot, n_active, -1, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_reduce_correct_step(const DevState& s, bool pot, int par, int64_t target_items, bool counting,
                                      hipStream_t st) {
  // pot only flags whether the potential row exists; the step writes s.pot.
  // The active list holds each cluster's block in its own segment, so every
  // entry index is below n.
  if (counting)
    hipLaunchKernelGGL((reduce_kernel<true, true>), dim3(kReduceGrid), dim3(256), 0, st, s, s.aoff, s.n, 0,
                       (double*)nullptr, (double*)nullptr, pot ? s.pot : nullptr, (int64_t)0, par, target_items);
  else
    hipLaunchKernelGGL((reduce_kernel<true, false>), dim3(kReduceGrid), dim3(256), 0, st, s, s.aoff, s.n, 0,
                       (double*)nullptr, (double*)nullptr, pot ? s.pot : nullptr, (int64_t)0, par, target_items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Power-of-two steps.

// Largest power of two not above x, for positive finite x (exactly: keep the
// exponent, clear the mantissa).  Subnormal x gives 0.
__device__ __forceinline__ double pow2_floor(double x) {
  return __longlong_as_double(__double_as_longlong(x) & 0x7FF0000000000000LL);
}

__device__ __forceinline__ double norm3(double a, double b, double c) { return sqrt(a * a + b * b + c * c); }

// New step from the criterion dt_raw (Sect. 2.1 block rule, read as: shrink
// freely; double at most once, only when t_now is a multiple of 2 dt_old;
// cap at dt_max; flag steps below dt_min).
__device__ __forceinline__ double quantize(double dt_raw, double dt_old, double t_now, double dt_max,
                                           double dt_min, int32_t* st) {
  if (isnan(dt_raw) || !isfinite(dt_old)) {
    *st |= ST_NONFINITE;
    return dt_old;
  }
  if (!(dt_raw > 0.0)) {
    *st |= ST_DTMIN;
    return dt_old;
  }
  double dn = isinf(dt_raw) ? dt_max : pow2_floor(dt_raw);
  if (dn < dt_old) {
    // t_now is a multiple of dt_old, hence of any smaller power of two
  } else {
    const double q = t_now / (2.0 * dt_old);  // exact: division by a power of two
    dn = (dn >= 2.0 * dt_old && q == floor(q)) ? 2.0 * dt_old : dt_old;
  }
  if (dn > dt_max) dn = dt_max;
  if (dn < dt_min) *st |= ST_DTMIN;
  return dn;
}

__global__ void __launch_bounds__(256) init_steps_kernel(DevState s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int64_t n = s.n;
  const Ctl ctl = *s.ctl;
  double a[3], k[3];
  int32_t st = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = s.fout[d * n + i];
    k[d] = s.fout[(3 + d) * n + i];
    s.a[d * n + i] = a[d];
    s.k[d * n + i] = k[d];
    if (!isfinite(a[d]) || !isfinite(k[d])) st |= ST_NONFINITE;
  }
  const double na = norm3(a[0], a[1], a[2]), nk = norm3(k[0], k[1], k[2]);
  double dt;
  if (nk == 0.0) {
    dt = ctl.dt_max;
  } else {
    const double raw = ctl.eta_init * na / nk;
    if (!(raw > 0.0) || !isfinite(raw)) {
      st |= (raw == 0.0) ? ST_DTMIN : ST_NONFINITE;
      dt = ctl.dt_min;
    } else {
      dt = pow2_floor(raw);
    }
  }
  if (dt > ctl.dt_max) dt = ctl.dt_max;
  if (dt < ctl.dt_min) st |= ST_DTMIN;
  s.t[i] = 0.0;
  s.dt[i] = dt;
  if (st) set_status(s, st);
}

hipError_t launch_init_steps(const DevState& s, hipStream_t st) {
  hipLaunchKernelGGL(init_steps_kernel, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hermite corrector (Sect. 2.1, corrector equations), Aarseth's criterion
// (Eq. timestep) with the end-of-step quantities, and quantisation.
// Entry q of the active list advances particle act[q] to tpred of its
// cluster.
// One particle: corrector, new step, state update.  i: particle, c: its
// cluster, first: whether this entry is the cluster's first of the block
// (it records the cluster's new time), in: its stored state (load_corr).
__device__ __forceinline__ double correct_one(const DevState& s, const Ctl& ctl, int c, int64_t i, bool first,
                                              const double a1[3], const double k1[3], const CorrIn& in) {
  const int64_t n = s.n;
  const double t_new = s.tpred[c];
  const double h = t_new - in.t;
  int32_t st = 0;
  if (!(h > 0.0)) {
    set_status(s, ST_STATE);
    return in.t + in.dt;
  }
  const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
  double a2[3], a3[3], a2p[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t o = d * n + i;
    const double a0 = in.a0[d], k0 = in.k0[d];
    const double da = a0 - a1[d];
    a2[d] = -6.0 * da / h2 - (4.0 * k0 + 2.0 * k1[d]) / h;
    a3[d] = 12.0 * da / h3 + 6.0 * (k0 + k1[d]) / h2;
    const double xn = in.xp[d] + a2[d] * h4 / 24.0 + a3[d] * h5 / 120.0;
    const double vn = in.vp[d] + a2[d] * h3 / 6.0 + a3[d] * h4 / 24.0;
    if (!isfinite(xn) || !isfinite(vn) || !isfinite(a1[d]) || !isfinite(k1[d])) st |= ST_NONFINITE;
    s.x[o] = xn;
    s.v[o] = vn;
    s.a[o] = a1[d];
    s.k[o] = k1[d];
    a2p[d] = a2[d] + a3[d] * h;
  }
  const double na = norm3(a1[0], a1[1], a1[2]);
  const double nk = norm3(k1[0], k1[1], k1[2]);
  const double na2 = norm3(a2p[0], a2p[1], a2p[2]);
  const double na3 = norm3(a3[0], a3[1], a3[2]);
  const double den = nk * na3 + na2 * na2;
  const double raw = den == 0.0 ? INFINITY : sqrt(ctl.eta * (na * na2 + nk * nk) / den);
  const double dt_new = quantize(raw, in.dt, t_new, ctl.dt_max, ctl.dt_min, &st);
  s.dt[i] = dt_new;
  s.t[i] = t_new;
  if (first) s.tnow[c] = t_new;
  if (st) set_status(s, st);
  return t_new + dt_new;
}

// Corrector for a caller's active list with its acc/jerk ([3][n_active]).
__global__ void __launch_bounds__(256) correct_kernel(DevState s, const int32_t* __restrict__ act,
                                                      const int64_t* __restrict__ aoff, int64_t n_active,
                                                      const double* __restrict__ acc,
                                                      const double* __restrict__ jerk) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_active) return;
  const int nc = s.nc;
  const Ctl ctl = *s.ctl;
  // cluster of entry q: last c with aoff[c] <= q
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (aoff[mid] <= q) lo = mid; else hi = mid - 1;
  }
  const int c = lo;
  if (q >= aoff[nc] || aoff[0] != 0) {  // n_active disagrees with the active offsets
    set_status(s, ST_INDEX);
    return;
  }
  const int64_t i = act[q];
  if (i < s.coff[c] || i >= s.coff[c + 1]) {
    set_status(s, ST_INDEX);
    return;
  }
  double a1[3], k1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a1[d] = acc[d * n_active + q];
    k1[d] = jerk[d * n_active + q];
  }
  correct_one(s, ctl, c, i, q == aoff[c], a1, k1, load_corr(s, i));
}

hipError_t launch_correct(const DevState& s, const int32_t* act, const int64_t* aoff, int64_t n_active,
                          const double* acc, const double* jerk, hipStream_t st) {
  const int64_t g = (n_active + 255) / 256;
  hipLaunchKernelGGL(correct_kernel, dim3((unsigned)g), dim3(256), 0, st, s, act, aoff, n_active, acc, jerk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block selection (Sect. 2.1: the particles with the smallest t_i + dt_i)
// and prediction in one kernel per block step, one workgroup per selection
// chunk of kSelChunk particles, then (several clusters) the plan of the
// force pass.
//
// The block time of cluster c is the minimum of t + dt over its particles.
// It is not recomputed by a pass of its own: the previous step left it in
// two pieces, the smallest t + dt of the particles it did not select (per
// chunk, cm2, written here) and the smallest new t + dt of the particles it
// corrected (per reduce unit, umin, written by the reduce kernel), and every
// workgroup of the cluster takes the minimum of both.  Members (t + dt equal
// to the block time; times are dyadic, so the test is exact) are appended to
// the cluster's own segment of the active list (starting at coff[c]) through
// an atomic counter; their order there does not change any particle's sums.
// Every particle of an advancing cluster is predicted.  A cluster whose
// block time is past t_end takes no step, and none does once the status word
// holds an error.
//
// The chunk minima (cm2) and the counters (acount) have one half per step
// parity `par`, a launch argument that the captured graphs alternate: step k
// reads cm2[par] and writes cm2[par ^ 1], counts into acount[par], and the
// previous step's counts stay readable in acount[par ^ 1] until the
// reduction of step k clears them for step k + 1.  So no kernel has to hand
// a device-side parity on, and with a single cluster no plan kernel runs at
// all: force and reduction derive the plan from acount[par].  (Planning
// inside this kernel by the last workgroup to take an atomic ticket was
// measured 70 us per step slower on a 256-cluster batch than the separate
// launch: every workgroup then needs a device-scope fence before its ticket.)

__device__ __forceinline__ double block_min(double v, double* buf) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = buf[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmin(r, buf[w]);
  return r;
}

// Start of a run of steps (after the state or the plan changed outside the
// step pipeline): cm2 = the chunk minima of t + dt, cm2n = how many
// particles of the chunk have that t + dt, no corrected particles.
__global__ void __launch_bounds__(kSelThreads) select_init_kernel(DevState s, int par) {
  __shared__ double buf[kSelThreads / 64];
  __shared__ int32_t nbuf[kSelThreads / 64];
  const int ch = blockIdx.x;
  const int c = s.ch_cluster[ch];
  const int64_t b = s.ch_begin[ch], e = s.ch_begin[ch + 1];
  double mn = INFINITY;
  int32_t cnt = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += kSelThreads) min_count(mn, cnt, s.t[i] + s.dt[i], 1);
  mn = block_min_count(mn, cnt, buf, nbuf);
  if (threadIdx.x == 0) {
    s.cm2[par * s.nch + ch] = mn;
    s.cm2n[par * s.nch + ch] = cnt;
    if (ch == s.cl_ch[c]) {
      s.plan[c].n_act = 0;
      s.acount[c] = 0;
      s.acount[s.nc + c] = 0;
    }
  }
}

// Layout of a block of na members of cluster c (the same decision as the
// plan's).
__device__ __forceinline__ int block_variant(const DevState& s, int c, int64_t na) {
  int32_t vmin_all[2 * (kNumVariants - 1) + 1];
  load_thresholds(s.ctl, vmin_all);
  return plan_variant(na, s.coff[c + 1] - s.coff[c], vmin_all);
}

template <bool COUNT>
__global__ void __launch_bounds__(kSelThreads) select_kernel(DevState s, int mode, int par, int64_t target_items) {
  static_assert(kSelChunk == kSelThreads, "one particle per thread");
  __shared__ double buf[kSelThreads / 64];
  __shared__ int32_t nbuf[kSelThreads / 64];
  __shared__ int64_t sbuf[kSelThreads / 64];
  __shared__ int64_t base_sh;
  const int ch = blockIdx.x;
  const int c = s.ch_cluster[ch];
  const int tid = threadIdx.x;
  const double* cur = s.cm2 + (int64_t)par * s.nch;
  double* nxt = s.cm2 + (int64_t)(par ^ 1) * s.nch;
  const int32_t* curn = s.cm2n + (int64_t)par * s.nch;
  int32_t* nxtn = s.cm2n + (int64_t)(par ^ 1) * s.nch;

  // this thread's particle: its t + dt and (for a cluster that has not
  // reached the end time) the predictor's inputs do not depend on the block
  // time, so they are loaded first and their latency overlaps that of the
  // block-time reduction
  const int64_t i = s.ch_begin[ch] + tid;
  const bool have = i < s.ch_begin[ch + 1];
  const bool ahead = s.tnow[c] < s.ctl->t_end;
  // plan of the previous step (the other parity)
  const Plan P = s.nc == 1 ? plan_single(s, par ^ 1, target_items) : s.plan[c];
  if (!ahead && P.n_act == 0) {
    // the cluster has reached the end time (so it takes no step: every
    // particle is at t_end) and took none last step either: the chunk's
    // minimum of t + dt is unchanged, nothing else to do
    if (tid == 0) {
      nxt[ch] = cur[ch];
      nxtn[ch] = curn[ch];
    }
    return;
  }
  double tt = INFINITY;
  PredIn pin{};
  if (have) {
    if (ahead) pin = load_pred(s, i);
    else pin.t = s.t[i];
    tt = pin.t + s.dt[i];
  }

  // block time of cluster c and, where it decides whether the tile frames
  // are formed (COUNT: tile-relative format with some cluster that can
  // reach the one-lane-per-i layout; the same for every step between two
  // initialisations), the size of its block: a particle at the block time
  // is either one the last selection left out (counted per chunk at the
  // chunk's minimum) or one the last step corrected (counted per reduce
  // unit at the unit's minimum), so the sizes of the minima equal to the
  // block time add up to the block size
  double mn = INFINITY;
  int32_t nblock = 0;
  const int64_t epw = 256 / P.red_tp;
  const int64_t units = P.n_act > 0 ? (P.n_act + epw - 1) / epw : 0;
  double tsys;
  if constexpr (COUNT) {
    for (int f = s.cl_ch[c] + tid; f < s.cl_ch[c + 1]; f += kSelThreads) min_count(mn, nblock, cur[f], curn[f]);
    for (int64_t u = tid; u < units; u += kSelThreads)
      min_count(mn, nblock, s.umin[P.red_off + u], s.ucnt[P.red_off + u]);
    tsys = block_min_count(mn, nblock, buf, nbuf);
  } else {
    for (int f = s.cl_ch[c] + tid; f < s.cl_ch[c + 1]; f += kSelThreads) mn = fmin(mn, cur[f]);
    for (int64_t u = tid; u < units; u += kSelThreads) mn = fmin(mn, s.umin[P.red_off + u]);
    tsys = block_min(mn, buf);
  }
  // an error recorded on the device (step underflow, non-finite value, bad
  // index) freezes the state: no cluster advances, so this step and every
  // later one select nothing and change nothing; the status word was written
  // by earlier kernels only, so every workgroup reads the same value
  const bool frozen = *s.status != 0;
  const bool advancing = !frozen && tsys <= s.ctl->t_end;
  const bool member = have && advancing && tt == tsys;
  // with the block size known: its layout, and whether the force pass
  // predicts its j-records itself (fused_prediction; the formats whose
  // j-split layouts read only x_p, v_p), in which case only the members
  // are predicted here
  const int var = COUNT ? block_variant(s, c, nblock) : 0;
  const int64_t iwg = variant_iwg(var);
  const bool fuse = COUNT && advancing && (mode == kF64 || mode == kTR) &&
                    fused_prediction(s.ctl->pred_in_force, var, (nblock + iwg - 1) / iwg);
  double xo[3] = {0.0, 0.0, 0.0}, vo[3] = {0.0, 0.0, 0.0};
  if (have && advancing && (member || !fuse))
    predict_from(s, i, ahead ? pin : load_pred(s, i), tsys, mode, member, xo, vo);
  // the mixed force pass reads the tile frame of every chunk of an
  // advancing cluster (the condition is the same for the whole workgroup);
  // the tile-relative mode only when this block takes a one-lane-per-i
  // layout (its split layouts run the FP64 arithmetic)
  if (advancing && mode != kF64 && (mode != kTR || (COUNT && var <= 1)))
    tile_frame(s, ch, have, xo, vo, have ? s.m[i] : 0.0, tsys);

  // members, and the smallest t + dt of the others (with their number)
  int32_t nrest = have && !member ? 1 : 0;
  double rest;
  if constexpr (COUNT)
    rest = block_min_count(member ? INFINITY : tt, nrest, buf, nbuf);
  else
    rest = block_min(member ? INFINITY : tt, buf);
  int64_t total;
  const int64_t before = wg_exclusive_scan(member ? 1 : 0, sbuf, &total);
  if (tid == 0) {
    nxt[ch] = rest;
    if (COUNT) nxtn[ch] = nrest;
    base_sh = total > 0 ? atomicAdd(&s.acount[(int64_t)par * s.nc + c], (int32_t)total) : 0;
    if (advancing) {
      s.tpstamp[ch] = fuse ? __builtin_nan("") : tsys;
      if (ch == s.cl_ch[c]) s.tpred[c] = tsys;
    }
  }
  __syncthreads();
  if (member) s.act[s.coff[c] + base_sh + before] = (int32_t)i;
}

// Plan of the step's force pass from the selection counts (one workgroup),
// then this parity's counters are cleared for the step after next.
__global__ void __launch_bounds__(256) plan_step_kernel(DevState s, int64_t target_items, int32_t* counts) {
  plan_body(s, nullptr, s.n, target_items, 1, counts);
  __syncthreads();
  for (int c = threadIdx.x; c < s.nc; c += 256) counts[c] = 0;  // read: cleared for the step after next
}

hipError_t launch_select_init(const DevState& s, int par, hipStream_t st) {
  hipLaunchKernelGGL(select_init_kernel, dim3(s.nch), dim3(kSelThreads), 0, st, s, par);
  return hipGetLastError();
}

hipError_t launch_select(const DevState& s, int64_t target_items, int mode, int par, bool counting, hipStream_t st) {
  if (counting)
    hipLaunchKernelGGL(select_kernel<true>, dim3(s.nch), dim3(kSelThreads), 0, st, s, mode, par, target_items);
  else
    hipLaunchKernelGGL(select_kernel<false>, dim3(s.nch), dim3(kSelThreads), 0, st, s, mode, par, target_items);
  if (s.nc == 1) return hipGetLastError();  // the force and reduce kernels plan for themselves
  int32_t* counts = s.acount + (int64_t)par * s.nc;
  if (s.nc <= 64)
    hipLaunchKernelGGL(plan_small_kernel, dim3(1), dim3(64), 0, st, s, (const int64_t*)nullptr, s.n, target_items,
                       1, counts);
  else
    hipLaunchKernelGGL(plan_step_kernel, dim3(1), dim3(256), 0, st, s, target_items, counts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mean relative error of the FP32 hardware reciprocal square root.  One
// workgroup evaluates v_rsq_f32 at 65536 arguments spread log-uniformly over
// [1, 4) (its error pattern repeats every two binades), compares each with
// 1/sqrt in FP64 (v_rsq_f64 estimate plus a third-order Newton step, exact
// to FP64 rounding), and averages the relative errors in a fixed order.
__global__ void __launch_bounds__(256) rsq_bias_kernel(Ctl* ctl, int correct) {
  __shared__ double red[256];
  constexpr int kSamples = 65536;
  double acc = 0.0;
  for (int q = threadIdx.x; q < kSamples; q += 256) {
    const double t = ((double)q + 0.5) / kSamples;
    const float x = (float)exp2(2.0 * t);  // log-uniform on [1, 4)
    const double xd = (double)x;
    double y = __builtin_amdgcn_rsq(xd);
    const double e = __builtin_fma(-(xd * y), y, 1.0);
    y = __builtin_fma(y * e, __builtin_fma(0.375, e, 0.5), y);
    const double yf = (double)__builtin_amdgcn_rsqf(x);
    acc += (yf - y) / y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double b = red[0] / kSamples;
    ctl->rsq_bias = b;
    ctl->rsq_scale3 = correct ? 1.0 - 3.0 * b : 1.0;
    ctl->rsq_scale1 = correct ? 1.0 - b : 1.0;
  }
}

hipError_t launch_rsq_bias(const DevState& s, int correct, hipStream_t st) {
  hipLaunchKernelGGL(rsq_bias_kernel, dim3(1), dim3(256), 0, st, s.ctl, correct);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-cluster softened energy, E = sum m v^2 / 2 + (1/2) sum m phi, from the
// potential row of s.fout (identity active list).  Fixed-order sums.
// Per-cluster diagnostics at the prediction time (Sect. 2.1, diagnostic
// output), FP64, one workgroup per cluster: out[8 c + ...] = kinetic energy
// sum m v^2 / 2, potential energy (1/2) sum m phi (phi from s.fout's
// potential row, self pair excluded), momentum sum m v (3), angular momentum
// sum m x cross v (3).  Positions and velocities are the predicted ones
// (equal to x, v when every particle is at the cluster's time).
__global__ void __launch_bounds__(256) diag_kernel(DevState s, double* out) {
  __shared__ double red[8][256];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t n = s.n;
  const int64_t b = s.coff[c], e = s.coff[c + 1];
  double acc[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) acc[d] = 0.0;
  for (int64_t i = b + tid; i < e; i += 256) {
    const double m = s.m[i];
    const double x = s.xp[i], y = s.xp[n + i], z = s.xp[2 * n + i];
    const double vx = s.vp[i], vy = s.vp[n + i], vz = s.vp[2 * n + i];
    acc[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    acc[1] += 0.5 * m * s.fout[6 * n + i];
    acc[2] += m * vx;
    acc[3] += m * vy;
    acc[4] += m * vz;
    acc[5] += m * (y * vz - z * vy);
    acc[6] += m * (z * vx - x * vz);
    acc[7] += m * (x * vy - y * vx);
  }
#pragma unroll
  for (int d = 0; d < 8; ++d) red[d][tid] = acc[d];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
#pragma unroll
      for (int d = 0; d < 8; ++d) red[d][tid] += red[d][tid + off];
    }
    __syncthreads();
  }
  if (tid < 8) out[8 * c + tid] = red[tid][0];
}

hipError_t launch_diag(const DevState& s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(diag_kernel, dim3(s.nc), dim3(256), 0, st, s, out);
  return hipGetLastError();
}

}  // namespace nb
