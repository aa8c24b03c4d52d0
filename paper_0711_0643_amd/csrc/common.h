// Shared device-side definitions of libnbody (gfx950).
//
// Everything the kernels read or write lives in the caller-owned workspace;
// DevState carries the pointers into it.  Vector arrays are
// structure-of-arrays FP64: component d of particle i is at [d * n + i].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

// Device status bits, OR-ed into DevState::status by kernels and mapped to
// nbody_status on the host (first set bit in this order wins).
enum : int32_t {
  ST_INDEX = 1,      // active index outside its cluster / bad active offsets
  ST_NONFINITE = 2,  // non-finite x, v, a or k, or NaN step criterion
  ST_DTMIN = 4,      // new step below dt_min
  ST_STATE = 8,      // corrector asked to step by a non-positive time, a force work item of a layout the launched
                     // kernel lacks, or a tile frame formed for another time than its cluster's prediction
};

// Batches of up to this many clusters look up the cluster of a work item in
// a copy of the plan offsets in LDS.
constexpr int kLdsClusters = 1024;
// Threads per workgroup of every force launch; the i x j layout of a
// workgroup is (256 / JL) i-slots times JL j-lanes.
constexpr int kForceThreads = 256;
// j-records staged in LDS per tile.
constexpr int kTile = 256;
// Largest total particle count: keeps every per-cluster count and slice
// length of the plan (int32) far from overflow.  (The workspace of that many
// particles, mostly partial rows, would exceed any GPU's memory anyway.)
constexpr int64_t kMaxParticles = (int64_t)1 << 30;
// Blocks of at least this many entries are reduced with one lane per entry.
constexpr int64_t kReduceSerialBlock = 2048;
// Largest slicing target a plan may be asked for.
constexpr int64_t kMaxTargetItems = 16384;
// Partial-row budget: a cluster of N particles may use up to
// kRowsPerParticle * N + kRowsPerCluster rows of slice partials.
constexpr int64_t kRowsPerParticle = 32;
constexpr int64_t kRowsPerCluster = 4096;
// Variants of the i x j layout, indexed by Plan::variant: lanes per i (JL)
// and i per lane (IPT).  v0: 1 lane, 2 i; v1: 1 lane, 1 i; v2: 4 lanes;
// v3: 16 lanes; v4: 64 lanes.
constexpr int kNumVariants = 5;
__host__ __device__ constexpr int variant_jl(int v) { return v <= 1 ? 1 : v == 2 ? 4 : v == 3 ? 16 : 64; }
__host__ __device__ constexpr int variant_ipt(int v) { return v == 0 ? 2 : 1; }
__host__ __device__ constexpr int variant_iwg(int v) { return kForceThreads / variant_jl(v) * variant_ipt(v); }

// Mixed j-record in HBM: ten FP32 rows of n entries each.
enum : int { JR_HX = 0, JR_HY, JR_HZ, JR_LX, JR_LY, JR_LZ, JR_VX, JR_VY, JR_VZ, JR_M, JR_ROWS };

// Per-tile frame of the tile-relative mixed mode, one entry of kTileMeta
// doubles per selection chunk (= LDS tile of kTile slots): the centre of the
// bounding box of the predicted positions (origin of the FP32 relative
// coordinates), the centre of the bounding box of the predicted velocities,
// the half-diagonal of that velocity box (no velocity of the tile is farther
// from the centre), the largest mass, the half-diagonal of the position box
// (no position of the tile is farther from the origin), and the time the
// particles were predicted to when the frame was formed.
enum : int { TM_OX = 0, TM_OY, TM_OZ, TM_VX, TM_VY, TM_VZ, TM_W, TM_MMAX, TM_D, TM_T, kTileMeta };

// Per-cluster force plan, written by the plan kernel.
struct Plan {
  int64_t item_off;   // first work item of this cluster
  int64_t slot_base;  // first partial row of this cluster
  int64_t act_off;    // first entry of this cluster in the active list
  int32_t n_act;      // active particles in this cluster
  int32_t variant;    // i x j layout (index into variant_jl)
  int32_t chunks;     // i-chunks of variant_iwg(variant) active particles
  int32_t slices;     // j-slices
  int32_t slice_len;  // j per slice (multiple of kTile; clusters hold at most kMaxParticles)
  int32_t red_tp;     // reduce: lanes per entry (power of two, <= 256)
  int64_t red_off;    // reduce: first work unit of this cluster
};

// Control block read by the captured step graph (so one graph serves any
// t_end) and per-cluster counters.
struct Ctl {
  double t_end;
  double eta, eta_init, dt_max, dt_min;
  int32_t compute_pot;
  // blocks that fill a single i-chunk of a layout splitting j over lanes
  // are predicted in the force pass (fused_prediction)
  int32_t pred_in_force;
  int64_t total_items;  // items of the current plan
  int64_t total_rows;   // partial rows of the current plan
  int64_t total_red;    // reduce work units of the current plan
  // plan tuning: smallest block size for variants 0..3 (else variant 4)
  int32_t vmin[kNumVariants - 1];
  // the same for clusters of fewer than small_n particles
  int32_t vmin_small[kNumVariants - 1];
  int64_t small_n;
  // mixed kernel: pairs with m_j / R^2 > near_tau |a_i|, or whose jerk term
  // may exceed near_tau_k |k_i|, are done in FP64
  double near_tau;
  double near_tau_k;
  // tile-relative mixed mode: a window whose closest pair has
  // term * (L / R) above mid_tau |a_i| or |k_i| is summed again with FP64
  // position differences (L: distance scale of the tile frame)
  double mid_tau;
  // FP64 factors applied to the FP32 windows of the mixed kernel (bias of
  // the hardware reciprocal square root removed): R^-3 terms, R^-1 terms
  double rsq_scale3;
  double rsq_scale1;
  double rsq_bias;  // measured mean relative error of v_rsq_f32
  int32_t pad3[2];
};

// Particles are stored in "slot" order: inside each cluster the library
// sorts them along a Morton curve of their initial positions, so that the
// kTile consecutive slots of an LDS tile are close in space.  The caller's
// particle ids map to slots through slot_of; order maps back.  Every state
// array of DevState is indexed by slot.
struct DevState {
  int64_t n;          // particles, all clusters
  int32_t nc;         // clusters
  int32_t nch;        // selection chunks
  const int64_t* coff;  // [nc+1] cluster offsets
  const double* eps;    // [nc] softening
  const int32_t* cid;   // [n] cluster of each particle
  const int32_t* ch_cluster;  // [nch] cluster of each selection chunk
  const int64_t* ch_begin;    // [nch+1] first particle of each chunk (ch_begin[nch] = n)
  const int32_t* cl_ch;       // [nc+1] first selection chunk of each cluster
  int32_t* order;             // [n] particle id stored at each slot
  int32_t* slot_of;           // [n] slot of each particle id
  double* tmeta;              // [nch][kTileMeta] tile frames (tile-relative mixed mode)
  int32_t* ulist;             // [n] a caller's active list mapped to slots
  double* m;
  double* x;
  double* v;
  double* a;
  double* k;
  double* t;
  double* dt;
  double* xp;
  double* vp;
  double* pot;     // [n] potential of the last block (when kept)
  float* jr;       // [JR_ROWS][n] mixed j-records
  double* tpred;   // [nc] time of the last prediction
  double* tnow;    // [nc] time of the last block step
  double* inter;   // [nc] pairwise interactions evaluated
  int64_t* steps;  // [nc] block steps taken
  double* cm2;     // [2][nch] per chunk: smallest t + dt of the particles the last selection left out
  int32_t* cm2n;   // [2][nch] per chunk: how many of those particles have that t + dt
  int32_t* acount; // [2][nc] block size of each cluster (selection counters, one half per step parity)
  double* umin;    // [n] per reduce unit: smallest new t + dt of the particles it corrected
  int32_t* ucnt;   // [n] per reduce unit: how many of those particles have that t + dt
  int32_t* act;    // [n] active list (step pipeline: cluster c's block at act[coff[c]...])
  int64_t* aoff;   // [nc+1] active offsets of the internal all-particle passes
  Plan* plan;      // [nc]
  int64_t* offs;   // [2][nc] item_off and red_off of the plan, contiguous (cluster lookup in LDS)
  Ctl* ctl;
  double* part;    // [7][rows_cap] partial sums
  int64_t rows_cap;
  double* fout;    // [7][n] reduced force of internal passes (a, k, pot)
  double* pid;     // [4][n] perturber pass: predicted x, y, z and mass in particle-id order
  int32_t* status;
  double* tpstamp;  // [nch] per chunk: time of the stored prediction (x_p, v_p) of all its particles, NaN
                    // when the selection predicted only the block's members (the force pass then predicts)
};

// Layout and slicing of a cluster of nn particles whose block has na
// members, from the layout thresholds vmin_all (min_block[0..3],
// small_min_block[0..3], small_cluster_n) and the slicing target: as many
// j-slices as bring the cluster alone to about target_items work items, at
// most one per LDS tile and at most what the cluster's partial-row budget
// allows.  Offsets (item_off, slot_base, act_off, red_off) are not set.
// Integer type T: every intermediate fits in it (32-bit divisions are much
// shorter than 64-bit ones, and this runs in kernel prologues).
// Layout of a block of na members in a cluster of nn particles: the lowest
// index whose threshold the block reaches (the last layout has none).
__host__ __device__ inline int plan_variant(int64_t na, int64_t nn, const int32_t* vmin_all) {
  const int32_t* vmin = nn < (int64_t)vmin_all[2 * (kNumVariants - 1)] ? vmin_all + (kNumVariants - 1) : vmin_all;
  int var = kNumVariants - 1;
  for (int vv = kNumVariants - 2; vv >= 0; --vv)
    if (na >= vmin[vv]) var = vv;
  return var;
}

template <typename T>
__host__ __device__ inline void plan_layout_t(T na, T nn, T target_items, const int32_t* vmin_all, Plan& P) {
  const int var = plan_variant((int64_t)na, (int64_t)nn, vmin_all);
  const T iwg = (T)variant_iwg(var);
  const T chunks = (na + iwg - 1) / iwg;
  T S = 1;
  if (chunks > 0) {
    const T smax_tiles = (nn + kTile - 1) / kTile;
    const T smax_rows = ((T)kRowsPerParticle * nn + (T)kRowsPerCluster) / na;
    S = (target_items + chunks - 1) / chunks;
    if (S > smax_tiles) S = smax_tiles;
    if (S > smax_rows) S = smax_rows;
    if (S < 1) S = 1;
  }
  T slen = (nn + S - 1) / S;
  slen = (slen + kTile - 1) / kTile * kTile;
  S = (nn + slen - 1) / slen;
  P.n_act = (int32_t)na;
  P.variant = var;
  P.chunks = (int32_t)chunks;
  P.slices = (int32_t)S;
  P.slice_len = (int32_t)slen;
  // reduce lanes per entry: for small blocks as many as there are slices
  // (summed in parallel, then by a tree); for large blocks one lane per
  // entry, which adds its slices in turn with coalesced loads and runs its
  // entry's corrector itself (no lanes idle during the corrector)
  int tp = 1;
  if ((int64_t)na < kReduceSerialBlock)
    while ((T)tp < S && tp < 256) tp <<= 1;
  P.red_tp = tp;
}

__host__ __device__ inline void plan_layout(int64_t na, int64_t nn, int64_t target_items, const int32_t* vmin_all,
                                            Plan& P) {
  // 32-bit when kRowsPerParticle * nn + kRowsPerCluster and every other
  // intermediate stays below 2^32
  if (nn < ((int64_t)1 << 26) && target_items < ((int64_t)1 << 30))
    plan_layout_t<uint32_t>((uint32_t)na, (uint32_t)nn, (uint32_t)target_items, vmin_all, P);
  else
    plan_layout_t<int64_t>(na, nn, target_items, vmin_all, P);
}

__device__ inline void load_thresholds(const Ctl* ctl, int32_t* vmin_all) {
#pragma unroll
  for (int v = 0; v < kNumVariants - 1; ++v) {
    vmin_all[v] = ctl->vmin[v];
    vmin_all[kNumVariants - 1 + v] = ctl->vmin_small[v];
  }
  vmin_all[2 * (kNumVariants - 1)] = (int32_t)(ctl->small_n < INT32_MAX ? ctl->small_n : INT32_MAX);
}

// Whether a block of layout `variant` in `chunks` i-chunks takes the fused
// predictor (Sect. 2.1: the prediction may run on the accelerator): the
// selection predicts only the block's members and the force pass forms each
// j-record from x, v, a, k and t itself.  Only the layouts that split j over
// lanes, and only a block that fills a single i-chunk, so that every j is
// predicted once per slice.
__host__ __device__ inline bool fused_prediction(int32_t enabled, int variant, int64_t chunks) {
  return enabled != 0 && variant >= 2 && chunks == 1;
}

// Hermite predictor of one coordinate to h = t_p - t (Sect. 2.1, predictor
// equations); every kernel that predicts calls this one expression, so
// that all of them round alike.
__device__ __forceinline__ void hermite_predict(double x, double v, double a, double k, double h, double& xp,
                                                double& vp) {
  xp = x + h * (v + h * (0.5 * a + h * (k * (1.0 / 6.0))));
  vp = v + h * (a + h * (0.5 * k));
}

// Reduce work units of a cluster's plan.
__host__ __device__ inline int64_t plan_units(const Plan& P) {
  const int64_t epw = 256 / P.red_tp;  // entries per unit
  return ((int64_t)P.n_act + epw - 1) / epw;
}

// The plan of the step pipeline when there is a single cluster: its block
// size is the selection counter of this step's parity, its offsets are 0.
// The selection, force and reduction kernels each compute it for
// themselves, so a step needs no plan kernel.
__device__ inline Plan plan_single(const DevState& s, int par, int64_t target_items) {
  int32_t vmin_all[2 * (kNumVariants - 1) + 1];
  load_thresholds(s.ctl, vmin_all);
  Plan P{};
  plan_layout(s.acount[par], s.n, target_items, vmin_all, P);
  return P;
}

// Index of the last of the nc ascending offsets that is <= x (offs[0] = 0).
__device__ inline int last_at_or_below(const int64_t* offs, int nc, int64_t x) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace nb
