// Launchers of libnbody's kernels (host side, internal).
#pragma once

#include "common.h"

namespace nb {

// Pairwise arithmetic modes of the force kernel.
enum : int { kF64 = 0, kDS = 1, kMX64 = 2, kTR = 3 };

// Selection chunk: particles per workgroup of the block-selection kernels.
constexpr int kSelChunk = 256;
constexpr int kSelThreads = 256;

// Force: every work item of the current plan, persistent grid of `grid`
// workgroups.  act: the active list the plan was made for.  pot: also sum
// the potential (partial row 6).  near: mixed modes evaluate pairs with
// m_j / R^2 > ctl->near_tau |a_i| in FP64.  split: the kernel with only the
// layouts that split j over lanes (higher occupancy); valid only when no
// cluster can reach a one-lane-per-i layout.  par: step parity in the step
// pipeline (with a single cluster the plan then comes from that parity's
// selection count and target_items), -1 for the plan in s.plan.  lean: the
// tile-relative near build without the masked sweep (every cluster's
// softening keeps the self pair finite in FP32; see force_impl.h).  window,
// waves, tile: FP32 window (16, 32, 64), waves per SIMD (2 to 5) and
// j-records per LDS tile (128 or 256) of the lean tile-relative kernel
// without the potential; other kernels use 32, their own occupancy and 256.
// pif: the build with the fused predictor (step pipeline only; there must
// be one for these arguments: has_pif_build).
hipError_t launch_force(const DevState& s, int mode, bool pot, bool near, bool split, bool lean, const int32_t* act,
                        int grid, int par, int64_t target_items, hipStream_t st, int window = 32, int waves = 4,
                        int tile = 256, bool pif = false);
bool has_pif_build(int mode, bool pot, bool near, bool split, bool lean, int window, int waves, int tile);

// Plan the force pass for the active offsets `aoff` (device, nc+1) of an
// active list of at most n_act_bound entries.  target_items: work items aimed
// at (fills the GPU); rows of partial sums are bounded by s.rows_cap.
// count_stats: add the pass to the per-cluster step / interaction counters.
hipError_t launch_plan(const DevState& s, const int64_t* aoff, int64_t n_act_bound, int64_t target_items,
                       hipStream_t st, int count_stats = 0);

// Persistent grid of the slice reduction.
constexpr int kReduceGrid = 2048;

// Sum the slice partials of every active entry into acc/jerk/pot
// ([3][n_active], [3][n_active], [n_active] or NULL).
hipError_t launch_reduce(const DevState& s, const int64_t* aoff, int64_t n_active, double* acc,
                         double* jerk, double* pot, hipStream_t st);

// Step pipeline: the same for the active list built by the selection, each
// sum handed straight to the corrector (pot: keep phi); records the smallest
// new t + dt per reduce unit for the next selection and clears the
// selection counters of the other parity.  par, target_items: as for
// launch_force; counting: as for launch_select (also records how many
// particles of a unit have its smallest t + dt).
hipError_t launch_reduce_correct_step(const DevState& s, bool pot, int par, int64_t target_items, bool counting,
                                      hipStream_t st);

// Perturber lists (perturbers.hip): for each entry q of the caller's
// active list (particle ids, cluster c's entries at aoff[c] .. aoff[c+1]),
// the ids j != i of its cluster with m_j / (|x_p,j - x_p,i|^2 + eps_c^2) >
// thr[c] in ascending order, the first cap of them in lists[q * cap ...]
// (-1 past the end) and their number in counts[q].  An id outside its
// cluster sets ST_INDEX and gets an empty list.
hipError_t launch_perturbers(const DevState& s, const int32_t* ids, const int64_t* aoff, int64_t n_active,
                             const double* thr, int32_t cap, int32_t* lists, int32_t* counts, hipStream_t st);

// Predict every particle of every cluster to s.tpred[c] (FP64 x_p, v_p,
// every field of the mixed j-records and the tile frames).
hipError_t launch_predict_all(const DevState& s, hipStream_t st);

// A caller's active list of particle ids mapped to slots (s.ulist);
// ids outside [0, n) map to -1, which the force pass reports.
hipError_t launch_map_active(const DevState& s, const int32_t* ids, int64_t n_active, hipStream_t st);

// Write the identity active list (act[i] = i, aoff = coff).
hipError_t launch_identity(const DevState& s, hipStream_t st);

// Start-up: a, k from s.fout, t = 0, dt from the initial rule.
hipError_t launch_init_steps(const DevState& s, hipStream_t st);

// Corrector + time step for an active list with its acc/jerk ([3][n_active]).
hipError_t launch_correct(const DevState& s, const int32_t* act, const int64_t* aoff, int64_t n_active,
                          const double* acc, const double* jerk, hipStream_t st);


// Step pipeline: block selection with the predictor (one kernel), then,
// with several clusters, the plan of the force pass (count_stats on).  par:
// the step's parity (0 or 1), alternating from step to step.
// launch_select_init (with the parity of the next step) must run first, and
// again whenever t, dt or the plan changed outside the step pipeline.
hipError_t launch_select_init(const DevState& s, int par, hipStream_t st);
// mode: force mode of the step (the predictor writes only what it reads).
// counting: derive each cluster's block size before the predictor runs, so
// that the tile-relative frames are formed only for blocks that take the
// one-lane-per-i layout (needed when some cluster can reach that layout;
// must stay the same from launch_select_init to the next one).
hipError_t launch_select(const DevState& s, int64_t target_items, int mode, int par, bool counting, hipStream_t st);

// Mean relative error b of the FP32 hardware reciprocal square root over
// log-uniform arguments in [1, 4); sets ctl->rsq_scale3 = 1 - 3b and
// ctl->rsq_scale1 = 1 - b (or both to 1 when correct == 0).
hipError_t launch_rsq_bias(const DevState& s, int correct, hipStream_t st);

// Per-cluster diagnostics (8 per cluster: kinetic and potential energy,
// momentum, angular momentum) from the predicted state and s.fout's
// potential row (identity active list).
hipError_t launch_diag(const DevState& s, double* out, hipStream_t st);

}  // namespace nb
