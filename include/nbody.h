/*
 * nbody.h -- C ABI of libnbody, a direct-summation N-body engine for AMD
 * Instinct MI355X (gfx950).
 *
 * The library advances one or more independent star clusters with the
 * fourth-order Hermite predictor-corrector and power-of-two block time
 * steps described in Portegies Zwart, McMillan, Groen, Gualandris, Sipior &
 * Vermin, "A parallel gravitational N-body kernel" (New Astronomy, 2008),
 * Sect. 2.1.  Its hot path is the O(n_act * N) pairwise evaluation of
 * acceleration, jerk and potential on the active block against every
 * predicted particle of the same cluster.
 *
 * Conventions shared by every call:
 *   - G = 1; N-body units are expected but not enforced.
 *   - Particle arrays are structure-of-arrays FP64: a vector array v of n
 *     particles holds v[0*n+i], v[1*n+i], v[2*n+i] for the x, y, z
 *     components of particle i.  Outputs for an active list use n_active in
 *     place of n and follow the order of the active list.
 *   - Particles are numbered globally 0..n_total-1; cluster c owns the
 *     contiguous range [cluster_offsets[c], cluster_offsets[c+1]).  Clusters
 *     never interact.
 *   - Memory: the caller owns every device buffer, including the workspace
 *     that holds the whole simulation state.  The library never allocates or
 *     frees device memory; nbody_destroy frees only the host-side context.
 *   - Streams: every call that takes a context is enqueued on the context's
 *     HIP stream and returns before the GPU work finishes, unless stated.
 *     Host-side validation errors are returned synchronously and enqueue
 *     nothing.  Errors detected on the device (step underflow, non-finite
 *     values, out-of-range indices) are recorded in a status word in the
 *     workspace, returned by nbody_sync and by the next call that reads it.
 *     Once the status word holds an error, the state is frozen: every later
 *     block step of nbody_step selects nothing and leaves every array and
 *     counter bitwise unchanged, until nbody_set_state restores a state.
 *   - A context is bound to one stream and is not thread-safe.
 *
 * Readings of the paper the library implements (the paper does not spell
 * these out): the pair vector is x_j - x_i (Eq. Force prints the repulsive
 * sign); Plummer softening R^2 = |x_j - x_i|^2 + eps^2 in acceleration, jerk
 * and potential; the jerk is the exact time derivative of the softened
 * acceleration; phi_i = -sum_{j != i} m_j / R; Aarseth's criterion
 * (Eq. timestep) uses the end-of-step |a|, |a2 + a3 dt|, |k|, |a3|; new
 * steps are rounded down to a power of two, may shrink freely, at most
 * double and only when the current time is a multiple of the doubled step,
 * and are capped at dt_max; initial steps are eta_init |a|/|k| rounded down.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define NBODY_API __attribute__((visibility("default")))
#else
#define NBODY_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nbody_ctx nbody_ctx;

typedef enum {
    NBODY_OK = 0,
    NBODY_E_INVAL = -1,     /* bad argument (host-side validation)               */
    NBODY_E_NOMEM = -2,     /* workspace too small / host allocation failed      */
    NBODY_E_HIP = -3,       /* a HIP runtime call failed                         */
    NBODY_E_STATE = -4,     /* call out of order (e.g. correct before predict);
                               device: an internal inconsistency (a work item
                               of a layout its kernel build does not hold, a
                               tile frame formed for another time, a
                               corrector step that does not advance)          */
    NBODY_E_DTMIN = -5,     /* device: a new step fell below dt_min              */
    NBODY_E_NONFINITE = -6, /* device: non-finite position, velocity or force    */
    NBODY_E_INDEX = -7      /* device: active index outside its cluster or
                               active offsets not monotonic                      */
} nbody_status;

/* Arithmetic of the pairwise kernel.
 *   NBODY_FP64:  plain FP64 throughout.
 *   NBODY_MIXED: positions held in FP64 and differenced with FP64
 *                accuracy (tile-relative, FP64 or double-single, see
 *                nbody_tuning), pair terms in FP32, partial sums over short
 *                j-windows in FP32 flushed into FP64 totals, near pairs in
 *                FP64.  Predictor, corrector and time steps stay FP64 in
 *                both modes. */
typedef enum { NBODY_FP64 = 0, NBODY_MIXED = 1 } nbody_precision;

typedef struct {
    double eta;          /* Aarseth accuracy parameter nu (Sect. 2.1: 0.01)      */
    double eta_init;     /* initial step eta_init*|a|/|k| (0.01)                 */
    double dt_max;       /* largest step, a power of two (2^-3)                  */
    double dt_min;       /* smallest allowed step (2^-40); below: NBODY_E_DTMIN  */
    int32_t precision;   /* nbody_precision                                      */
    int32_t compute_pot; /* nonzero: nbody_step also keeps phi of the block      */
} nbody_params;

/* Fills *p with the defaults given in parentheses above (FP64, no pot). */
NBODY_API void nbody_default_params(nbody_params *p);

/* Bytes of device workspace needed for n_total particles in n_clusters
 * clusters.  Pure host computation; never fails for valid sizes
 * (n_total >= 1, 1 <= n_clusters <= n_total, n_total <= 2^30). */
NBODY_API nbody_status nbody_workspace_bytes(int64_t n_total, int32_t n_clusters, const nbody_params *p,
                                   size_t *bytes);

/* Creates a context and starts the integration (Sect. 2.1: every particle
 * gets a and k by direct summation, t_i = 0 and its initial step).
 *   cluster_offsets: host, n_clusters+1 ascending entries, [0] = 0,
 *                    [n_clusters] = n_total, every cluster non-empty.
 *   m (host, n_total), x, v (host, [3][n_total]): initial state.
 *   eps: host, n_clusters softening lengths (>= 0).
 *   workspace: device, at least nbody_workspace_bytes(), 256-byte aligned,
 *              owned by the caller and kept alive until nbody_destroy.
 *   hip_stream: a hipStream_t (NULL = the default stream).
 * Copies the host arrays (synchronously with respect to the host arrays:
 * they may be freed on return) and enqueues the start-up force pass. */
NBODY_API nbody_status nbody_init(nbody_ctx **ctx, int64_t n_total, int32_t n_clusters,
                        const int64_t *cluster_offsets, const double *m, const double *x,
                        const double *v, const double *eps, const nbody_params *p,
                        void *workspace, size_t workspace_bytes, void *hip_stream);

/* Replaces the parameters (e.g. switches precision).  dt_max/dt_min changes
 * take effect at the next step. */
NBODY_API nbody_status nbody_set_params(nbody_ctx *ctx, const nbody_params *p);

/* Hermite predictor (Sect. 2.1, predictor equations): predicts every
 * particle of cluster c to time t_pred[c] (host array, n_clusters entries),
 * giving x_p, v_p in FP64 and the record the mixed kernel reads.  NULL
 * predicts every cluster to its current time (x_p = x, v_p = v). */
NBODY_API nbody_status nbody_predict(nbody_ctx *ctx, const double *t_pred);

/* Pairwise acceleration, jerk and (optionally) potential (Sect. 2.1,
 * Eq. Force and the jerk by direct summation) on the listed particles from
 * every predicted particle j != i of the same cluster.  The predicted state
 * is that of the last nbody_predict; after block steps (nbody_step), every
 * particle is first predicted again to its cluster's current time.
 *   active_idx: device, n_active global particle ids, cluster-major, each
 *               id at most once (any order inside a cluster; lists in the
 *               storage order of nbody_get_layout run fastest in mixed
 *               precision).
 *   active_offsets: device, n_clusters+1 int64; the entries of cluster c are
 *               active_idx[active_offsets[c] .. active_offsets[c+1]).
 *   acc, jerk: device, [3][n_active] FP64 outputs; pot: device [n_active]
 *              or NULL.
 * Uses the context's precision.  Indices outside their cluster set
 * NBODY_E_INDEX on the device and produce zeros for that entry. */
NBODY_API nbody_status nbody_force(nbody_ctx *ctx, const int32_t *active_idx, const int64_t *active_offsets,
                         int64_t n_active, double *acc, double *jerk, double *pot);

/* nbody_force for callers that cannot allocate device memory or must not
 * touch the context's workspace beyond its state (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, kernels and results, bit for bit, but the slice partial sums of
 * the force pass go to a static device array of the library (64 MiB, one per
 * GPU, held until the process ends) instead of the workspace.  Allocates
 * nothing: no hipMalloc, hipFree or allocating library call.
 * Limit: the pass may plan at most 1198372 partial rows (7 FP64 each); a
 * call that could exceed it returns NBODY_E_INVAL and enqueues nothing.  It
 * is accepted whenever n_active * ceil(N_max / 256) <= 1198372 (N_max: the
 * largest cluster) or n_clusters * target_items * C + n_active <= 1198372,
 * C the largest i-chunk of the layouts the block can reach under min_block
 * (512 entries with two i per lane, 256 with one, 64, 16, 4 with 4, 16, 64
 * lanes per i): e.g. any block of a single cluster of up to 65536 particles
 * at the default tuning (target_items 4096 on 256 CUs, C = 256).
 * Every call on one GPU, from any context, shares that array, and the
 * array keeps the last call's contents: calls that overlap on one GPU (on
 * different streams) race and give wrong results.  NBODY_E_HIP if the
 * library could not look up the array's address on the context's device
 * at nbody_init. */
NBODY_API nbody_status nbody_force_noalloc(nbody_ctx *ctx, const int32_t *active_idx,
                                 const int64_t *active_offsets, int64_t n_active, double *acc,
                                 double *jerk, double *pot);

/* Perturber lists (Sect. 3.1): for each listed particle i, the particles
 * j != i of its cluster whose force on i exceeds the cluster's threshold,
 * m_j / (|x_j - x_i|^2 + eps^2) > threshold[c] on the predicted positions
 * (the state nbody_force would use), in ascending particle id -- the order
 * in which a serial sweep over the particles identifies them, which keeps
 * the lists identical to a serial code's -- at most max_pert of them.  R^2
 * is formed as ((dx dx + dy dy) + dz dz) + eps^2 in FP64, each operation
 * rounded, so the lists are reproducible bit for bit.
 *   active_idx, active_offsets, n_active: as for nbody_force.
 *   threshold: device, n_clusters doubles (e.g. a small fraction of the
 *              cluster's mean |a|).
 *   max_pert: 1 .. 256 (the paper's codes keep 256).
 *   lists: device, [n_active][max_pert] int32: the ids, then -1.
 *   counts: device, [n_active] int32: how many j pass (may exceed max_pert).
 * Asynchronous on the library's stream.  NBODY_E_INVAL for bad sizes or
 * NULL pointers; an id outside its cluster is reported as NBODY_E_INDEX
 * (device) and gets an empty list. */
NBODY_API nbody_status nbody_perturbers(nbody_ctx *ctx, const int32_t *active_idx,
                              const int64_t *active_offsets, int64_t n_active,
                              const double *threshold, int32_t max_pert, int32_t *lists,
                              int32_t *counts);

/* Hermite corrector, Aarseth step and block quantisation (Sect. 2.1) for the
 * listed particles, advancing each to its cluster's last predicted time
 * (the prediction time of nbody_predict, or of the last block step).
 * acc, jerk: device [3][n_active], the values at the predicted time (as
 * returned by nbody_force on the same list). */
NBODY_API nbody_status nbody_correct(nbody_ctx *ctx, const int32_t *active_idx,
                           const int64_t *active_offsets, int64_t n_active, const double *acc,
                           const double *jerk);

/* Up to n_block_steps block steps (Sect. 2.1 item list: select the particles
 * with the smallest t_i + dt_i, predict all, force on the block, correct,
 * new steps).  Each step advances every cluster whose time is below t_end by
 * exactly one of its own block steps; clusters at t_end stay put.  t_end
 * must be a multiple of dt_max.  Runs as captured HIP graphs (runs of 32
 * steps and single steps), replayed without host synchronisation.
 * Device errors freeze the state (see above): the step in which a new step
 * falls below dt_min completes, later ones change nothing.  Once the host
 * has read an error (nbody_sync), nbody_step returns it and enqueues
 * nothing. */
NBODY_API nbody_status nbody_step(nbody_ctx *ctx, int32_t n_block_steps, double t_end);

/* Waits for the context's stream; returns the first device-side error
 * (the status word is sticky: it is returned again until nbody_set_state). */
NBODY_API nbody_status nbody_sync(nbody_ctx *ctx);

/* Per-cluster softened energy E = sum m v^2/2 + (1/2) sum m phi in FP64,
 * written to E_host (n_clusters).  Synchronous.  Meaningful only when every
 * particle of a cluster is at the same time (multiples of dt_max). */
NBODY_API nbody_status nbody_energy(nbody_ctx *ctx, double *E_host);

/* Per-cluster diagnostics (Sect. 2.1, diagnostic output), FP64, written to
 * out_host[8 * c + k] for k = 0 kinetic energy sum m v^2/2, 1 potential
 * energy (1/2) sum m phi (softened, self pair excluded, phi from an FP64
 * force pass on every particle), 2..4 momentum sum m v, 5..7 angular
 * momentum sum m x cross v.  Evaluated on the state predicted to each
 * cluster's time (x, v themselves when every particle is at that time).
 * Synchronous; out_host holds 8 * n_clusters doubles. */
NBODY_API nbody_status nbody_diagnostics(nbody_ctx *ctx, double *out_host);

/* Per-cluster progress, synchronous: time of the last block step, number of
 * block steps taken and pairwise interactions evaluated (block size times
 * cluster size, summed).  Any pointer may be NULL. */
NBODY_API nbody_status nbody_progress(nbody_ctx *ctx, double *t_host, int64_t *steps_host,
                            double *interactions_host);

/* Checkpoint: bytes of the state blob, and copies of the full FP64 state
 * (m, x, v, a, k, t, dt, softening, cluster times and counters) to / from a
 * host buffer.  Synchronous.  Restoring and continuing gives the same bits
 * as an uninterrupted run.  nbody_set_state also clears the recorded device
 * errors (e.g. restore the last good checkpoint, lower dt_min, continue). */
NBODY_API nbody_status nbody_state_bytes(const nbody_ctx *ctx, size_t *bytes);
NBODY_API nbody_status nbody_get_state(nbody_ctx *ctx, void *host_buf, size_t bytes);
NBODY_API nbody_status nbody_set_state(nbody_ctx *ctx, const void *host_buf, size_t bytes);

/* Byte offsets, inside the workspace, of the FP64 state arrays, so the owner
 * of the workspace can read them in place (e.g. as tensors).  The arrays are
 * in the library's storage order, not in particle-id order: inside each
 * cluster the library stores particles along a Morton curve of their
 * initial positions (spatially close particles in consecutive slots, which
 * the mixed force pass relies on).  Slot q of every array holds particle
 * order[q]; entries of a cluster stay inside the cluster's id range.  An
 * active list given in storage order (active_idx[q] = order[slot]) gives the
 * fastest mixed force pass. */
typedef struct {
    int64_t n_total;
    int32_t n_clusters;
    int32_t reserved;
    size_t m, x, v, a, k, t, dt; /* [n], [3][n], [3][n], [3][n], [3][n], [n], [n] */
    size_t xp, vp;               /* predicted state, [3][n] each                 */
    size_t pot;                  /* potential of the last block (compute_pot)    */
    size_t order;                /* int32 [n]: particle id stored at each slot   */
} nbody_layout;
NBODY_API nbody_status nbody_get_layout(const nbody_ctx *ctx, nbody_layout *out);

/* Launch tuning of the force pass.  Results for a cluster depend only on
 * its own size, its block size and these values (never on other clusters
 * in the batch); changing them changes force sums at rounding level only.
 *   target_items: work items (i-chunk x j-slice) a cluster's force pass is
 *                 split into when it has enough tiles (default: 16 per
 *                 CU; 1 .. 16384).
 *   min_block: smallest block size that uses, in order, the layouts with
 *              two i per lane, one i per lane, 4 lanes per i and 16 lanes
 *              per i (default 2^30, 1024, 48, 12: the two-i-per-lane
 *              layout is off by default, and the tile-relative format never
 *              uses it: min_block[0] and small_min_block[0] are ignored
 *              there); smaller blocks use 64
 *              lanes per i.  Must be non-increasing and >= 1.
 *   small_cluster_n, small_min_block: clusters of fewer than
 *              small_cluster_n particles use small_min_block instead of
 *              min_block (default 16384 and 2^30, 2^30, 24, 6: small
 *              clusters have few j-tiles, and chunks of 512 or 256 active
 *              particles leave too few work items); small_cluster_n = 0
 *              applies min_block to every cluster.  When no cluster is as
 *              large as its threshold for one lane per i (the second
 *              entry), the force pass runs a kernel build with only the
 *              j-split layouts, at higher occupancy; results per layout
 *              are the same bits either way.
 *   grid: persistent workgroups of the force launch (default: 16 per CU).
 *   mixed_format: how the mixed kernel forms the FP32 pair difference
 *                 x_j - x_i: 0 from double-single FP32 pairs
 *                 (hi_j - hi_i) + (lo_j - lo_i); 1 in FP64 from the FP64
 *                 positions, rounded once; 2 (default) tile-relative: every
 *                 position is rounded to FP32 relative to the centre of its
 *                 LDS tile (kTile consecutive slots, compact in space), so
 *                 the difference is one FP32 subtraction; pairs much closer
 *                 than their tile's size are caught by the near test below.
 *   rsq_bias_correct: 1 (default) removes the mean relative error of the
 *                 hardware FP32 reciprocal square root, measured on the
 *                 device at nbody_init, from the mixed kernel's sums (each
 *                 FP32 window is scaled in FP64 by 1 - 3b, potential 1 - b);
 *                 0 leaves the hardware estimate as is.
 *   near_tau, near_tau_k: in the mixed kernel no pair whose acceleration
 *                 term m_j / R^2 may exceed near_tau * |a_i|, or whose
 *                 jerk term (at most 2 m_j |v_j - v_i| / R^3) may exceed
 *                 near_tau_k * |k_i| (|a_i|, |k_i| from the last step), is
 *                 summed in FP32: a window of 32 j that may hold one is
 *                 evaluated in FP64 instead (defaults 0.25 and 1;
 *                 near_tau = 0 turns the whole test off, near_tau_k = 0 only
 *                 its jerk part).  One FP32 term carries a few units of FP32
 *                 rounding, which limits the relative error of a sum only
 *                 when that term is comparable to the whole sum (close
 *                 neighbours).
 *   mid_tau: tile-relative format only.  Its FP32 coordinates carry an
 *                 error of about 2^-24 times the tile's size, so a pair much
 *                 closer than its tile is large loses precision in its
 *                 difference although its term passes the test above: a
 *                 window whose closest pair has term * (L / R) above
 *                 mid_tau * |a_i| (or the jerk analogue above mid_tau * |k_i|)
 *                 is summed again with FP64 position differences (L: the
 *                 i's distance from the tile centre plus the tile's size;
 *                 default 4).
 *   window, waves, tile: build of the tile-relative kernel with the near
 *                 test on the lean path (every cluster softened) and no
 *                 potential: FP32 window of 16, 32 or 64 pairs, an
 *                 occupancy of 2 to 5 waves per SIMD and j-tiles of 128 or
 *                 256 records in LDS (128 only with windows of 16 or 32;
 *                 NBODY_E_INVAL otherwise; default 32, 4 and 256, the build that
 *                 needs no scratch memory; results change at rounding level
 *                 with the window and the tile).  Other passes use their
 *                 own fixed build.
 *   pred_in_force: 0 (default) or 1.  With 1, a block step whose block
 *                 fills a single i-chunk of a layout that splits j over
 *                 lanes (small blocks) predicts only the block's members in
 *                 the selection, and the force pass predicts each j-record
 *                 from x, v, a, k and t as it loads it (Sect. 2.1: the
 *                 prediction may run on the accelerator).  Same arithmetic,
 *                 so the results are bitwise those of 0.  Applies to
 *                 nbody_step in the FP64 format, and in the tile-relative
 *                 format where its default build runs (near test on, every
 *                 cluster softened, default window, waves and tile or the
 *                 potential on) or only the j-split layouts can occur;
 *                 elsewhere it has no effect.  Direct nbody_force calls
 *                 always read the stored prediction.  Other values:
 *                 NBODY_E_INVAL.
 * In the tile-relative format the mixed arithmetic runs in the
 * one-lane-per-i layout (blocks from min_block[1] on); the layouts that
 * split j over lanes (small blocks, latency-bound) run the FP64 arithmetic,
 * which is as fast there and exact. */
typedef struct {
    int32_t target_items;
    int32_t min_block[4];
    int32_t grid;
    int32_t mixed_format;
    int32_t rsq_bias_correct;
    double near_tau;
    int32_t small_cluster_n;
    int32_t small_min_block[4];
    double near_tau_k;
    double mid_tau;
    int32_t window;
    int32_t waves;
    int32_t tile;
    int32_t pred_in_force;
} nbody_tuning;
NBODY_API nbody_status nbody_get_tuning(const nbody_ctx *ctx, nbody_tuning *out);
NBODY_API nbody_status nbody_set_tuning(nbody_ctx *ctx, const nbody_tuning *t);

/* Kernel timing of the force pass: while enabled, nbody_force brackets its
 * force-kernel launch with HIP events on the context's stream.
 * nbody_profile_read waits for the stream and returns the summed kernel
 * time in milliseconds and the number of timed launches since the last
 * read (or since enabling), then resets both. */
NBODY_API nbody_status nbody_profile_force(nbody_ctx *ctx, int32_t enable);
NBODY_API nbody_status nbody_profile_read(nbody_ctx *ctx, double *ms, int64_t *launches);

/* Frees the host context (never the workspace).  NULL is accepted. */
NBODY_API nbody_status nbody_destroy(nbody_ctx *ctx);

/* Static description of a status code. */
NBODY_API const char *nbody_strerror(nbody_status s);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
