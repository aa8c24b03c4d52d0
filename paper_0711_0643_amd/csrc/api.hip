// Host side of libnbody: the C ABI declared in include/nbody.h.
//
// The library owns no device memory: nbody_init carves the caller's
// workspace into the arrays of DevState, and every call enqueues kernels on
// the context's stream.  nbody_step captures block steps (select -> plan
// -> force -> correct; no plan kernel with a single cluster) into HIP
// graphs once and replays them.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "nbody.h"

using namespace nb;

// Device scratch of nbody_force_noalloc: the slice partial sums of its force
// pass (7 rows of FP64 per partial row), for callers that cannot allocate
// device memory.  Every GPU the library runs on holds one copy until the
// process ends.  Host code never uses the array's name as an address: it
// uses the per-device address that scratch_address() looks up.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int64_t kScratchRows = (int64_t)(kScratchBytes / (7 * sizeof(double)));
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
bool g_scratch_looked_up[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (device `dev`, which
// must be current), looked up once per device; nullptr if the lookup failed.
double* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_looked_up[dev]) {
    g_scratch_looked_up[dev] = true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess)
      g_scratch[dev] = (double*)ptr;
    else
      (void)hipGetLastError();  // do not leave the error for the next launch check
  }
  return g_scratch[dev];
}

constexpr uint32_t kStateMagic = 0x5453424eu;  // "NBST"
constexpr uint32_t kStateVersion = 2;

struct Layout {
  size_t coff, eps, cid, ch_cluster, ch_begin, cl_ch, order, slot_of, tmeta, ulist;
  size_t m, x, v, a, k, t, dt, xp, vp, pot, jr;
  size_t tpred, tnow, inter, steps, cm2, cm2n, acount, umin, ucnt, act, aoff, plan, offs, ctl, part, fout, pid, status,
      eout, tpstamp;
  size_t total;
  int64_t rows_cap;
  int64_t nch_max;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout make_layout(int64_t n, int32_t nc) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t N = (size_t)n, C = (size_t)nc;
  L.nch_max = n / kSelChunk + nc;
  L.rows_cap = kRowsPerParticle * n + kRowsPerCluster * (int64_t)nc;
  L.coff = take(8 * (C + 1));
  L.eps = take(8 * C);
  L.cid = take(4 * N);
  L.ch_cluster = take(4 * (size_t)L.nch_max);
  L.ch_begin = take(8 * ((size_t)L.nch_max + 1));
  L.cl_ch = take(4 * (C + 1));
  L.order = take(4 * N);
  L.slot_of = take(4 * N);
  L.tmeta = take(8 * kTileMeta * (size_t)L.nch_max);
  L.ulist = take(4 * N);
  L.m = take(8 * N);
  L.x = take(24 * N);
  L.v = take(24 * N);
  L.a = take(24 * N);
  L.k = take(24 * N);
  L.t = take(8 * N);
  L.dt = take(8 * N);
  L.xp = take(24 * N);
  L.vp = take(24 * N);
  L.pot = take(8 * N);
  L.jr = take(4 * JR_ROWS * N);
  L.tpred = take(8 * C);
  L.tnow = take(8 * C);
  L.inter = take(8 * C);
  L.steps = take(8 * C);
  L.cm2 = take(16 * (size_t)L.nch_max);
  L.cm2n = take(8 * (size_t)L.nch_max);
  L.acount = take(8 * C);  // two halves of int32 counters, by step parity
  L.umin = take(8 * N);
  L.ucnt = take(4 * N);
  L.act = take(4 * N);
  L.aoff = take(8 * (C + 1));
  L.plan = take(sizeof(Plan) * C);
  L.offs = take(16 * C);
  L.ctl = take(sizeof(Ctl));
  L.part = take(8 * 7 * (size_t)L.rows_cap);
  L.fout = take(8 * 7 * N);
  L.pid = take(8 * 4 * N);
  L.status = take(4);
  L.eout = take(64 * C);
  L.tpstamp = take(8 * (size_t)L.nch_max);
  L.total = o;
  return L;
}

// Spread the low 21 bits of v to every third bit (Morton interleave).
uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Storage order of the particles: inside each cluster, ascending Morton
// code of the initial position in the cluster's bounding box (21 bits per
// axis), ties by particle id, so that consecutive slots (and the kTile slots
// of a force tile) are close in space.  order[slot] = particle id.
std::vector<int32_t> morton_order(int64_t n, int32_t nc, const int64_t* coff, const double* x) {
  std::vector<int32_t> order((size_t)n);
  std::vector<std::pair<uint64_t, int32_t>> key;
  for (int c = 0; c < nc; ++c) {
    const int64_t b = coff[c], e = coff[c + 1];
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = INFINITY;
      hi[d] = -INFINITY;
      for (int64_t i = b; i < e; ++i) {
        lo[d] = fmin(lo[d], x[d * n + i]);
        hi[d] = fmax(hi[d], x[d * n + i]);
      }
    }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) ext = fmax(ext, hi[d] - lo[d]);
    const double scale = ext > 0.0 ? 2097151.0 / ext : 0.0;
    key.resize((size_t)(e - b));
    for (int64_t i = b; i < e; ++i) {
      uint64_t code = 0;
      for (int d = 0; d < 3; ++d) {
        double q = (x[d * n + i] - lo[d]) * scale;
        q = q < 0.0 ? 0.0 : q > 2097151.0 ? 2097151.0 : q;
        code |= spread3((uint64_t)q) << d;
      }
      key[(size_t)(i - b)] = {code, (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    for (int64_t i = b; i < e; ++i) order[(size_t)i] = key[(size_t)(i - b)].second;
  }
  return order;
}

bool valid_params(const nbody_params* p) {
  if (!p) return false;
  if (!(p->eta > 0.0) || !isfinite(p->eta)) return false;
  if (!(p->eta_init > 0.0) || !isfinite(p->eta_init)) return false;
  if (!(p->dt_max > 0.0) || !isfinite(p->dt_max)) return false;
  if (!(p->dt_min > 0.0) || !(p->dt_min <= p->dt_max)) return false;
  int e;
  if (frexp(p->dt_max, &e) != 0.5) return false;  // dt_max must be a power of two
  if (p->precision != NBODY_FP64 && p->precision != NBODY_MIXED) return false;
  return true;
}

}  // namespace

struct nbody_ctx {
  DevState s{};
  Layout L{};
  nbody_params p{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
  unsigned char* ws = nullptr;
  int64_t n = 0;
  int32_t nc = 0;
  int32_t nch = 0;
  int grid = 4096;        // persistent force grid
  int target_items = 4096;  // work items a force pass aims at per cluster
  int mixed_mode = kTR;   // position format of the mixed kernel
  int kwindow = 32;       // FP32 window of the lean tile-relative kernel (16, 32, 64)
  int kwaves = 4;         // its occupancy, waves per SIMD (2 to 5)
  int ktile = kTile;      // its j-records per LDS tile (128 or 256)
  int rsq_correct = 1;    // remove the mean bias of v_rsq_f32 in the mixed kernel
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};  // one block step, of parity 0 and 1
  hipGraph_t graph_k = nullptr;
  hipGraphExec_t gexec_k = nullptr;  // kStepsPerGraph block steps in sequence, from parity 0
  int parity = 0;  // parity of the next block step (which halves of the selection buffers it uses)
  int graph_mode = -1;    // force mode the graph was captured with
  int graph_pot = -1;
  bool predicted = false;
  // the predicted state holds every field (x_p, v_p, all j-record rows) for
  // every particle: true after a full prediction, false after block steps,
  // whose predictor writes only what the step's force and corrector read
  bool pred_full = false;
  // the step pipeline's selection state (chunk minima, unit minima, plan)
  // matches t, dt; cleared by every call that changes them outside the graph
  bool sel_valid = false;
  // device status bits the host has read (nbody_sync); nbody_step returns
  // them without enqueuing work until nbody_set_state restores a state
  int32_t seen_bits = 0;
  std::vector<int64_t> coff;
  std::vector<int32_t> order;  // particle id stored at each slot
  // every cluster keeps the self pair of the mixed kernel finite in FP32
  // (eps^2 representable, largest m / eps^3 far from overflow): the lean
  // tile-relative build may run
  bool lean_ok = false;
  int pif = 0;  // fused predictor requested (nbody_tuning.pred_in_force)
  // this device's copy of the static scratch (nbody_force_noalloc), looked
  // up at init with the context's device current; nullptr if unavailable
  double* scratch = nullptr;
  Ctl ctl{};
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;  // recorded, not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_free;     // reusable event pairs
};

namespace {

#define HIP_OK(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return NBODY_E_HIP; \
  } while (0)

// Longest perturber list (Sect. 3.1: the paper's codes keep 256).
constexpr int32_t kMaxPerturbers = 256;

int force_mode(const nbody_ctx* c) { return c->p.precision == NBODY_FP64 ? kF64 : c->mixed_mode; }

bool split_only(const nbody_ctx* c, int64_t n_active);

// Whether the step pipeline runs the fused predictor: requested, and a
// force build with it exists for the current settings (the device flag the
// selection reads is set from this, so selection and force pass agree).
bool pif_active(const nbody_ctx* c) {
  return c->pif != 0 && has_pif_build(force_mode(c), c->p.compute_pot != 0, c->ctl.near_tau > 0.0,
                                      split_only(c, c->n), c->lean_ok, c->kwindow, c->kwaves, c->ktile);
}

nbody_status upload_ctl(nbody_ctx* c) {
  c->ctl.eta = c->p.eta;
  c->ctl.eta_init = c->p.eta_init;
  c->ctl.dt_max = c->p.dt_max;
  c->ctl.dt_min = c->p.dt_min;
  c->ctl.compute_pot = c->p.compute_pot ? 1 : 0;
  // the tile-relative format has no two-i-per-lane build: plan without it
  Ctl up = c->ctl;
  if (force_mode(c) == kTR) up.vmin[0] = up.vmin_small[0] = INT32_MAX;  // above any block (<= 2^30)
  up.pred_in_force = pif_active(c) ? 1 : 0;
  // host-owned fields only: the rsq_* fields at the end are written on the device
  HIP_OK(hipMemcpyAsync(c->ws + c->L.ctl, &up, offsetof(Ctl, rsq_scale3), hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));  // `up` is host memory the copy reads
  return NBODY_OK;
}

nbody_status status_from_bits(int32_t bits) {
  if (bits & ST_INDEX) return NBODY_E_INDEX;
  if (bits & ST_NONFINITE) return NBODY_E_NONFINITE;
  if (bits & ST_DTMIN) return NBODY_E_DTMIN;
  if (bits & ST_STATE) return NBODY_E_STATE;
  return NBODY_OK;
}

// Whether no cluster can reach a one-lane-per-i layout: a block holds at
// most all of its cluster and at most the n_active entries of the active
// list, so a cluster whose bound is below the threshold of layout 1 (the
// lower of the two; thresholds do not increase with the layout index) never
// uses layouts 0 or 1.  Then the force pass runs the kernel with only the
// j-split layouts, which has the higher occupancy.
bool split_only(const nbody_ctx* c, int64_t n_active) {
  for (int k = 0; k < c->nc; ++k) {
    const int64_t nk = c->coff[k + 1] - c->coff[k];
    const int64_t thr = nk < c->ctl.small_n ? c->ctl.vmin_small[1] : c->ctl.vmin[1];
    if (std::min(nk, n_active) >= thr) return false;
  }
  return true;
}

// Force on the internal identity active list into s.fout (start-up, energy).
nbody_status force_all_internal(nbody_ctx* c, int mode) {
  const DevState& s = c->s;
  HIP_OK(launch_identity(s, c->stream));
  HIP_OK(launch_plan(s, s.aoff, s.n, c->target_items, c->stream));
  HIP_OK(launch_force(s, mode, true, c->ctl.near_tau > 0.0, split_only(c, s.n), c->lean_ok, s.act, c->grid, -1,
                      c->target_items, c->stream));
  HIP_OK(launch_reduce(s, s.aoff, s.n, s.fout, s.fout + 3 * s.n, s.fout + 6 * s.n, c->stream));
  return NBODY_OK;
}

void destroy_graph(nbody_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    if (c->gexec[p]) (void)hipGraphExecDestroy(c->gexec[p]);
    if (c->graph[p]) (void)hipGraphDestroy(c->graph[p]);
    c->gexec[p] = nullptr;
    c->graph[p] = nullptr;
  }
  if (c->gexec_k) (void)hipGraphExecDestroy(c->gexec_k);
  if (c->graph_k) (void)hipGraphDestroy(c->graph_k);
  c->gexec_k = nullptr;
  c->graph_k = nullptr;
  c->graph_mode = -1;
}

// Block steps captured into graphs: one block step = selection (with the
// predictor) -> plan (several clusters only) -> force -> slice reduction
// with the corrector.  Each step carries its parity (which halves of the
// selection buffers it uses) as a launch argument, alternating 0, 1, 0, ...
// Three graphs: one step of parity 0, one of parity 1, and kStepsPerGraph
// steps from parity 0 (fewer graph launches and no gaps between them for
// long runs).  Captured once, replayed; the host tracks the parity.
constexpr int kStepsPerGraph = 32;

hipError_t capture_steps(nbody_ctx* c, int steps, int par0, hipGraph_t* g) {
  const DevState& s = c->s;
  const int mode = force_mode(c);
  // block sizes are counted where they decide the tile frames (the
  // tile-relative format with some cluster that can reach its
  // one-lane-per-i layout) or the fused predictor
  const bool pif = pif_active(c);
  const bool counting = (mode == kTR && !split_only(c, s.n)) || pif;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  for (int k = 0; k < steps && e == hipSuccess; ++k) {
    const int par = (par0 + k) & 1;
    e = launch_select(s, c->target_items, mode, par, counting, c->cap_stream);
    if (e == hipSuccess)
      e = launch_force(s, mode, c->p.compute_pot != 0, c->ctl.near_tau > 0.0, split_only(c, s.n), c->lean_ok, s.act,
                       c->grid, par, c->target_items, c->cap_stream, c->kwindow, c->kwaves, c->ktile, pif);
    if (e == hipSuccess)
      e = launch_reduce_correct_step(s, c->p.compute_pot != 0, par, c->target_items, counting, c->cap_stream);
  }
  *g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, g);
  if (e == hipSuccess && (e2 != hipSuccess || !*g)) e = e2 != hipSuccess ? e2 : hipErrorUnknown;
  if (e != hipSuccess && *g) {
    (void)hipGraphDestroy(*g);
    *g = nullptr;
  }
  return e;
}

nbody_status build_graph(nbody_ctx* c) {
  destroy_graph(c);
  if (!c->cap_stream) HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  static_assert(kStepsPerGraph % 2 == 0, "a run of steps must return to parity 0");
  if (capture_steps(c, 1, 0, &c->graph[0]) != hipSuccess || capture_steps(c, 1, 1, &c->graph[1]) != hipSuccess ||
      capture_steps(c, kStepsPerGraph, 0, &c->graph_k) != hipSuccess ||
      hipGraphInstantiate(&c->gexec[0], c->graph[0], nullptr, nullptr, 0) != hipSuccess ||
      hipGraphInstantiate(&c->gexec[1], c->graph[1], nullptr, nullptr, 0) != hipSuccess ||
      hipGraphInstantiate(&c->gexec_k, c->graph_k, nullptr, nullptr, 0) != hipSuccess) {
    destroy_graph(c);
    return NBODY_E_HIP;
  }
  c->graph_mode = force_mode(c);
  c->graph_pot = c->p.compute_pot;
  return NBODY_OK;
}

}  // namespace

namespace {
struct Part {
  size_t off;    // device offset in the workspace
  size_t bytes;
};
std::vector<Part> state_parts(const nbody_ctx* c) {
  const size_t N = (size_t)c->n, C = (size_t)c->nc;
  const Layout& L = c->L;
  return {{L.coff, 8 * (C + 1)}, {L.eps, 8 * C}, {L.order, 4 * N}, {L.slot_of, 4 * N}, {L.m, 8 * N},
          {L.x, 24 * N},         {L.v, 24 * N},  {L.a, 24 * N},     {L.k, 24 * N},       {L.t, 8 * N},
          {L.dt, 8 * N},         {L.tnow, 8 * C}, {L.inter, 8 * C}, {L.steps, 8 * C}};
}
}  // namespace

extern "C" {

void nbody_default_params(nbody_params* p) {
  if (!p) return;
  p->eta = 0.01;
  p->eta_init = 0.01;
  p->dt_max = 0.125;
  p->dt_min = ldexp(1.0, -40);
  p->precision = NBODY_FP64;
  p->compute_pot = 0;
}

nbody_status nbody_workspace_bytes(int64_t n_total, int32_t n_clusters, const nbody_params* p, size_t* bytes) {
  (void)p;
  if (!bytes || n_total < 1 || n_total > kMaxParticles || n_clusters < 1 || n_clusters > n_total)
    return NBODY_E_INVAL;
  *bytes = make_layout(n_total, n_clusters).total;
  return NBODY_OK;
}

nbody_status nbody_init(nbody_ctx** out, int64_t n_total, int32_t n_clusters, const int64_t* cluster_offsets,
                        const double* m, const double* x, const double* v, const double* eps,
                        const nbody_params* p, void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!out) return NBODY_E_INVAL;
  *out = nullptr;
  if (!cluster_offsets || !m || !x || !v || !eps || !workspace || !valid_params(p)) return NBODY_E_INVAL;
  if (n_total < 1 || n_total > kMaxParticles || n_clusters < 1 || n_clusters > n_total)
    return NBODY_E_INVAL;
  if (((uintptr_t)workspace & 255) != 0) return NBODY_E_INVAL;
  if (cluster_offsets[0] != 0 || cluster_offsets[n_clusters] != n_total) return NBODY_E_INVAL;
  for (int c = 0; c < n_clusters; ++c) {
    if (cluster_offsets[c + 1] <= cluster_offsets[c]) return NBODY_E_INVAL;
    if (!(eps[c] >= 0.0) || !isfinite(eps[c])) return NBODY_E_INVAL;
  }
  for (int64_t i = 0; i < n_total; ++i) {
    if (!isfinite(m[i]) || m[i] < 0.0) return NBODY_E_INVAL;
    for (int d = 0; d < 3; ++d)
      if (!isfinite(x[d * n_total + i]) || !isfinite(v[d * n_total + i])) return NBODY_E_INVAL;
  }
  const Layout L = make_layout(n_total, n_clusters);
  if (workspace_bytes < L.total) return NBODY_E_NOMEM;

  nbody_ctx* c = new (std::nothrow) nbody_ctx();
  if (!c) return NBODY_E_NOMEM;
  c->L = L;
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)workspace;
  {
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess) c->scratch = scratch_address(dev);
    else (void)hipGetLastError();
  }
  c->n = n_total;
  c->nc = n_clusters;
  c->coff.assign(cluster_offsets, cluster_offsets + n_clusters + 1);

  c->lean_ok = true;
  for (int cc = 0; cc < n_clusters; ++cc) {
    double mmax = 0.0;
    for (int64_t i = cluster_offsets[cc]; i < cluster_offsets[cc + 1]; ++i) mmax = fmax(mmax, m[i]);
    const float e2 = (float)(eps[cc] * eps[cc]);
    if (!(e2 >= 1e-30f) || !(mmax / (eps[cc] * eps[cc] * eps[cc]) < 1e30)) c->lean_ok = false;
  }
  // storage order: Morton order inside each cluster; the inputs are copied
  // to the device in that order
  c->order = morton_order(n_total, n_clusters, cluster_offsets, x);
  std::vector<int32_t> slot_of((size_t)n_total);
  std::vector<double> ms((size_t)n_total), xs(3 * (size_t)n_total), vs(3 * (size_t)n_total);
  for (int64_t q = 0; q < n_total; ++q) {
    const int64_t id = c->order[(size_t)q];
    slot_of[(size_t)id] = (int32_t)q;
    ms[(size_t)q] = m[id];
    for (int d = 0; d < 3; ++d) {
      xs[(size_t)(d * n_total + q)] = x[d * n_total + id];
      vs[(size_t)(d * n_total + q)] = v[d * n_total + id];
    }
  }

  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  c->grid = cus * 16;
  c->target_items = cus * 16;

  // host-side tables: cluster of each particle, selection chunks
  std::vector<int32_t> cid((size_t)n_total), cl_ch((size_t)n_clusters + 1);
  std::vector<int32_t> ch_cluster;
  std::vector<int64_t> ch_begin;
  for (int cc = 0; cc < n_clusters; ++cc) {
    cl_ch[cc] = (int32_t)ch_begin.size();
    for (int64_t i = cluster_offsets[cc]; i < cluster_offsets[cc + 1]; ++i) cid[(size_t)i] = cc;
    for (int64_t b = cluster_offsets[cc]; b < cluster_offsets[cc + 1]; b += kSelChunk) {
      ch_cluster.push_back(cc);
      ch_begin.push_back(b);
    }
  }
  cl_ch[n_clusters] = (int32_t)ch_begin.size();
  c->nch = (int32_t)ch_begin.size();
  ch_begin.push_back(n_total);

  DevState& s = c->s;
  unsigned char* w = c->ws;
  s.n = n_total;
  s.nc = n_clusters;
  s.nch = c->nch;
  s.coff = (const int64_t*)(w + L.coff);
  s.eps = (const double*)(w + L.eps);
  s.cid = (const int32_t*)(w + L.cid);
  s.ch_cluster = (const int32_t*)(w + L.ch_cluster);
  s.ch_begin = (const int64_t*)(w + L.ch_begin);
  s.cl_ch = (const int32_t*)(w + L.cl_ch);
  s.order = (int32_t*)(w + L.order);
  s.slot_of = (int32_t*)(w + L.slot_of);
  s.tmeta = (double*)(w + L.tmeta);
  s.ulist = (int32_t*)(w + L.ulist);
  s.m = (double*)(w + L.m);
  s.x = (double*)(w + L.x);
  s.v = (double*)(w + L.v);
  s.a = (double*)(w + L.a);
  s.k = (double*)(w + L.k);
  s.t = (double*)(w + L.t);
  s.dt = (double*)(w + L.dt);
  s.xp = (double*)(w + L.xp);
  s.vp = (double*)(w + L.vp);
  s.pot = (double*)(w + L.pot);
  s.jr = (float*)(w + L.jr);
  s.tpred = (double*)(w + L.tpred);
  s.tnow = (double*)(w + L.tnow);
  s.inter = (double*)(w + L.inter);
  s.steps = (int64_t*)(w + L.steps);
  s.cm2 = (double*)(w + L.cm2);
  s.cm2n = (int32_t*)(w + L.cm2n);
  s.acount = (int32_t*)(w + L.acount);
  s.umin = (double*)(w + L.umin);
  s.ucnt = (int32_t*)(w + L.ucnt);
  s.act = (int32_t*)(w + L.act);
  s.aoff = (int64_t*)(w + L.aoff);
  s.plan = (Plan*)(w + L.plan);
  s.offs = (int64_t*)(w + L.offs);
  s.ctl = (Ctl*)(w + L.ctl);
  s.part = (double*)(w + L.part);
  s.rows_cap = L.rows_cap;
  s.fout = (double*)(w + L.fout);
  s.pid = (double*)(w + L.pid);
  s.status = (int32_t*)(w + L.status);
  s.tpstamp = (double*)(w + L.tpstamp);

  c->ctl.vmin[0] = 1 << 30;  // two i per lane: off (one i per lane is faster on gfx950)
  c->ctl.vmin[1] = 1024;
  c->ctl.vmin[2] = 48;
  c->ctl.vmin[3] = 12;
  c->ctl.small_n = 16384;
  c->ctl.vmin_small[0] = 1 << 30;
  c->ctl.vmin_small[1] = 1 << 30;
  c->ctl.vmin_small[2] = 24;
  c->ctl.vmin_small[3] = 6;
  c->ctl.near_tau = 0.25;
  c->ctl.near_tau_k = 1.0;
  c->ctl.mid_tau = 4.0;

  const size_t N = (size_t)n_total;
  hipStream_t st = c->stream;
  bool ok = true;
  ok = ok && hipMemsetAsync(w, 0, L.total, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.coff, cluster_offsets, 8 * ((size_t)n_clusters + 1), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.eps, eps, 8 * (size_t)n_clusters, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.cid, cid.data(), 4 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.ch_cluster, ch_cluster.data(), 4 * ch_cluster.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.ch_begin, ch_begin.data(), 8 * ch_begin.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.cl_ch, cl_ch.data(), 4 * cl_ch.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.order, c->order.data(), 4 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.slot_of, slot_of.data(), 4 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.m, ms.data(), 8 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.x, xs.data(), 24 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(w + L.v, vs.data(), 24 * N, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    delete c;
    return NBODY_E_HIP;
  }
  nbody_status r = upload_ctl(c);
  if (r == NBODY_OK && launch_rsq_bias(s, c->rsq_correct, st) != hipSuccess) r = NBODY_E_HIP;
  // start-up (Sect. 2.1): a, k of every particle at t = 0, then initial steps
  if (r == NBODY_OK && launch_predict_all(s, st) != hipSuccess) r = NBODY_E_HIP;  // tpred = 0: x_p = x
  c->pred_full = true;
  // the start-up pass is FP64 in every precision: one N^2 pass, and its |a|
  // is what the mixed kernel's near-pair test reads at the first step
  if (r == NBODY_OK) r = force_all_internal(c, kF64);
  if (r == NBODY_OK && launch_init_steps(s, st) != hipSuccess) r = NBODY_E_HIP;
  if (r != NBODY_OK) {
    delete c;
    return r;
  }
  c->predicted = true;
  *out = c;
  return NBODY_OK;
}

nbody_status nbody_set_params(nbody_ctx* c, const nbody_params* p) {
  if (!c || !valid_params(p)) return NBODY_E_INVAL;
  c->p = *p;
  return upload_ctl(c);
}

nbody_status nbody_predict(nbody_ctx* c, const double* t_pred) {
  if (!c) return NBODY_E_INVAL;
  if (t_pred) {
    for (int i = 0; i < c->nc; ++i)
      if (!isfinite(t_pred[i])) return NBODY_E_INVAL;
    HIP_OK(hipMemcpyAsync(c->s.tpred, t_pred, 8 * (size_t)c->nc, hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
  } else {
    HIP_OK(hipMemcpyAsync(c->s.tpred, c->s.tnow, 8 * (size_t)c->nc, hipMemcpyDeviceToDevice, c->stream));
  }
  HIP_OK(launch_predict_all(c->s, c->stream));
  c->predicted = true;
  c->pred_full = true;
  return NBODY_OK;
}

namespace {

// After block steps the predicted state is partial and the corrected
// particles' entries are from before their correction: predict every
// particle again to each cluster's time before a direct force or corrector
// call reads it.
nbody_status complete_prediction(nbody_ctx* c) {
  if (!c->pred_full) {
    HIP_OK(launch_predict_all(c->s, c->stream));
    c->pred_full = true;
  }
  return NBODY_OK;
}

// The force pass of nbody_force on the state view `s` (the context's, or
// one whose partial rows live in the static scratch).
nbody_status force_pass(nbody_ctx* c, const DevState& s, const int32_t* active_idx, const int64_t* active_offsets,
                        int64_t n_active, double* acc, double* jerk, double* pot, bool profile) {
  const nbody_status r = complete_prediction(c);
  if (r != NBODY_OK) return r;
  c->sel_valid = false;  // the plan is replaced
  HIP_OK(launch_map_active(s, active_idx, n_active, c->stream));  // particle ids -> slots
  HIP_OK(launch_plan(s, active_offsets, n_active, c->target_items, c->stream));
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (profile) {
    if (!c->prof_free.empty()) {
      ev = c->prof_free.back();
      c->prof_free.pop_back();
    } else {
      HIP_OK(hipEventCreate(&ev.first));
      HIP_OK(hipEventCreate(&ev.second));
    }
    HIP_OK(hipEventRecord(ev.first, c->stream));
  }
  HIP_OK(launch_force(s, force_mode(c), pot != nullptr, c->ctl.near_tau > 0.0, split_only(c, n_active), c->lean_ok,
                      s.ulist,
                      c->grid, -1, c->target_items, c->stream, c->kwindow, c->kwaves, c->ktile));
  if (profile) {
    HIP_OK(hipEventRecord(ev.second, c->stream));
    c->prof_pending.push_back(ev);
  }
  HIP_OK(launch_reduce(s, active_offsets, n_active, acc, jerk, pot, c->stream));
  return NBODY_OK;
}

}  // namespace

nbody_status nbody_force(nbody_ctx* c, const int32_t* active_idx, const int64_t* active_offsets, int64_t n_active,
                         double* acc, double* jerk, double* pot) {
  if (!c || n_active < 0 || n_active > c->n) return NBODY_E_INVAL;
  if (n_active == 0) return NBODY_OK;
  if (!active_idx || !active_offsets || !acc || !jerk) return NBODY_E_INVAL;
  if (!c->predicted) return NBODY_E_STATE;
  return force_pass(c, c->s, active_idx, active_offsets, n_active, acc, jerk, pot, c->profile);
}

namespace {

// Most partial rows a force pass over n_active entries can plan.  A cluster
// with na > 0 entries gets S * na rows, where S <= ceil(target / chunks)
// (chunks = ceil(na / iwg) i-chunks of iwg entries, iwg that of the layout
// the plan picks) and S <= its number of LDS tiles; so S * na < target *
// iwg + na, and S * na <= na * (tiles of the largest cluster).  iwg is
// bounded by the largest i-chunk of the layouts a block of at most n_active
// entries can reach under the current thresholds.  Never more than the
// context's own partial-row capacity.
int64_t planned_rows_bound(const nbody_ctx* c, int64_t n_active) {
  int64_t tiles = 1, iwg = variant_iwg(kNumVariants - 1);
  for (int k = 0; k < c->nc; ++k) {
    const int64_t nn = c->coff[k + 1] - c->coff[k];
    tiles = std::max(tiles, (nn + kTile - 1) / kTile);
    for (int v = 0; v < kNumVariants - 1; ++v) {
      const int64_t thr = nn < c->ctl.small_n ? c->ctl.vmin_small[v] : c->ctl.vmin[v];
      if (thr <= std::min(n_active, nn)) iwg = std::max(iwg, (int64_t)variant_iwg(v));
    }
  }
  const int64_t by_target = (int64_t)c->nc * c->target_items * iwg + n_active;
  const int64_t by_tiles = n_active * tiles;
  return std::min(c->s.rows_cap, std::min(by_target, by_tiles));
}

}  // namespace

nbody_status nbody_force_noalloc(nbody_ctx* c, const int32_t* active_idx, const int64_t* active_offsets,
                                 int64_t n_active, double* acc, double* jerk, double* pot) {
  if (!c || n_active < 0 || n_active > c->n) return NBODY_E_INVAL;
  if (n_active == 0) return NBODY_OK;
  if (!active_idx || !active_offsets || !acc || !jerk) return NBODY_E_INVAL;
  if (!c->predicted) return NBODY_E_STATE;
  if (!c->scratch) return NBODY_E_HIP;
  if (planned_rows_bound(c, n_active) > kScratchRows) return NBODY_E_INVAL;
  DevState s = c->s;
  s.part = c->scratch;  // every row a pass reads is written by that pass first: nothing to clear
  s.rows_cap = kScratchRows;
  return force_pass(c, s, active_idx, active_offsets, n_active, acc, jerk, pot, false);
}

nbody_status nbody_perturbers(nbody_ctx* c, const int32_t* active_idx, const int64_t* active_offsets,
                              int64_t n_active, const double* threshold, int32_t max_pert, int32_t* lists,
                              int32_t* counts) {
  if (!c || n_active < 0 || n_active > c->n || max_pert < 1 || max_pert > kMaxPerturbers) return NBODY_E_INVAL;
  if (n_active == 0) return NBODY_OK;
  if (!active_idx || !active_offsets || !threshold || !lists || !counts) return NBODY_E_INVAL;
  if (!c->predicted) return NBODY_E_STATE;
  const nbody_status r = complete_prediction(c);
  if (r != NBODY_OK) return r;
  HIP_OK(launch_perturbers(c->s, active_idx, active_offsets, n_active, threshold, max_pert, lists, counts,
                           c->stream));
  return NBODY_OK;
}

nbody_status nbody_correct(nbody_ctx* c, const int32_t* active_idx, const int64_t* active_offsets, int64_t n_active,
                           const double* acc, const double* jerk) {
  if (!c || n_active < 0 || n_active > c->n) return NBODY_E_INVAL;
  if (n_active == 0) return NBODY_OK;
  if (!active_idx || !active_offsets || !acc || !jerk) return NBODY_E_INVAL;
  if (!c->predicted) return NBODY_E_STATE;
  const nbody_status r = complete_prediction(c);
  if (r != NBODY_OK) return r;
  c->sel_valid = false;  // t and dt change
  HIP_OK(launch_map_active(c->s, active_idx, n_active, c->stream));  // particle ids -> slots
  HIP_OK(launch_correct(c->s, c->s.ulist, active_offsets, n_active, acc, jerk, c->stream));
  return NBODY_OK;
}

nbody_status nbody_step(nbody_ctx* c, int32_t n_block_steps, double t_end) {
  if (!c || n_block_steps < 0 || !(t_end >= 0.0) || !isfinite(t_end)) return NBODY_E_INVAL;
  if (fmod(t_end, c->p.dt_max) != 0.0) return NBODY_E_INVAL;
  // a device error the host has already read: the state is frozen (the
  // selection kernel takes no step while the status word holds an error)
  if (c->seen_bits) return status_from_bits(c->seen_bits);
  if (n_block_steps == 0) return NBODY_OK;
  if (!c->gexec_k || c->graph_mode != force_mode(c) || c->graph_pot != c->p.compute_pot) {
    const nbody_status r = build_graph(c);
    if (r != NBODY_OK) return r;
  }
  if (c->ctl.t_end != t_end) {
    c->ctl.t_end = t_end;
    HIP_OK(hipMemcpyAsync(&c->s.ctl->t_end, &c->ctl.t_end, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
  }
  if (!c->sel_valid) {
    HIP_OK(launch_select_init(c->s, c->parity, c->stream));
    c->sel_valid = true;
  }
  // runs of kStepsPerGraph steps start (and end) at parity 0
  for (int32_t left = n_block_steps; left > 0;) {
    if (c->parity == 0 && left >= kStepsPerGraph) {
      HIP_OK(hipGraphLaunch(c->gexec_k, c->stream));
      left -= kStepsPerGraph;
    } else {
      HIP_OK(hipGraphLaunch(c->gexec[c->parity], c->stream));
      c->parity ^= 1;
      left -= 1;
    }
  }
  c->predicted = true;
  c->pred_full = false;
  return NBODY_OK;
}

nbody_status nbody_sync(nbody_ctx* c) {
  if (!c) return NBODY_E_INVAL;
  HIP_OK(hipStreamSynchronize(c->stream));
  int32_t bits = 0;
  HIP_OK(hipMemcpy(&bits, c->s.status, sizeof(int32_t), hipMemcpyDeviceToHost));
  c->seen_bits |= bits;
  return status_from_bits(bits);
}

nbody_status nbody_diagnostics(nbody_ctx* c, double* out_host) {
  if (!c || !out_host) return NBODY_E_INVAL;
  const DevState& s = c->s;
  HIP_OK(hipMemcpyAsync(s.tpred, s.tnow, 8 * (size_t)c->nc, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(launch_predict_all(s, c->stream));
  c->pred_full = true;
  c->sel_valid = false;  // the plan is replaced
  nbody_status r = force_all_internal(c, kF64);
  if (r != NBODY_OK) return r;
  double* eout = (double*)(c->ws + c->L.eout);
  HIP_OK(launch_diag(s, eout, c->stream));
  HIP_OK(hipMemcpyAsync(out_host, eout, 64 * (size_t)c->nc, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  c->predicted = true;
  return nbody_sync(c);
}

nbody_status nbody_energy(nbody_ctx* c, double* E_host) {
  if (!c || !E_host) return NBODY_E_INVAL;
  std::vector<double> d(8 * (size_t)c->nc);
  const nbody_status r = nbody_diagnostics(c, d.data());
  if (r != NBODY_OK) return r;
  for (int i = 0; i < c->nc; ++i) E_host[i] = d[8 * (size_t)i] + d[8 * (size_t)i + 1];
  return NBODY_OK;
}

nbody_status nbody_progress(nbody_ctx* c, double* t_host, int64_t* steps_host, double* inter_host) {
  if (!c) return NBODY_E_INVAL;
  const size_t C = (size_t)c->nc;
  if (t_host) HIP_OK(hipMemcpyAsync(t_host, c->s.tnow, 8 * C, hipMemcpyDeviceToHost, c->stream));
  if (steps_host) HIP_OK(hipMemcpyAsync(steps_host, c->s.steps, 8 * C, hipMemcpyDeviceToHost, c->stream));
  if (inter_host) HIP_OK(hipMemcpyAsync(inter_host, c->s.inter, 8 * C, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return NBODY_OK;
}

// State blob: header {magic, version, n (int64), nc (int32), pad} then
// coff[nc+1] (int64), eps[nc], order[n], slot_of[n] (int32: the storage
// order), then in storage order m[n], x[3n], v[3n], a[3n], k[3n], t[n],
// dt[n], and tnow[nc], inter[nc] (FP64), steps[nc] (int64).
nbody_status nbody_state_bytes(const nbody_ctx* c, size_t* bytes) {
  if (!c || !bytes) return NBODY_E_INVAL;
  const size_t N = (size_t)c->n, C = (size_t)c->nc;
  *bytes = 24 + 8 * (C + 1) + 8 * C + 8 * N + 8 * (15 * N) + 8 * 3 * C;
  return NBODY_OK;
}


nbody_status nbody_get_state(nbody_ctx* c, void* host_buf, size_t bytes) {
  size_t need = 0;
  if (!c || !host_buf || nbody_state_bytes(c, &need) != NBODY_OK || bytes < need) return NBODY_E_INVAL;
  unsigned char* h = (unsigned char*)host_buf;
  const uint32_t hdr[2] = {kStateMagic, kStateVersion};
  memcpy(h, hdr, 8);
  memcpy(h + 8, &c->n, 8);
  const int32_t nc2[2] = {c->nc, 0};
  memcpy(h + 16, nc2, 8);
  size_t o = 24;
  for (const Part& p : state_parts(c)) {
    HIP_OK(hipMemcpyAsync(h + o, c->ws + p.off, p.bytes, hipMemcpyDeviceToHost, c->stream));
    o += p.bytes;
  }
  HIP_OK(hipStreamSynchronize(c->stream));
  return NBODY_OK;
}

nbody_status nbody_set_state(nbody_ctx* c, const void* host_buf, size_t bytes) {
  size_t need = 0;
  if (!c || !host_buf || nbody_state_bytes(c, &need) != NBODY_OK || bytes < need) return NBODY_E_INVAL;
  const unsigned char* h = (const unsigned char*)host_buf;
  uint32_t hdr[2];
  int64_t n;
  int32_t nc2[2];
  memcpy(hdr, h, 8);
  memcpy(&n, h + 8, 8);
  memcpy(nc2, h + 16, 8);
  if (hdr[0] != kStateMagic || hdr[1] != kStateVersion || n != c->n || nc2[0] != c->nc) return NBODY_E_INVAL;
  if (memcmp(h + 24, c->coff.data(), 8 * ((size_t)c->nc + 1)) != 0) return NBODY_E_INVAL;
  // the storage order of the blob: every slot holds a particle of its own
  // cluster, and slot_of inverts order
  const size_t N = (size_t)c->n;
  std::vector<int32_t> order(N), slot_of(N);
  const size_t oo = 24 + 8 * ((size_t)c->nc + 1) + 8 * (size_t)c->nc;
  memcpy(order.data(), h + oo, 4 * N);
  memcpy(slot_of.data(), h + oo + 4 * N, 4 * N);
  for (int cc = 0; cc < c->nc; ++cc) {
    for (int64_t q = c->coff[cc]; q < c->coff[cc + 1]; ++q) {
      const int32_t id = order[(size_t)q];
      if (id < c->coff[cc] || id >= c->coff[cc + 1] || slot_of[(size_t)id] != q) return NBODY_E_INVAL;
    }
  }
  c->order = order;
  size_t o = 24;
  for (const Part& p : state_parts(c)) {
    HIP_OK(hipMemcpyAsync(c->ws + p.off, h + o, p.bytes, hipMemcpyHostToDevice, c->stream));
    o += p.bytes;
  }
  // a restored state starts with no recorded device error
  HIP_OK(hipMemsetAsync(c->s.status, 0, sizeof(int32_t), c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  c->seen_bits = 0;
  c->sel_valid = false;
  // the prediction no longer matches the state
  HIP_OK(hipMemcpyAsync(c->s.tpred, c->s.tnow, 8 * (size_t)c->nc, hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(launch_predict_all(c->s, c->stream));
  c->predicted = true;
  c->pred_full = true;
  return NBODY_OK;
}

nbody_status nbody_get_layout(const nbody_ctx* c, nbody_layout* out) {
  if (!c || !out) return NBODY_E_INVAL;
  memset(out, 0, sizeof(*out));
  out->n_total = c->n;
  out->n_clusters = c->nc;
  out->m = c->L.m;
  out->x = c->L.x;
  out->v = c->L.v;
  out->a = c->L.a;
  out->k = c->L.k;
  out->t = c->L.t;
  out->dt = c->L.dt;
  out->xp = c->L.xp;
  out->vp = c->L.vp;
  out->pot = c->L.pot;
  out->order = c->L.order;
  return NBODY_OK;
}

nbody_status nbody_get_tuning(const nbody_ctx* c, nbody_tuning* t) {
  if (!c || !t) return NBODY_E_INVAL;
  t->target_items = c->target_items;
  for (int i = 0; i < kNumVariants - 1; ++i) t->min_block[i] = c->ctl.vmin[i];
  t->small_cluster_n = (int32_t)c->ctl.small_n;
  for (int i = 0; i < kNumVariants - 1; ++i) t->small_min_block[i] = c->ctl.vmin_small[i];
  t->grid = c->grid;
  t->mixed_format = c->mixed_mode == kTR ? 2 : c->mixed_mode == kMX64 ? 1 : 0;
  t->rsq_bias_correct = c->rsq_correct;
  t->near_tau = c->ctl.near_tau;
  t->near_tau_k = c->ctl.near_tau_k;
  t->mid_tau = c->ctl.mid_tau;
  t->window = c->kwindow;
  t->waves = c->kwaves;
  t->tile = c->ktile;
  t->pred_in_force = c->pif;
  return NBODY_OK;
}

nbody_status nbody_set_tuning(nbody_ctx* c, const nbody_tuning* t) {
  if (!c || !t) return NBODY_E_INVAL;
  if (t->target_items < 1 || t->target_items > kMaxTargetItems || t->grid < 1 || t->grid > (1 << 20))
    return NBODY_E_INVAL;
  if (t->mixed_format < 0 || t->mixed_format > 2) return NBODY_E_INVAL;
  if (t->rsq_bias_correct != 0 && t->rsq_bias_correct != 1) return NBODY_E_INVAL;
  if (!(t->near_tau >= 0.0) || !isfinite(t->near_tau)) return NBODY_E_INVAL;
  if (!(t->near_tau_k >= 0.0) || !isfinite(t->near_tau_k)) return NBODY_E_INVAL;
  if (!(t->mid_tau > 0.0) || !isfinite(t->mid_tau)) return NBODY_E_INVAL;
  for (int i = 0; i < kNumVariants - 1; ++i) {
    if (t->min_block[i] < 1 || t->small_min_block[i] < 1) return NBODY_E_INVAL;
    if (i > 0 && t->min_block[i - 1] < t->min_block[i]) return NBODY_E_INVAL;
    if (i > 0 && t->small_min_block[i - 1] < t->small_min_block[i]) return NBODY_E_INVAL;
  }
  if (t->small_cluster_n < 0 || (t->pred_in_force != 0 && t->pred_in_force != 1)) return NBODY_E_INVAL;
  if ((t->window != 16 && t->window != 32 && t->window != 64) || t->waves < 2 || t->waves > 5) return NBODY_E_INVAL;
  if ((t->tile != 128 && t->tile != kTile) || (t->tile == 128 && t->window == 64)) return NBODY_E_INVAL;
  c->target_items = t->target_items;
  c->grid = t->grid;
  c->mixed_mode = t->mixed_format == 2 ? kTR : t->mixed_format == 1 ? kMX64 : kDS;
  const bool recal = c->rsq_correct != t->rsq_bias_correct;
  c->rsq_correct = t->rsq_bias_correct;
  c->ctl.near_tau = t->near_tau;
  c->ctl.near_tau_k = t->near_tau_k;
  c->ctl.mid_tau = t->mid_tau;
  c->kwindow = t->window;
  c->kwaves = t->waves;
  c->ktile = t->tile;
  for (int i = 0; i < kNumVariants - 1; ++i) c->ctl.vmin[i] = t->min_block[i];
  for (int i = 0; i < kNumVariants - 1; ++i) c->ctl.vmin_small[i] = t->small_min_block[i];
  c->ctl.small_n = t->small_cluster_n;
  c->pif = t->pred_in_force;
  destroy_graph(c);  // the captured step bakes in grid, plan target and format
  // the step pipeline's carried-over state (with one cluster, the previous
  // step's plan is recomputed from its count) assumes the plan settings it
  // was made with: rebuild it at the next step
  c->sel_valid = false;
  const nbody_status r = upload_ctl(c);
  if (r == NBODY_OK && recal) HIP_OK(launch_rsq_bias(c->s, c->rsq_correct, c->stream));
  return r;
}

nbody_status nbody_profile_force(nbody_ctx* c, int32_t enable) {
  if (!c) return NBODY_E_INVAL;
  c->profile = enable != 0;
  return NBODY_OK;
}

nbody_status nbody_profile_read(nbody_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return NBODY_E_INVAL;
  HIP_OK(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (auto& ev : c->prof_pending) {
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, ev.first, ev.second));
    total += t;
    c->prof_free.push_back(ev);
  }
  *launches = (int64_t)c->prof_pending.size();
  *ms = total;
  c->prof_pending.clear();
  return NBODY_OK;
}

nbody_status nbody_destroy(nbody_ctx* c) {
  if (!c) return NBODY_OK;
  for (auto& ev : c->prof_pending) c->prof_free.push_back(ev);
  for (auto& ev : c->prof_free) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  destroy_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return NBODY_OK;
}

const char* nbody_strerror(nbody_status s) {
  switch (s) {
    case NBODY_OK: return "ok";
    case NBODY_E_INVAL: return "invalid argument";
    case NBODY_E_NOMEM: return "workspace too small or host allocation failed";
    case NBODY_E_HIP: return "HIP runtime error";
    case NBODY_E_STATE: return "call out of order";
    case NBODY_E_DTMIN: return "time step fell below dt_min";
    case NBODY_E_NONFINITE: return "non-finite value in the state or forces";
    case NBODY_E_INDEX: return "active index outside its cluster or inconsistent active offsets";
  }
  return "unknown status";
}

}  // extern "C"
