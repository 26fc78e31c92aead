// Host-runtime objects shared by the C ABI implementation (lge_host.cpp)
// and the serving scheduler (lge_server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <map>
#include <vector>

#include "../../include/lge.h"
#include "lge_hostmath.h"
#include "lge_internal.h"

using lge::Bins;
using lge::kNumClasses;
using lge::RangeDesc;
using lge::SlotDesc;

struct lge_graph {
  lge_ctx *ctx = nullptr;
  int64_t n = 0, m = 0;
  int32_t max_deg = 0;
  const int32_t *row_ptr = nullptr;
  const int32_t *col = nullptr;
  int32_t *own_row_ptr = nullptr;
  int32_t *own_col = nullptr;
  uint64_t *edges = nullptr;
  int64_t *vol2 = nullptr;
  int64_t *hoff = nullptr;
  uint32_t *htab = nullptr;
  int64_t htab_len = 0;
  int32_t *crank = nullptr;
  uint16_t *codeg = nullptr;  // hc x hc co-degrees, 16 bits (see codeg_sat)
  int64_t hc = 0;
  int32_t codeg_sat = 0;      // first rank of degree >= 65535 (hc if none)
  unsigned long long *hbits = nullptr;  // hc x hcw adjacency bit rows of the ranked vertices
  int64_t hcw = 0;
  int4 *vinfo = nullptr;     // n: (row start, degree, rank or -1, co-degree row or -1)
  uint32_t *arh = nullptr;   // 2m: packed rank word of every arc's head
  int32_t *hrow = nullptr;   // n: co-degree row index, -1 if none (graph creation only)
  int32_t *rcol = nullptr;   // n: column in the co-degree rows, -1 if none (graph creation only)
  int32_t *row_hubs = nullptr;  // nrows: vertex of every co-degree row (graph creation only)
  int64_t ncol = 0;             // columns of the co-degree rows
  uint8_t *rows = nullptr;   // nrows x rows_stride co-degree rows over the unranked vertices
  int64_t nrows = 0, rows_stride = 0;  // rows, columns per row
  int32_t rows_w = 0;                 // bytes per entry (1 or 2)
  int32_t rows_floor = 0;             // unranked vertices above this degree have a column
  int32_t codeg_tau = 0;
  double work_per_id = 0.0;  // scheduling weight per canonical edge id
  // cumulative scheduling weight at every kWorkBlock-th canonical edge id
  // (host; the last entry is the whole graph's)
  std::vector<double> work_pref;
  double build_ms = 0.0;     // preprocessing wall time (after validation and the edge list)
  // micro statistics, built on first use: t of every arc, triangles per
  // vertex, the arcs' t at the hub-table slots, and a small reduction buffer
  // (column maxima, error flag)
  int32_t *t_arc = nullptr;
  int64_t *tri = nullptr;
  int32_t *t_slot = nullptr;  // htab_len: t of every arc at its head's slot of the tail's hub table
  unsigned long long *mred = nullptr;
  // weighted sampling, built on first use: k-core numbers, and per weight
  // mode (1 degree, 2 k-core) the class of every edge and the class sizes
  int32_t *core = nullptr;
  int32_t max_core = -1;
  uint8_t *wlevel[2] = {nullptr, nullptr};
  uint64_t whist[2][16] = {};
};

struct Workspace {
  int64_t cap_edges = 0;  // capacity of each class list
  int32_t cap_slots = 0;
  int32_t cap_ranges = 0;
  int32_t *bin_slot[kNumClasses] = {};
  int32_t *bin_a[kNumClasses] = {};
  int32_t *bin_b[kNumClasses] = {};
  // device control block: kNumCtrs counters followed by the per-slot
  // accumulators (cap_slots * kAccSlots * 2), zeroed by one kernel and read
  // back by one copy per launch sequence; pinned host mirror h_ctl
  unsigned long long *ctl = nullptr;
  unsigned long long *counters = nullptr;  // ctl
  unsigned long long *acc = nullptr;       // ctl + kNumCtrs
  // job descriptors: cap_ranges RangeDesc followed by cap_slots SlotDesc,
  // written by one copy; pinned host mirror h_desc
  void *desc = nullptr;
  RangeDesc *ranges = nullptr;
  SlotDesc *slots = nullptr;
  int64_t *items = nullptr;           // cap_edges
  int64_t *item_pref = nullptr;       // cap_edges
  int64_t *tcap = nullptr;            // cap_edges
  int64_t *tbase = nullptr;           // cap_edges
  int32_t *item_edge = nullptr;       // cap_items: split-class work item -> edge
  unsigned long long *tmask = nullptr;  // cap_items x kGlobalChunkMax/64: T_e membership of item positions
  int64_t cap_items = 0;
  int32_t *tlist = nullptr;           // 3 * cap_tlist: (id, degree, rank) of T_e members
  unsigned long long *tbw = nullptr;  // cap_tlist: non-zero words of the ranked-member bit sets
  int16_t *tbi = nullptr;             // cap_tlist: their word indices
  int64_t cap_tlist = 0;              // T_e entries
  void *gacc = nullptr;               // cap_edges * gedge_bytes()
  int64_t *scan_tmp = nullptr;
  int64_t scan_tmp_len = 0;
  // split-class edges reordered by table-side endpoint (cap_edges each)
  int32_t *sort_slot = nullptr;
  int32_t *sort_a = nullptr;
  int32_t *sort_b = nullptr;
  int64_t *sort_hist = nullptr;  // kSortKeys
  int64_t *sort_off = nullptr;   // kSortKeys
  int64_t *sort_tmp = nullptr;   // scan scratch for kSortKeys
  // pinned host staging
  void *h_desc = nullptr;
  RangeDesc *h_ranges = nullptr;
  SlotDesc *h_slots = nullptr;
  unsigned long long *h_ctl = nullptr;
  unsigned long long *h_counters = nullptr;  // h_ctl
  unsigned long long *h_acc = nullptr;       // h_ctl + kNumCtrs
};

struct lge_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Workspace ws;
  // allocation-free estimate: the device's scratch array (looked up at open)
  // and pinned staging for one range, one slot and its accumulator replicas
  void *scratch = nullptr;
  void *na_h_desc = nullptr;
  unsigned long long *na_h_ctl = nullptr;
  lge_opts opts{};
  // autotuned options per graph class (bit lengths of m and of the maximum
  // degree, p in quarter octaves)
  std::map<std::array<int32_t, 3>, lge_opts> tuned;
  // split-class list bytes one launch sequence may hold (a quarter of the
  // device's memory), and what the last sequence over it asked for
  int64_t list_budget = (int64_t)16 << 30;
  int64_t list_need = 0;
  // caps on the co-degree table and co-degree row bytes of graphs created
  // on this context (0: the library's own budgets)
  int64_t codeg_budget = 0;
  int64_t rows_budget = 0;
  // cap on a graph creation's temporary row-fill scratch (0: the default)
  int64_t build_scratch = 0;
  lge_timing timing{};
  hipEvent_t ev[8] = {};
  int num_cu = 256;
};


// One estimate job of a launch sequence: a canonical edge-id range of a
// resident graph with its own p and seed.
struct Job {
  const lge_graph *g;
  double p;
  uint64_t seed;
  int64_t e0, e1;       // canonical edge range (of the graph's own ids)
  int64_t n_override;   // graph-level sizes for the closed forms (batch unions)
  int64_t m_override;
  int64_t eid_base;     // subtracted from edge ids before the sampler
  double p_lo = 0.0;    // sample only edges whose uniform is >= p_lo (adaptive rounds)
  long long *micro = nullptr;  // per-edge (t, k4, cyc) write-out rows for [e0, e1)
  int32_t design = 0;          // lge::SampleDesign
  const uint8_t *level = nullptr;
  const double *plev = nullptr;  // kWeightLevels class probabilities (host)
  uint64_t kkey = 0;
  int64_t keid = -1;
};

// Slot of job j's first accumulator: jobs take one slot each, weighted jobs
// kWeightLevels (one per class).
int lge_job_slots(const Job &j);

// Runs sample -> bin -> count for the jobs in one launch sequence on the
// ctx stream; on success the per-slot accumulators (kAccSlots x {lo, hi}) are
// in ctx->ws.h_acc, job j's from slot sum_{i<j} lge_job_slots(job i).
// Returns an LGE_* code.
int lge_run_jobs(lge_ctx *ctx, const Job *jobs, int njobs, const lge_opts *opts);

// lge_finalize (exact integers -> lge_result) is declared in lge_hostmath.h.

// Device bytes a context's workspace holds per canonical edge id of a launch
// sequence (class lists, split-class per-edge arrays and records, sort
// arrays, scan scratch), and the bytes its workspace holds now in all.
int64_t lge_ws_bytes_per_id();
int64_t lge_ws_bytes(const lge_ctx *ctx);
