// Host runtime of the C ABI declared in include/lge.h: contexts, resident
// graphs, workspaces, the estimate / batch launch sequences and the exact
// integer -> FP64 finalisation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/lge.h"
#include "lge_hostmath.h"
#include "lge_internal.h"
#include "lge_runtime.h"

using namespace lge;

namespace {

// Co-degree table: ranked vertices of degree > kCodegMinDeg, at most
// kMaxRanked of them and hc^2 * 4 bytes within kCodegBytes and
// kCodegPerCsr times the graph's CSR bytes (kCodegBytesCompact with
// LGE_FLAG_COMPACT, or when the first allocation fails).  The budgets depend
// on the graph only, so a graph's build and speed do not depend on what else
// is resident.
constexpr double kCodegBytes = 34359738368.0;       // 32 GiB: 131008 ranked vertices (2-byte entries)
constexpr double kCodegBytesCompact = 1073741824.0;  // 1 GiB: 23168
constexpr double kCodegPerCsr = 64.0;
// Ranked vertices above this degree get a co-degree row over the unranked
// vertices (largest degrees first, while the build work, the sum of their
// 2-hop volumes, and the memory stay within these budgets).  Every ranked
// vertex qualifies: the rows of mid-degree vertices serve the wavefront and
// workgroup classes, whose b rarely exceeds degree 1024.
constexpr int32_t kRowDeg = 96;
// co-degree rows: build work (sum of 2-hop volumes) and HBM per graph, the
// bytes also within kRowsPerCsr times the CSR bytes; LGE_FLAG_COMPACT (or a
// failed first allocation) keeps the small budgets.
constexpr double kRowBudgetOps = 1.5e11;
constexpr double kRowBudgetBytes = 32e9;
constexpr double kRowsPerCsr = 256.0;
constexpr double kRowBudgetOpsCompact = 4e9;
constexpr double kRowBudgetBytesCompact = 4e9;
// default cap on the scratch for the row fill's segment ends (freed when
// the graph is built)
constexpr int64_t kRowsOffBytes = (int64_t)1 << 30;
// Ranked vertices have degree > kCodegMinDeg: a walk of a shorter row costs
// about as much as the table read that replaces it.
constexpr int32_t kCodegMinDeg = 96;

#define LGE_HIP(expr)                        \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return hip_err(e_); \
  } while (0)

int hip_err(hipError_t e) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LGE_ENOMEM;
  return LGE_EDEVICE;
}

template <typename T>
int dev_alloc(T **p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return LGE_OK;
  hipError_t e = hipMalloc((void **)p, (size_t)count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    // a failed allocation stays the thread's last error, which the launch
    // wrappers read back after their launches: clear it, so a caller that
    // retries smaller (or gives up) is not handed it again
    (void)hipGetLastError();
    return hip_err(e);
  }
  return LGE_OK;
}

// a direct hipMalloc / hipHostMalloc failed: the same clearing, and ENOMEM
static int alloc_failed() {
  (void)hipGetLastError();
  return LGE_ENOMEM;
}

template <typename T>
void dev_free(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------

struct lge_event {
  std::thread worker;  // runs the launch sequence and the finalisation
  int status = LGE_OK;
};

// ---------------------------------------------------------------------------
// errors, options
// ---------------------------------------------------------------------------

extern "C" const char *lge_strerror(int code) {
  switch (code) {
    case LGE_OK: return "ok";
    case LGE_EINVAL: return "invalid argument";
    case LGE_ENOMEM: return "out of memory";
    case LGE_EGRAPH: return "invalid graph (CSR must be sorted, symmetric, loop-free and simple)";
    case LGE_EDEVICE: return "HIP device error or no usable GPU";
    case LGE_ERANGE: return "graph too large for exact 128-bit sums";
    case LGE_EBUSY: return "server queue full";
    case LGE_ETIMEDOUT: return "timed out";
    case LGE_ECANCELED: return "cancelled";
    case LGE_ENOTFOUND: return "not found";
    case LGE_EINTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

extern "C" int lge_opts_default(lge_opts *o) {
  if (!o) return LGE_EINVAL;
  memset(o, 0, sizeof(*o));
  o->wave_max_deg = 256;
  o->block_max_deg = kHubDeg;
  o->probe_ratio = 4;
  o->grid_per_cu = 0;
  o->global_chunk = kGlobalChunkMax;
  o->flags = LGE_OPT_SORT_HUB | LGE_OPT_XCD_LOCAL;
  return LGE_OK;
}

static KernelCfg make_cfg(const lge_ctx *ctx, const lge_opts *o) {
  lge_opts d;
  lge_opts_default(&d);
  if (!o) o = &ctx->opts;
  KernelCfg c;
  int wmd = o->wave_max_deg > 0 ? o->wave_max_deg : d.wave_max_deg;
  c.wave_max_deg = std::min(std::max(wmd, 1), 512);
  c.block_max_deg = o->block_max_deg > 0 ? std::min(o->block_max_deg, kHubDeg) : kHubDeg;
  c.probe_ratio = o->probe_ratio >= 0 ? o->probe_ratio : d.probe_ratio;
  const int per_cu = o->grid_per_cu > 0 ? o->grid_per_cu : 0;
  const int cu = ctx->num_cu > 0 ? ctx->num_cu : 256;
  c.grid_wave = cu * (per_cu ? per_cu : 24);
  c.grid_block = cu * (per_cu ? per_cu : 8);
  c.grid_global = cu * (per_cu ? per_cu : 4);  // 512-thread workgroups
  if (o->grid_share > 0 && o->grid_share < 100) {  // a share of each grid, whole multiples of kXcds
    auto part = [&](int32_t g) {
      return std::max<int32_t>(kXcds, (int32_t)((int64_t)g * o->grid_share / 100) / kXcds * kXcds);
    };
    c.grid_wave = part(c.grid_wave);
    c.grid_block = part(c.grid_block);
    c.grid_global = part(c.grid_global);
  }
  c.grid_sample = cu * 16;
  c.global_chunk = o->global_chunk > 0 ? std::min<int32_t>(o->global_chunk, kGlobalChunkMax) : d.global_chunk;
  c.flags = o->flags;
  c.list_budget = o->max_list_mib > 0 ? (int64_t)o->max_list_mib << 20 : ctx->list_budget;
  return c;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

static void ws_free(Workspace &w) {
  for (int c = 0; c < kNumClasses; ++c) {
    dev_free(w.bin_slot[c]);
    dev_free(w.bin_a[c]);
    dev_free(w.bin_b[c]);
  }
  dev_free(w.ctl);
  if (w.desc) (void)hipFree(w.desc);
  dev_free(w.items);
  dev_free(w.item_pref);
  dev_free(w.tcap);
  dev_free(w.tbase);
  dev_free(w.tlist);
  dev_free(w.tbw);
  dev_free(w.tbi);
  dev_free(w.item_edge);
  dev_free(w.tmask);
  if (w.gacc) (void)hipFree(w.gacc);
  w.gacc = nullptr;
  dev_free(w.scan_tmp);
  dev_free(w.sort_slot);
  dev_free(w.sort_a);
  dev_free(w.sort_b);
  dev_free(w.sort_hist);
  dev_free(w.sort_off);
  dev_free(w.sort_tmp);
  if (w.h_desc) (void)hipHostFree(w.h_desc);
  if (w.h_ctl) (void)hipHostFree(w.h_ctl);
  w = Workspace();
}

static int ws_reserve(lge_ctx *ctx, int64_t edges, int32_t slots, int32_t ranges);

extern "C" int lge_open(int device, lge_ctx **out) {
  if (!out) return LGE_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return LGE_EDEVICE;
  if (device < 0 || device >= count) return LGE_EDEVICE;
  lge_ctx *ctx = new (std::nothrow) lge_ctx();
  if (!ctx) return LGE_ENOMEM;
  ctx->device = device;
  lge_opts_default(&ctx->opts);
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return LGE_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cu = prop.multiProcessorCount;
  size_t mem_free = 0, mem_total = 0;
  if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_total > 0)
    ctx->list_budget = (int64_t)(mem_total / 4);
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return LGE_EDEVICE;
  }
  for (auto &e : ctx->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      lge_close(ctx);
      return LGE_EDEVICE;
    }
  }
  // the device's scratch array for the allocation-free estimate, and its
  // pinned staging (one range, one slot, kAccReplicas accumulator replicas)
  if (scratch_address(device, &ctx->scratch) != hipSuccess) {
    lge_close(ctx);
    return LGE_EDEVICE;
  }
  if (hipHostMalloc(&ctx->na_h_desc, sizeof(RangeDesc) + sizeof(SlotDesc), 0) != hipSuccess ||
      hipHostMalloc((void **)&ctx->na_h_ctl,
                    (size_t)(kNumCtrs + (int64_t)kAccReplicas * kAccSlots * 2) * sizeof(unsigned long long),
                    0) != hipSuccess) {
    lge_close(ctx);
    return LGE_ENOMEM;
  }
  Workspace &w = ctx->ws;
  if (ws_reserve(ctx, 0, kAccReplicas, 16) != LGE_OK || dev_alloc(&w.sort_hist, kSortKeys) != LGE_OK ||
      dev_alloc(&w.sort_off, kSortKeys) != LGE_OK ||
      dev_alloc(&w.sort_tmp, scan_tmp_size(kSortKeys)) != LGE_OK) {
    lge_close(ctx);
    return LGE_ENOMEM;
  }
  *out = ctx;
  return LGE_OK;
}

extern "C" int lge_close(lge_ctx *ctx) {
  if (!ctx) return LGE_EINVAL;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ws_free(ctx->ws);
  if (ctx->na_h_desc) (void)hipHostFree(ctx->na_h_desc);
  if (ctx->na_h_ctl) (void)hipHostFree(ctx->na_h_ctl);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return LGE_OK;
}

// grows the workspace to hold `edges` binned edges, `slots` slots, `ranges` ranges
static int ws_reserve(lge_ctx *ctx, int64_t edges, int32_t slots, int32_t ranges) {
  Workspace &w = ctx->ws;
  if (edges > w.cap_edges) {
    int64_t cap = std::max<int64_t>(edges, 1024);
    for (int c = 0; c < kNumClasses; ++c) {
      dev_free(w.bin_slot[c]);
      dev_free(w.bin_a[c]);
      dev_free(w.bin_b[c]);
    }
    dev_free(w.items);
    dev_free(w.item_pref);
    dev_free(w.tcap);
    dev_free(w.tbase);
    if (w.gacc) (void)hipFree(w.gacc);
    w.gacc = nullptr;
    dev_free(w.scan_tmp);
    dev_free(w.sort_slot);
    dev_free(w.sort_a);
    dev_free(w.sort_b);
    w.cap_edges = 0;
    for (int c = 0; c < kNumClasses; ++c) {
      int rc;
      if ((rc = dev_alloc(&w.bin_slot[c], cap)) != LGE_OK) return rc;
      if ((rc = dev_alloc(&w.bin_a[c], cap)) != LGE_OK) return rc;
      if ((rc = dev_alloc(&w.bin_b[c], cap)) != LGE_OK) return rc;
    }
    int rc;
    if ((rc = dev_alloc(&w.items, cap)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.item_pref, cap)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.tcap, cap)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.tbase, cap)) != LGE_OK) return rc;
    if (hipMalloc(&w.gacc, (size_t)cap * gedge_bytes()) != hipSuccess) {
      w.gacc = nullptr;
      return alloc_failed();
    }
    w.scan_tmp_len = scan_tmp_size(cap);
    if ((rc = dev_alloc(&w.scan_tmp, w.scan_tmp_len)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.sort_slot, cap)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.sort_a, cap)) != LGE_OK) return rc;
    if ((rc = dev_alloc(&w.sort_b, cap)) != LGE_OK) return rc;
    w.cap_edges = cap;
  }
  if (slots > w.cap_slots || ranges > w.cap_ranges) {
    const int32_t cs = std::max(std::max<int32_t>(slots, w.cap_slots), 16);
    const int32_t cr = std::max(std::max<int32_t>(ranges, w.cap_ranges), 16);
    dev_free(w.ctl);
    if (w.desc) (void)hipFree(w.desc);
    if (w.h_desc) (void)hipHostFree(w.h_desc);
    if (w.h_ctl) (void)hipHostFree(w.h_ctl);
    w.desc = w.h_desc = nullptr;
    w.h_ctl = nullptr;
    w.cap_slots = w.cap_ranges = 0;
    const int64_t nctl = kNumCtrs + (int64_t)cs * kAccSlots * 2;
    const size_t ndesc = (size_t)cr * sizeof(RangeDesc) + (size_t)cs * sizeof(SlotDesc);
    int rc;
    if ((rc = dev_alloc(&w.ctl, nctl)) != LGE_OK) return rc;
    if (hipMalloc(&w.desc, ndesc) != hipSuccess) {
      w.desc = nullptr;
      return alloc_failed();
    }
    if (hipHostMalloc((void **)&w.h_ctl, (size_t)nctl * sizeof(unsigned long long), 0) != hipSuccess) {
      w.h_ctl = nullptr;
      return alloc_failed();
    }
    if (hipHostMalloc(&w.h_desc, ndesc, 0) != hipSuccess) {
      w.h_desc = nullptr;
      return alloc_failed();
    }
    w.counters = w.ctl;
    w.acc = w.ctl + kNumCtrs;
    w.h_counters = w.h_ctl;
    w.h_acc = w.h_ctl + kNumCtrs;
    w.ranges = (RangeDesc *)w.desc;
    w.slots = (SlotDesc *)((char *)w.desc + (size_t)cr * sizeof(RangeDesc));
    w.h_ranges = (RangeDesc *)w.h_desc;
    w.h_slots = (SlotDesc *)((char *)w.h_desc + (size_t)cr * sizeof(RangeDesc));
    w.cap_slots = cs;
    w.cap_ranges = cr;
  }
  return LGE_OK;
}

static int ws_reserve_items(lge_ctx *ctx, int64_t len) {
  Workspace &w = ctx->ws;
  if (len <= w.cap_items) return LGE_OK;
  dev_free(w.item_edge);
  dev_free(w.tmask);
  w.cap_items = 0;
  const int64_t cap = std::max<int64_t>(len + len / 4, 4096);
  int rc = dev_alloc(&w.item_edge, cap);
  if (rc != LGE_OK) return rc;
  if ((rc = dev_alloc(&w.tmask, cap * (kGlobalChunkMax / 64))) != LGE_OK) return rc;
  w.cap_items = cap;
  return LGE_OK;
}

// room for `len` T_e entries: (id, degree, rank) triples plus the compact
// bit-set words
static int ws_reserve_tlist(lge_ctx *ctx, int64_t len) {
  Workspace &w = ctx->ws;
  if (len <= w.cap_tlist) return LGE_OK;
  dev_free(w.tlist);
  dev_free(w.tbw);
  dev_free(w.tbi);
  w.cap_tlist = 0;
  const int64_t cap = std::max<int64_t>(len + len / 4, 4096);
  int rc;
  if ((rc = dev_alloc(&w.tlist, 3 * cap)) != LGE_OK) return rc;
  if ((rc = dev_alloc(&w.tbw, cap)) != LGE_OK) return rc;
  if ((rc = dev_alloc(&w.tbi, cap)) != LGE_OK) return rc;
  w.cap_tlist = cap;
  return LGE_OK;
}

// device bytes of the split-class lists for `items` work items and `tl` T_e
// entries, as the two functions above allocate them
static int64_t list_bytes(int64_t items, int64_t tl) {
  return (items + items / 4) * (int64_t)(sizeof(int32_t) + (kGlobalChunkMax / 64) * sizeof(unsigned long long)) +
         (tl + tl / 4) * (int64_t)(3 * sizeof(int32_t) + sizeof(unsigned long long) + sizeof(int16_t));
}

int64_t lge_ws_bytes_per_id() {
  return (int64_t)(3 * kNumClasses * sizeof(int32_t)     // class lists (slot, a, b)
                   + 4 * sizeof(int64_t)                 // items, item_pref, tcap, tbase
                   + gedge_bytes()                       // per-edge records
                   + 3 * sizeof(int32_t)                 // sorted split-class lists
                   + 2 * sizeof(int64_t));               // scan scratch (bound)
}

int64_t lge_ws_bytes(const lge_ctx *ctx) {
  const Workspace &w = ctx->ws;
  int64_t b = w.cap_edges * lge_ws_bytes_per_id() + list_bytes(w.cap_items, w.cap_tlist) * 4 / 5;
  b += (int64_t)(kNumCtrs + (int64_t)w.cap_slots * kAccSlots * 2) * (int64_t)sizeof(unsigned long long);
  b += (int64_t)w.cap_ranges * (int64_t)sizeof(RangeDesc) + (int64_t)w.cap_slots * (int64_t)sizeof(SlotDesc);
  b += 3 * (int64_t)kSortKeys * (int64_t)sizeof(int64_t);
  return b;
}

// run_sequence's answer when the split-class lists would exceed the budget
constexpr int kRunSplit = 1 << 20;

// ---------------------------------------------------------------------------
// graph validation and creation
// ---------------------------------------------------------------------------



static int build_codeg(lge_ctx *ctx, lge_graph *g, const int32_t *host_row_ptr, uint32_t flags);
static int build_rows(lge_ctx *ctx, lge_graph *g, const int32_t *host_row_ptr, uint32_t flags);

// forget a partial co-degree table / co-degree rows (before a retry)
static void drop_codeg(lge_graph *g) {
  dev_free(g->crank);
  dev_free(g->codeg);
  dev_free(g->hbits);
  g->hc = g->hcw = 0;
}

static void drop_rows(lge_graph *g) {
  dev_free(g->hrow);
  dev_free(g->rcol);
  dev_free(g->row_hubs);
  dev_free(g->rows);
  g->nrows = g->rows_stride = g->ncol = 0;
}

static int graph_preprocess(lge_ctx *ctx, lge_graph *g, uint32_t flags, const int32_t *host_row_ptr) {
  const auto t_build = std::chrono::steady_clock::now();
  hipStream_t s = ctx->stream;
  const int64_t n = g->n;
  int rc;
  if (!(flags & LGE_FLAG_TRUSTED) && n > 0) {
    int *derr = nullptr;
    if ((rc = dev_alloc(&derr, 1)) != LGE_OK) return rc;
    int herr = 0;
    hipError_t e = hipMemsetAsync(derr, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_graph_validate(g->row_ptr, g->col, n, derr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(derr);
    if (e != hipSuccess) return hip_err(e);
    if (herr) return LGE_EGRAPH;
  }
  // canonical edge list
  int32_t *up = nullptr;
  int64_t *cnt = nullptr, *base = nullptr, *tmp = nullptr;
  const int64_t tl = scan_tmp_size(std::max<int64_t>(n, 1));
  if ((rc = dev_alloc(&up, std::max<int64_t>(n, 1))) != LGE_OK) return rc;
  if ((rc = dev_alloc(&cnt, std::max<int64_t>(n, 1))) != LGE_OK || (rc = dev_alloc(&base, std::max<int64_t>(n, 1))) != LGE_OK ||
      (rc = dev_alloc(&tmp, tl)) != LGE_OK) {
    dev_free(up);
    dev_free(cnt);
    dev_free(base);
    dev_free(tmp);
    return rc;
  }
  auto cleanup = [&]() {
    dev_free(up);
    dev_free(cnt);
    dev_free(base);
    dev_free(tmp);
  };
  hipError_t e = hipSuccess;
  if (g->m > 0) {
    if ((rc = dev_alloc(&g->edges, g->m)) != LGE_OK) {
      cleanup();
      return rc;
    }
  }
  if ((rc = dev_alloc(&g->vol2, std::max<int64_t>(n, 1))) != LGE_OK || (rc = dev_alloc(&g->hoff, std::max<int64_t>(n, 1))) != LGE_OK) {
    cleanup();
    return rc;
  }
  e = launch_graph_upper(g->row_ptr, g->col, n, up, cnt, s);
  if (e == hipSuccess) e = launch_scan_i64(cnt, base, n, tmp, s);
  int64_t last[2] = {0, 0};
  if (e == hipSuccess && n > 0) e = hipMemcpyAsync(&last[0], base + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && n > 0) e = hipMemcpyAsync(&last[1], cnt + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_err(e);
  }
  if (n > 0 && last[0] + last[1] != g->m) {
    cleanup();
    return LGE_EGRAPH;  // upper triangle does not hold half the entries
  }
  if (g->m > 0) e = launch_graph_edges(g->row_ptr, g->col, up, base, n, g->edges, s);
  if (e == hipSuccess) e = launch_graph_vol2(g->row_ptr, g->col, n, g->vol2, s);
  if (e == hipSuccess && g->m > 0) {
    // the work profile along the canonical edge ids, for chunking ranges by work
    const int64_t nb = (g->m + kWorkBlock - 1) / kWorkBlock;
    unsigned long long *wb = nullptr;
    if ((rc = dev_alloc(&wb, nb)) != LGE_OK) {
      cleanup();
      return rc;
    }
    std::vector<unsigned long long> hb((size_t)nb);
    e = launch_graph_work(g->row_ptr, g->edges, g->vol2, g->m, wb, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hb.data(), wb, (size_t)nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(wb);
    g->work_pref.assign((size_t)nb + 1, 0.0);
    for (int64_t k = 0; k < nb; ++k) g->work_pref[(size_t)k + 1] = g->work_pref[(size_t)k] + (double)hb[(size_t)k];
    g->work_per_id = g->work_pref.back() / (double)g->m;
  }
  // hub tables
  if (e == hipSuccess) e = launch_hub_sizes(g->row_ptr, n, cnt, s);
  if (e == hipSuccess) e = launch_scan_i64(cnt, g->hoff, n, tmp, s);
  if (e == hipSuccess && n > 0) e = hipMemcpyAsync(&last[0], g->hoff + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && n > 0) e = hipMemcpyAsync(&last[1], cnt + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_err(e);
  }
  g->htab_len = n > 0 ? last[0] + last[1] : 0;
  if (g->htab_len > 0) {
    if ((rc = dev_alloc(&g->htab, g->htab_len)) != LGE_OK) {
      cleanup();
      return rc;
    }
    e = launch_hub_build(g->row_ptr, g->col, n, g->hoff, g->htab, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_err(e);
  if (!(flags & LGE_FLAG_NO_TABLES)) {
    rc = build_codeg(ctx, g, host_row_ptr, flags);
    if (rc == LGE_ENOMEM && !(flags & LGE_FLAG_COMPACT)) {  // the small budgets, once
      drop_codeg(g);
      rc = build_codeg(ctx, g, host_row_ptr, flags | LGE_FLAG_COMPACT);
    }
    if (rc != LGE_OK) return rc;
    rc = build_rows(ctx, g, host_row_ptr, flags);
    if (rc == LGE_ENOMEM && !(flags & LGE_FLAG_COMPACT)) {
      drop_rows(g);
      rc = build_rows(ctx, g, host_row_ptr, flags | LGE_FLAG_COMPACT);
    }
    if (rc != LGE_OK) return rc;
  }
  if ((rc = dev_alloc(&g->vinfo, std::max<int64_t>(n, 1))) != LGE_OK) return rc;
  if ((rc = dev_alloc(&g->arh, std::max<int64_t>(2 * g->m, 1))) != LGE_OK) return rc;
  const bool rows = g->nrows > 0;
  LGE_HIP(launch_vinfo(g->row_ptr, g->hc > 0 ? g->crank : nullptr, rows ? g->hrow : nullptr,
                       rows ? g->rcol : nullptr, n, g->vinfo, s));
  LGE_HIP(launch_arc_rank(g->col, g->vinfo, 2 * g->m, g->arh, s));
  // the co-degree rows, tile by tile, from every vertex's list of
  // neighbour columns (taken from the arc words), with the segment ends of
  // the lists at the tile bounds in a scratch buffer of at most
  // kRowsOffBytes or the context's cap (but two ends per vertex); all of it
  // freed here
  if (rows) {
    int64_t *ccnt = nullptr, *coff = nullptr, *tmp = nullptr;
    int32_t *clist = nullptr, *toff = nullptr;
    auto release = [&]() {
      dev_free(ccnt);
      dev_free(coff);
      dev_free(tmp);
      dev_free(clist);
      dev_free(toff);
    };
    if ((rc = dev_alloc(&ccnt, n)) != LGE_OK || (rc = dev_alloc(&coff, n)) != LGE_OK ||
        (rc = dev_alloc(&tmp, scan_tmp_size(n))) != LGE_OK) {
      release();
      return rc;
    }
    e = launch_col_count(g->row_ptr, g->arh, n, ccnt, s);
    if (e == hipSuccess) e = launch_scan_i64(ccnt, coff, n, tmp, s);
    int64_t last[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&last[0], coff + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&last[1], ccnt + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      release();
      return hip_err(e);
    }
    const int64_t ntiles = (g->ncol + rows_tile_entries(g->rows_w) - 1) / rows_tile_entries(g->rows_w);
    const int64_t cap = ctx->build_scratch > 0 ? ctx->build_scratch : kRowsOffBytes;
    int64_t toff_len = std::max<int64_t>(2 * n, std::min<int64_t>(n * (ntiles + 1), cap / 4));
    if ((rc = dev_alloc(&clist, std::max<int64_t>(last[0] + last[1], 1))) == LGE_OK) {
      rc = dev_alloc(&toff, toff_len);
      if (rc == LGE_ENOMEM && toff_len > 2 * n) {  // one tile per pass
        toff_len = 2 * n;
        rc = dev_alloc(&toff, toff_len);
      }
    }
    if (rc != LGE_OK) {
      release();
      return rc;
    }
    e = launch_col_fill(g->row_ptr, g->arh, n, coff, clist, s);
    if (e == hipSuccess)
      e = launch_rows_fill(g->row_ptr, g->col, coff, ccnt, clist, g->row_hubs, g->nrows, g->ncol, g->rows_stride,
                           g->rows_w, g->rows, n, toff, toff_len, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return hip_err(e);
  }
  LGE_HIP(hipStreamSynchronize(s));
  // rows and columns now live in the vertex records and arc words
  dev_free(g->hrow);
  dev_free(g->rcol);
  dev_free(g->row_hubs);
  g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_build).count();
  return LGE_OK;
}

// Co-degree table of the vertices of degree > tau, tau the smallest threshold
// >= kCodegMinDeg that leaves at most hc_max of them (hc_max from the table's
// memory budget).  Ranks go by increasing degree (ties by id): the split
// kernel counts each edge between two ranked members of T_e once, from its
// lower-rank end, over the bit-row words above that rank, and high-degree
// members, the common ones, then have few words above them.
static int build_codeg(lge_ctx *ctx, lge_graph *g, const int32_t *host_row_ptr, uint32_t flags) {
  const int64_t n = g->n;
  g->hc = 0;
  if (n <= 0) return LGE_OK;
  const double csr_bytes = 4.0 * ((double)n + 1.0 + 2.0 * (double)g->m);
  double budget = (flags & LGE_FLAG_COMPACT) ? kCodegBytesCompact : kCodegBytes;
  budget = std::min(budget, std::max(kCodegBytesCompact, kCodegPerCsr * csr_bytes));
  if (ctx->codeg_budget > 0) budget = std::min(budget, (double)ctx->codeg_budget);
  int64_t hc_max = std::min<int64_t>(kMaxRanked, (int64_t)std::sqrt(budget / (double)sizeof(uint16_t)));
  hc_max &= ~(int64_t)63;
  std::vector<int32_t> deg((size_t)n);
  for (int64_t u = 0; u < n; ++u) deg[u] = host_row_ptr[u + 1] - host_row_ptr[u];
  int32_t tau = kCodegMinDeg;
  if (hc_max < 2) return LGE_OK;
  if (n > hc_max) {
    std::vector<int32_t> tmpd(deg);
    std::nth_element(tmpd.begin(), tmpd.begin() + hc_max, tmpd.end(), std::greater<int32_t>());
    tau = std::max(tau, tmpd[hc_max]);
  }
  std::vector<int32_t> ranked;
  for (int64_t u = 0; u < n; ++u)
    if (deg[u] > tau) ranked.push_back((int32_t)u);
  const int64_t hc = (int64_t)ranked.size();
  g->codeg_tau = tau;
  if (hc < 2) return LGE_OK;
  std::stable_sort(ranked.begin(), ranked.end(), [&](int32_t x, int32_t y) { return deg[x] < deg[y]; });
  std::vector<int32_t> hrank((size_t)n, -1);
  for (int64_t r = 0; r < hc; ++r) hrank[ranked[r]] = (int32_t)r;
  // ranks grow with degree: a co-degree can reach 2^16 - 1 only between two
  // vertices of degree >= 65535, whose pairs are then never read
  int32_t sat = (int32_t)hc;
  while (sat > 0 && deg[ranked[sat - 1]] >= 65535) --sat;
  hipStream_t s = ctx->stream;
  int64_t *cnt = nullptr, *off = nullptr, *tmp = nullptr;
  int32_t *list = nullptr, *nlo = nullptr;
  auto cleanup = [&]() {
    dev_free(cnt);
    dev_free(off);
    dev_free(tmp);
    dev_free(list);
    dev_free(nlo);
  };
  int rc;
  if ((rc = dev_alloc(&cnt, n)) != LGE_OK || (rc = dev_alloc(&off, n)) != LGE_OK || (rc = dev_alloc(&nlo, n)) != LGE_OK ||
      (rc = dev_alloc(&tmp, scan_tmp_size(n))) != LGE_OK || (rc = dev_alloc(&g->crank, n)) != LGE_OK ||
      (rc = dev_alloc(&g->codeg, hc * hc)) != LGE_OK) {
    cleanup();
    return rc;
  }
  hipError_t e = hipMemcpyAsync(g->crank, hrank.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_codeg_count(g->row_ptr, g->col, g->crank, n, cnt, s);
  if (e == hipSuccess) e = launch_scan_i64(cnt, off, n, tmp, s);
  int64_t last[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(&last[0], off + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&last[1], cnt + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_err(e);
  }
  const int64_t total = last[0] + last[1];
  if ((rc = dev_alloc(&list, std::max<int64_t>(total, 1))) != LGE_OK) {
    cleanup();
    return rc;
  }
  const int64_t hcw = (hc + 63) / 64;
  if ((rc = dev_alloc(&g->hbits, hc * hcw)) != LGE_OK) {
    cleanup();
    return rc;
  }
  // the table row by row (every entry written): the ranked vertices in rank
  // order on the device
  int32_t *dranked = nullptr;
  if ((rc = dev_alloc(&dranked, hc)) != LGE_OK) {
    cleanup();
    return rc;
  }
  e = hipMemcpyAsync(dranked, ranked.data(), (size_t)hc * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_codeg_fill(g->row_ptr, g->col, g->crank, n, off, cnt, list, nlo, s);
  if (e == hipSuccess) e = launch_codeg_rows(g->row_ptr, g->col, dranked, off, cnt, list, nlo, hc, g->codeg, s);
  if (e == hipSuccess) e = launch_zero_u64(g->hbits, hc * hcw, s);
  if (e == hipSuccess) e = launch_codeg_bits(g->row_ptr, g->col, g->crank, n, hcw, g->hbits, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(dranked);
  cleanup();
  if (e != hipSuccess) return hip_err(e);
  g->hc = hc;
  g->hcw = hcw;
  g->codeg_sat = sat;
  return LGE_OK;
}

// Co-degree rows: for the chosen ranked hubs y, |Gamma(y) n Gamma(w)| for the
// unranked w of degree above a floor, each at w's column (its position among
// those vertices); ranked pairs use the co-degree table.  The floor is the
// smallest of 0, 1, 2, 4, ..., 64 at which the rows of every hub within the
// build-work budget fit the byte budget (isolated vertices never need a
// column; an S_a member of degree at or below it is walked instead).  An
// unranked degree is at most the ranking threshold, so one byte holds a count
// when that is <= kRowMaxDeg, two bytes otherwise.  Leaves g->hrow (row of
// every vertex) and g->rcol (column of every vertex) for the vertex records.
static int build_rows(lge_ctx *ctx, lge_graph *g, const int32_t *host_row_ptr, uint32_t flags) {
  g->nrows = 0;
  const int64_t n = g->n;
  if (n <= 0 || g->hc <= 0 || g->codeg_tau > 65535) return LGE_OK;
  const int width = g->codeg_tau <= kRowMaxDeg ? 1 : 2;
  std::vector<std::pair<int32_t, int32_t>> cand;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t d = host_row_ptr[v + 1] - host_row_ptr[v];
    if (d > kRowDeg) cand.push_back({d, (int32_t)v});
  }
  if (cand.empty()) return LGE_OK;
  std::sort(cand.begin(), cand.end(), [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
    return x.first != y.first ? x.first > y.first : x.second < y.second;
  });
  std::vector<int64_t> vol2((size_t)n);
  std::vector<int32_t> rank((size_t)n);
  hipStream_t s = ctx->stream;
  LGE_HIP(hipMemcpyAsync(vol2.data(), g->vol2, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LGE_HIP(hipMemcpyAsync(rank.data(), g->crank, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LGE_HIP(hipStreamSynchronize(s));
  const bool compact = (flags & LGE_FLAG_COMPACT) != 0;
  const double budget_ops = compact ? kRowBudgetOpsCompact : kRowBudgetOps;
  double budget_bytes = compact ? kRowBudgetBytesCompact : kRowBudgetBytes;
  const double csr_bytes = 4.0 * ((double)n + 1.0 + 2.0 * (double)g->m);
  budget_bytes = std::min(budget_bytes, std::max(kRowBudgetBytesCompact, kRowsPerCsr * csr_bytes));
  if (ctx->rows_budget > 0) budget_bytes = std::min(budget_bytes, (double)ctx->rows_budget);
  std::vector<int32_t> hubs;  // ranked hubs within the build-work budget, largest degree first
  double ops = 0.0;
  for (const auto &c : cand) {
    if (rank[c.second] < 0) continue;
    if (ops + (double)vol2[c.second] > budget_ops || (int64_t)hubs.size() >= kMaxRows) break;
    ops += (double)vol2[c.second];
    hubs.push_back(c.second);
  }
  if (hubs.empty()) return LGE_OK;
  // the column floor, and the columns
  static const int32_t kFloors[] = {0, 1, 2, 4, 8, 16, 32, 64};
  int32_t floor_deg = kFloors[7];
  int64_t ncol = 0;
  for (int32_t f : kFloors) {
    int64_t c = 0;
    for (int64_t v = 0; v < n; ++v) c += (rank[v] < 0 && host_row_ptr[v + 1] - host_row_ptr[v] > f) ? 1 : 0;
    floor_deg = f;
    ncol = c;
    const double bytes = (double)hubs.size() * (double)((c + 7) & ~(int64_t)7) * width;
    if (bytes <= budget_bytes) break;
  }
  const int64_t stride = (ncol + 7) & ~(int64_t)7;  // entries, rows on 8-byte boundaries
  if (stride == 0) return LGE_OK;
  const int64_t nh = std::min<int64_t>((int64_t)hubs.size(), (int64_t)(budget_bytes / ((double)stride * width)));
  if (nh <= 0) return LGE_OK;
  // columns go to the vertices in id order, so every sorted adjacency list
  // lists its columns in increasing order
  std::vector<int32_t> rcol((size_t)n, -1), hrow((size_t)n, -1);
  {
    int32_t c = 0;
    for (int64_t v = 0; v < n; ++v)
      if (rank[v] < 0 && host_row_ptr[v + 1] - host_row_ptr[v] > floor_deg) rcol[v] = c++;
  }
  for (int64_t h = 0; h < nh; ++h) hrow[hubs[h]] = (int32_t)h;
  int rc;
  const int64_t nent = nh * stride * width;  // bytes
  if ((rc = dev_alloc(&g->hrow, n)) != LGE_OK || (rc = dev_alloc(&g->rcol, n)) != LGE_OK ||
      (rc = dev_alloc(&g->row_hubs, nh)) != LGE_OK ||
      (rc = dev_alloc(&g->rows, nent)) != LGE_OK)
    return rc;  // graph_free releases the partial allocations
  hipError_t e = hipMemcpyAsync(g->row_hubs, hubs.data(), (size_t)nh * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->hrow, hrow.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->rcol, rcol.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors go out of scope
  if (e != hipSuccess) return hip_err(e);
  g->ncol = ncol;
  g->nrows = nh;
  g->rows_stride = stride;
  g->rows_w = width;
  g->rows_floor = floor_deg;
  return LGE_OK;
}

static void graph_free(lge_graph *g) {
  dev_free(g->own_row_ptr);
  dev_free(g->own_col);
  dev_free(g->edges);
  dev_free(g->vol2);
  dev_free(g->hoff);
  dev_free(g->htab);
  dev_free(g->crank);
  dev_free(g->codeg);
  dev_free(g->hbits);
  dev_free(g->hrow);
  dev_free(g->rcol);
  dev_free(g->row_hubs);
  dev_free(g->rows);
  dev_free(g->vinfo);
  dev_free(g->arh);
  dev_free(g->t_arc);
  dev_free(g->tri);
  dev_free(g->t_slot);
  dev_free(g->mred);
  dev_free(g->core);
  dev_free(g->wlevel[0]);
  dev_free(g->wlevel[1]);
}

static int32_t host_max_deg(int64_t n, const int32_t *row_ptr) {
  int32_t d = 0;
  for (int64_t u = 0; u < n; ++u) d = std::max(d, row_ptr[u + 1] - row_ptr[u]);
  return d;
}

// check_sizes: the graph's own exact sums must fit (sizes_in_range); a batch
// union skips it, since every member's sums use the member's own n and m and
// were checked one by one
static int create_host(lge_ctx *ctx, int64_t n, const int32_t *row_ptr, const int32_t *col, uint32_t flags,
                       bool check_sizes, lge_graph **out) {
  if (!ctx || !out || !row_ptr || n < 0) return LGE_EINVAL;
  *out = nullptr;
  if (n >= kMaxVertices) return LGE_ERANGE;
  if (row_ptr[0] != 0) return LGE_EGRAPH;
  for (int64_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return LGE_EGRAPH;
  const int64_t nnz = row_ptr[n];
  if (nnz % 2) return LGE_EGRAPH;
  if (nnz > 0 && !col) return LGE_EINVAL;
  const int32_t dmax = host_max_deg(n, row_ptr);
  if (check_sizes && !sizes_in_range(n, nnz / 2, dmax)) return LGE_ERANGE;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  lge_graph *g = new (std::nothrow) lge_graph();
  if (!g) return LGE_ENOMEM;
  g->ctx = ctx;
  g->n = n;
  g->m = nnz / 2;
  g->max_deg = dmax;
  int rc;
  if ((rc = dev_alloc(&g->own_row_ptr, n + 1)) != LGE_OK || (rc = dev_alloc(&g->own_col, std::max<int64_t>(nnz, 1))) != LGE_OK) {
    graph_free(g);
    delete g;
    return rc;
  }
  hipError_t e = hipMemcpyAsync(g->own_row_ptr, row_ptr, (size_t)(n + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess && nnz > 0)
    e = hipMemcpyAsync(g->own_col, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) {
    graph_free(g);
    delete g;
    return hip_err(e);
  }
  g->row_ptr = g->own_row_ptr;
  g->col = g->own_col;
  if ((rc = graph_preprocess(ctx, g, flags, row_ptr)) != LGE_OK) {
    graph_free(g);
    delete g;
    return rc;
  }
  *out = g;
  return LGE_OK;
}

extern "C" int lge_graph_create_host(lge_ctx *ctx, int64_t n, const int32_t *row_ptr, const int32_t *col,
                                     uint32_t flags, lge_graph **out) {
  return create_host(ctx, n, row_ptr, col, flags, true, out);
}

extern "C" int lge_graph_create_device(lge_ctx *ctx, int64_t n, const int32_t *d_row_ptr, const int32_t *d_col,
                                       void *hip_stream, uint32_t flags, lge_graph **out) {
  if (!ctx || !out || !d_row_ptr || n < 0) return LGE_EINVAL;
  *out = nullptr;
  if (n >= kMaxVertices) return LGE_ERANGE;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  if (hip_stream) LGE_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
  // row_ptr checks need it on the host once (n+1 ints)
  std::vector<int32_t> rp((size_t)n + 1);
  LGE_HIP(hipMemcpy(rp.data(), d_row_ptr, (size_t)(n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (rp[0] != 0) return LGE_EGRAPH;
  for (int64_t u = 0; u < n; ++u)
    if (rp[u + 1] < rp[u]) return LGE_EGRAPH;
  const int64_t nnz = rp[n];
  if (nnz % 2) return LGE_EGRAPH;
  if (nnz > 0 && !d_col) return LGE_EINVAL;
  const int32_t dmax = host_max_deg(n, rp.data());
  if (!sizes_in_range(n, nnz / 2, dmax)) return LGE_ERANGE;
  lge_graph *g = new (std::nothrow) lge_graph();
  if (!g) return LGE_ENOMEM;
  g->ctx = ctx;
  g->n = n;
  g->m = nnz / 2;
  g->max_deg = dmax;
  g->row_ptr = d_row_ptr;
  g->col = d_col;
  int rc;
  if ((rc = graph_preprocess(ctx, g, flags, rp.data())) != LGE_OK) {
    graph_free(g);
    delete g;
    return rc;
  }
  *out = g;
  return LGE_OK;
}

extern "C" int lge_graph_destroy(lge_graph *g) {
  if (!g) return LGE_EINVAL;
  if (g->ctx) {
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
  }
  graph_free(g);
  delete g;
  return LGE_OK;
}

extern "C" int64_t lge_graph_n(const lge_graph *g) { return g ? g->n : -1; }

extern "C" int lge_graph_query(const lge_graph *g, lge_graph_info *out) {
  if (!g || !out) return LGE_EINVAL;
  memset(out, 0, sizeof(*out));
  out->n = g->n;
  out->m = g->m;
  out->max_deg = g->max_deg;
  out->ranked = (int32_t)g->hc;
  out->rows = (int32_t)g->nrows;
  out->rows_floor = g->rows_floor;
  out->rows_width = g->rows_w;
  out->build_ms = g->build_ms;
  const int64_t n = g->n, m = g->m;
  int64_t b = 0;
  if (g->own_row_ptr) b += 4 * (n + 1);
  if (g->own_col) b += 8 * m;
  b += 8 * m + 8 * n + 8 * n + 4 * g->htab_len;  // edge list, 2-hop volumes, hub-table offsets, hub tables
  b += 16 * n + 8 * m;                           // vertex records, arc words
  if (g->hc > 0) b += 4 * n + 2 * g->hc * g->hc + 8 * g->hc * g->hcw;  // ranks, co-degree table, bit rows
  if (g->nrows > 0) b += g->nrows * g->rows_stride * g->rows_w;
  if (g->t_arc) b += 8 * m;
  if (g->tri) b += 8 * n;
  if (g->t_slot) b += 4 * g->htab_len;
  if (g->core) b += 4 * n;
  for (int k = 0; k < 2; ++k)
    if (g->wlevel[k]) b += m;
  out->state_bytes = (uint64_t)b;
  return LGE_OK;
}
extern "C" int64_t lge_graph_m(const lge_graph *g) { return g ? g->m : -1; }

// ---------------------------------------------------------------------------
// finalisation (exact integers -> FP64)
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// launch sequence for a set of slots and ranges
// ---------------------------------------------------------------------------



static Bins make_bins(Workspace &w) {
  Bins b;
  for (int c = 0; c < kNumClasses; ++c) {
    b.slot[c] = w.bin_slot[c];
    b.a[c] = w.bin_a[c];
    b.b[c] = w.bin_b[c];
  }
  b.count = w.counters + kCtrCount;
  b.cursor = w.counters + kCtrCursor;
  b.words = w.counters + kCtrWords;
  b.alg = w.counters + kCtrAlg;
  b.xcd_cursor = w.counters + kCtrXcd;
  b.lds_xcd = w.counters + kCtrLdsXcd;
  b.gtot = w.counters + kCtrItems;
  b.cap = w.cap_edges;
  b.cap_items = w.cap_items;
  b.cap_tlist = w.cap_tlist;
  return b;
}

// Runs sample -> bin -> count for every job; leaves per-job accumulators in
// ws.h_acc (host) on success.
int lge_job_slots(const Job &j) { return j.design == kDesignWeighted ? kWeightLevels : 1; }

// Accumulator replicas per slot for a sequence of nslots slots: few slots
// are shared by many workgroups, whose final atomics would otherwise queue on
// the same few cache lines.
static int acc_replicas(int nslots) {
  return std::min(kAccReplicas, std::max(1, kAccReplicaBudget / std::max(nslots, 1)));
}

// The launch sequence of `jobs` on workspace w, whose buffers hold the
// range length, the slots times acc_replicas(slots) accumulators, the
// ranges, and (when split-class edges are possible) some items and T_e
// entries.  Allocates nothing unless can_grow (then w is ctx->ws): when the
// split-class lists outgrow w's buffers it grows them and runs the class's
// tail again, otherwise it returns LGE_ERANGE.  On success the per-slot sums
// are packed at w.h_acc + k * kAccSlots * 2.
static int run_sequence(lge_ctx *ctx, Workspace &w, const Job *jobs, int njobs, const KernelCfg &cfg, bool can_grow,
                        int64_t budget) {
  int64_t total = 0;
  int nslots = 0;
  for (int j = 0; j < njobs; ++j) {
    total += jobs[j].e1 - jobs[j].e0;
    nslots += lge_job_slots(jobs[j]);
  }
  const int reps = acc_replicas(nslots);
  if (total > w.cap_edges || nslots * reps > w.cap_slots || njobs > w.cap_ranges) return LGE_EINTERNAL;
  int rc;
  hipStream_t s = ctx->stream;
  const int64_t rep_words = (int64_t)reps * kAccSlots * 2;
  int64_t pref = 0;
  int slot0 = 0;
  for (int j = 0; j < njobs; ++j) {
    const lge_graph *g = jobs[j].g;
    SlotDesc &sd = w.h_slots[slot0];
    sd.row_ptr = g->row_ptr;
    sd.col = g->col;
    sd.edges = g->edges ? g->edges + jobs[j].eid_base : nullptr;
    sd.vol2 = g->vol2;
    sd.hoff = g->hoff;
    sd.htab = g->htab;
    sd.crank = g->crank;
    sd.codeg = g->codeg;
    sd.hc = g->hc;
    sd.hbits = g->hbits;
    sd.hcw = g->hcw;
    sd.vinfo = g->vinfo;
    sd.arh = g->arh;
    sd.rows = g->rows;
    sd.rows_stride = g->rows_stride;
    sd.rows_w = g->rows_w;
    sd.n = jobs[j].n_override >= 0 ? jobs[j].n_override : g->n;
    sd.m = jobs[j].m_override >= 0 ? jobs[j].m_override : g->m;
    sd.p = jobs[j].p;
    sd.p_lo = jobs[j].p_lo;
    sd.seed = jobs[j].seed;
    sd.acc = w.acc + (int64_t)slot0 * rep_words;
    sd.acc_reps = reps;
    sd.codeg_sat = g->codeg_sat;
    sd.micro = jobs[j].micro;
    sd.micro_base = jobs[j].e0 - jobs[j].eid_base;
    sd.micro_len = jobs[j].e1 - jobs[j].e0;
    sd.design = jobs[j].design;
    sd.level = jobs[j].level;
    sd.kkey = jobs[j].kkey;
    sd.keid = jobs[j].keid;
    for (int l = 0; l < kWeightLevels; ++l) sd.plev[l] = jobs[j].plev ? jobs[j].plev[l] : 0.0;
    for (int l = 1; l < lge_job_slots(jobs[j]); ++l) {  // one accumulator slot per class
      w.h_slots[slot0 + l] = sd;
      w.h_slots[slot0 + l].acc = w.acc + (int64_t)(slot0 + l) * rep_words;
    }
    RangeDesc &rd = w.h_ranges[j];
    rd.slot = slot0;
    slot0 += lge_job_slots(jobs[j]);
    rd.pad = 0;
    rd.e0 = jobs[j].e0 - jobs[j].eid_base;
    rd.e1 = jobs[j].e1 - jobs[j].eid_base;
    rd.pref = pref;
    pref += jobs[j].e1 - jobs[j].e0;
  }
  ctx->timing = lge_timing();
  hipEvent_t *ev = ctx->ev;
  // Could any job have split-class edges?  (An endpoint above the workgroup
  // bound; otherwise the class stays empty and its kernels are not enqueued.)
  bool split = false;
  for (int j = 0; j < njobs; ++j) split = split || jobs[j].g->max_deg > cfg.block_max_deg;
  if (split && (w.cap_items == 0 || w.cap_tlist == 0)) return LGE_EINTERNAL;
  // Everything is enqueued at once: each kernel reads the sizes it needs
  // (class counts, split-class totals) from the device counters, and grids
  // are sized by `total`, which bounds every class count.
  // one copy of the descriptors (all range entries, then the used slots),
  // one kernel zeroing the counters and the used accumulators
  const size_t desc_bytes = (size_t)w.cap_ranges * sizeof(RangeDesc) + (size_t)nslots * sizeof(SlotDesc);
  const int64_t ctl_words = kNumCtrs + (int64_t)nslots * rep_words;
  if (njobs == 1 && nslots == 1) {  // the descriptors travel as kernel arguments
    LGE_HIP(launch_seq_init(w.ctl, ctl_words, w.ranges, w.slots, w.h_ranges[0], w.h_slots[0], s));
  } else {
    LGE_HIP(hipMemcpyAsync(w.desc, w.h_desc, desc_bytes, hipMemcpyHostToDevice, s));
    LGE_HIP(launch_zero_u64(w.ctl, ctl_words, s));
  }
  Bins bins = make_bins(w);
  LGE_HIP(hipEventRecord(ev[0], s));
  LGE_HIP(launch_sample_bin(w.slots, w.ranges, njobs, total, bins, cfg, s));
  LGE_HIP(hipEventRecord(ev[1], s));
  LGE_HIP(launch_count_wave(w.slots, bins, total, cfg, s));
  LGE_HIP(hipEventRecord(ev[3], s));
  LGE_HIP(launch_count_block(w.slots, bins, total, cfg, s));
  LGE_HIP(hipEventRecord(ev[4], s));
  // split class: ordering, per-edge work items and T_e capacities, their
  // scans (totals into the device counters), then the tail: item map,
  // classify, bit sets, counting, fold.  The tail kernels do nothing when the
  // totals exceed the item or T_e buffers; the host then grows them and runs
  // the tail again (the class's lists, items and offsets stay valid).
  auto split_tail = [&](Bins &bb) -> int {
    LGE_HIP(launch_item_fill(bb, w.item_pref, w.items, w.tbase, total, w.item_edge, w.gacc, s));
    LGE_HIP(launch_global_classify(w.slots, bb, w.item_pref, w.items, w.item_edge, w.tbase, w.tlist, w.tmask,
                                   w.gacc, cfg, s));
    LGE_HIP(launch_global_tbits(w.slots, bb, total, w.tbase, w.tlist, w.tbw, w.tbi, w.gacc, s));
    LGE_HIP(hipEventRecord(ev[6], s));
    LGE_HIP(launch_count_global(w.slots, bb, w.item_pref, w.items, w.item_edge, w.tlist, w.tbw, w.tbi, w.tmask,
                                w.gacc, cfg, s));
    LGE_HIP(hipEventRecord(ev[7], s));  // the counting kernel alone, for its roofline
    LGE_HIP(launch_global_finish(w.slots, bb, total, w.items, w.gacc, s));
    return LGE_OK;
  };
  if (split) {
    if (cfg.flags & kOptSortHub) {
      LGE_HIP(launch_sort_global(w.slots, bins, total, w.sort_slot, w.sort_a, w.sort_b, w.sort_hist, w.sort_off,
                                 w.sort_tmp, s));
      bins.slot[kClassGlobal] = w.sort_slot;
      bins.a[kClassGlobal] = w.sort_a;
      bins.b[kClassGlobal] = w.sort_b;
    }
    LGE_HIP(launch_global_prep(w.slots, bins, total, cfg.global_chunk, w.items, w.tcap, w.gacc, s));
    LGE_HIP(launch_global_scans(bins, w.items, w.item_pref, w.tcap, w.tbase, w.scan_tmp, s));
    if ((rc = split_tail(bins)) != LGE_OK) return rc;
  }
  LGE_HIP(hipEventRecord(ev[5], s));
  LGE_HIP(hipMemcpyAsync(w.h_ctl, w.ctl, (size_t)ctl_words * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  LGE_HIP(hipStreamSynchronize(s));  // the sequence's only wait, unless the split lists outgrew their buffers
  auto read_timing = [&](int64_t reruns) {
    lge_timing &t = ctx->timing;
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev[0], ev[5]) == hipSuccess) t.total_ms = ms;
    if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) t.sample_ms = ms;
    if (hipEventElapsedTime(&ms, ev[1], ev[3]) == hipSuccess) t.count_ms[0] = ms;
    if (hipEventElapsedTime(&ms, ev[3], ev[4]) == hipSuccess) t.count_ms[1] = ms;
    if (split) {  // without split-class edges the class's kernels are not enqueued
      if (hipEventElapsedTime(&ms, ev[6], ev[7]) == hipSuccess) t.count_ms[2] = ms;
      if (hipEventElapsedTime(&ms, ev[4], ev[6]) == hipSuccess) t.global_prep_ms = ms;
    }
    for (int c = 0; c < kNumClasses; ++c) t.class_edges[c] = w.h_counters[kCtrCount + c];
    for (int c = 0; c < kNumClasses; ++c) {
      t.words_read[c] = t.alg_bytes[c] = 0;
      for (int x = 0; x < kXcds; ++x) {
        t.words_read[c] += w.h_counters[kCtrWords + (kXcds * c + x) * kLine];
        t.alg_bytes[c] += w.h_counters[kCtrAlg + (kXcds * c + x) * kLine];
      }
    }
    t.launches = 5 + (split ? 16 + 6 * reruns : 0);
    t.host_waits = 1 + (uint32_t)reruns;
  };
  int64_t reruns = 0;
  if (split && !split_fits(bins, w.h_counters[kCtrItems], w.h_counters[kCtrTList])) {
    if (!can_grow) return LGE_ERANGE;
    // grow to the totals the scans found and run the tail again; the
    // accumulators hold the other classes' sums, the tail adds the split
    // class.  Lists beyond the budget (or beyond free memory) make the
    // caller run the range in pieces instead.
    const int64_t ni = (int64_t)w.h_counters[kCtrItems], nt = (int64_t)w.h_counters[kCtrTList];
    const int64_t need = list_bytes(ni, nt);
    if (need > budget) {
      read_timing(0);
      ctx->list_need = need;
      return kRunSplit;
    }
    rc = ws_reserve_items(ctx, ni);
    if (rc == LGE_OK) rc = ws_reserve_tlist(ctx, nt);
    if (rc == LGE_ENOMEM && budget < INT64_MAX) {
      read_timing(0);
      ctx->list_need = need;
      return kRunSplit;
    }
    if (rc != LGE_OK) return rc;
    bins.cap_items = w.cap_items;
    bins.cap_tlist = w.cap_tlist;
    if (!split_fits(bins, w.h_counters[kCtrItems], w.h_counters[kCtrTList])) return LGE_EINTERNAL;
    if ((rc = split_tail(bins)) != LGE_OK) return rc;
    LGE_HIP(hipEventRecord(ev[5], s));
    LGE_HIP(hipMemcpyAsync(w.h_ctl, w.ctl, (size_t)ctl_words * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s));
    LGE_HIP(hipStreamSynchronize(s));
    reruns = 1;
  }
  // add up each slot's replicas (exact 128-bit sums) and pack the slots:
  // slot k's sums end at h_acc + k * kAccSlots * 2, as the callers read them
  if (reps > 1) {
    for (int k = 0; k < nslots; ++k) {
      unsigned long long sum[kAccSlots * 2];
      const unsigned long long *src = w.h_acc + (int64_t)k * rep_words;
      for (int q = 0; q < kAccSlots; ++q) {
        u128 v = 0;
        for (int r = 0; r < reps; ++r) {
          const unsigned long long *x = src + (int64_t)r * kAccSlots * 2 + 2 * q;
          v += ((u128)x[1] << 64) | (u128)x[0];
        }
        sum[2 * q] = (unsigned long long)v;
        sum[2 * q + 1] = (unsigned long long)(v >> 64);
      }
      memcpy(w.h_acc + (int64_t)k * kAccSlots * 2, sum, sizeof(sum));
    }
  }
  read_timing(reruns);
  return LGE_OK;
}

// Adds the device times and launch counts of one sequence to *sum, and its
// class sizes and read counters when its sums were kept.
static void add_timing(lge_timing *sum, const lge_timing &t, bool kept) {
  sum->total_ms += t.total_ms;
  sum->sample_ms += t.sample_ms;
  sum->global_prep_ms += t.global_prep_ms;
  for (int c = 0; c < kNumClasses; ++c) {
    sum->count_ms[c] += t.count_ms[c];
    if (kept) {
      sum->class_edges[c] += t.class_edges[c];
      sum->words_read[c] += t.words_read[c];
      sum->alg_bytes[c] += t.alg_bytes[c];
    }
  }
  sum->launches += t.launches;
  sum->host_waits += t.host_waits;
}

// The jobs' per-slot sums into acc (kAccSlots * 2 words per slot, slots in
// job order).  One launch sequence when its split-class lists fit the
// budget; otherwise each job alone, and a lone job's edge-id range in
// consecutive pieces sized from the lists the failed sequence asked for.
// Sums over sampled edges are exact and additive over disjoint ranges.
static int run_pieces(lge_ctx *ctx, const Job *jobs, int njobs, const KernelCfg &cfg, unsigned long long *acc,
                      lge_timing *tsum, int depth) {
  int nslots = 0;
  bool split = false;
  for (int j = 0; j < njobs; ++j) {
    nslots += lge_job_slots(jobs[j]);
    split = split || jobs[j].g->max_deg > cfg.block_max_deg;
  }
  Workspace &w = ctx->ws;
  int rc;
  if (split && list_bytes(w.cap_items, w.cap_tlist) > cfg.list_budget + cfg.list_budget / 4) {
    // lists grown under a larger budget: give them back
    dev_free(w.item_edge);
    dev_free(w.tmask);
    dev_free(w.tlist);
    dev_free(w.tbw);
    dev_free(w.tbi);
    w.cap_items = w.cap_tlist = 0;
  }
  if (split && (w.cap_items == 0 || w.cap_tlist == 0)) {  // first use: a modest start, grown on demand
    const bool tight = cfg.list_budget < ((int64_t)64 << 20);
    if ((rc = ws_reserve_items(ctx, tight ? 1 : 1 << 14)) != LGE_OK) return rc;
    if ((rc = ws_reserve_tlist(ctx, tight ? 1 : 1 << 20)) != LGE_OK) return rc;
  }
  const bool single_edge = njobs == 1 && jobs[0].e1 - jobs[0].e0 <= 1;
  rc = run_sequence(ctx, w, jobs, njobs, cfg, true, single_edge ? INT64_MAX : cfg.list_budget);
  if (rc != LGE_OK && rc != kRunSplit) return rc;
  add_timing(tsum, ctx->timing, rc == LGE_OK);
  if (rc == LGE_OK) {
    memcpy(acc, w.h_acc, (size_t)nslots * kAccSlots * 2 * sizeof(unsigned long long));
    return LGE_OK;
  }
  if (depth > 48) return LGE_ENOMEM;
  if (njobs > 1) {
    for (int j = 0, s0 = 0; j < njobs; s0 += lge_job_slots(jobs[j]), ++j)
      if ((rc = run_pieces(ctx, jobs + j, 1, cfg, acc + (int64_t)s0 * kAccSlots * 2, tsum, depth + 1)) != LGE_OK)
        return rc;
    return LGE_OK;
  }
  const Job &J = jobs[0];
  const int64_t len = J.e1 - J.e0;
  const int64_t want = ctx->list_need / std::max<int64_t>(cfg.list_budget, 1) + 1;
  const int64_t k = std::min<int64_t>(std::max<int64_t>(want + want / 4 + 1, 2), std::min<int64_t>(len, 4096));
  std::vector<unsigned long long> part((size_t)nslots * kAccSlots * 2);
  memset(acc, 0, part.size() * sizeof(unsigned long long));
  for (int64_t i = 0; i < k; ++i) {
    Job sub = J;
    sub.e0 = J.e0 + len * i / k;
    sub.e1 = J.e0 + len * (i + 1) / k;
    if (sub.e1 == sub.e0) continue;
    if (J.micro) sub.micro = J.micro + (sub.e0 - J.e0) * kMicroCols;
    if ((rc = run_pieces(ctx, &sub, 1, cfg, part.data(), tsum, depth + 1)) != LGE_OK) return rc;
    for (size_t q = 0; q < part.size(); q += 2) {
      const u128 v = (((u128)acc[q + 1] << 64) | (u128)acc[q]) + (((u128)part[q + 1] << 64) | (u128)part[q]);
      acc[q] = (unsigned long long)v;
      acc[q + 1] = (unsigned long long)(v >> 64);
    }
  }
  return LGE_OK;
}

int lge_run_jobs(lge_ctx *ctx, const Job *jobs, int njobs, const lge_opts *opts) {
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  int64_t total = 0;
  int nslots = 0;
  for (int j = 0; j < njobs; ++j) {
    total += jobs[j].e1 - jobs[j].e0;
    nslots += lge_job_slots(jobs[j]);
  }
  int rc = ws_reserve(ctx, std::max<int64_t>(total, 1), nslots * acc_replicas(nslots), njobs);
  if (rc != LGE_OK) return rc;
  const KernelCfg cfg = make_cfg(ctx, opts);
  lge_timing tsum{};
  std::vector<unsigned long long> acc((size_t)nslots * kAccSlots * 2);
  rc = run_pieces(ctx, jobs, njobs, cfg, acc.data(), &tsum, 0);
  if (rc != LGE_OK) return rc;
  memcpy(ctx->ws.h_acc, acc.data(), acc.size() * sizeof(unsigned long long));
  ctx->timing = tsum;
  return LGE_OK;
}

static bool p_ok(double p) { return p > 0.0 && p <= 1.0; }

extern "C" int lge_estimate(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, const lge_opts *opts,
                            lge_result *out) {
  if (!p_ok(p)) return LGE_EINVAL;
  if (!ctx || !g || !out) return LGE_EINVAL;
  if (g->ctx != ctx) return LGE_EINVAL;
  Job job{g, p, seed, 0, g->m, -1, -1, 0};
  int rc = lge_run_jobs(ctx, &job, 1, opts);
  if (rc != LGE_OK) return rc;
  lge_finalize(g->n, g->m, p, seed, ctx->ws.h_acc, out);
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free estimate: the launch sequence of lge_estimate on a
// workspace carved out of the device's scratch array (fixed layout for at
// most kNoAllocEdges edge ids) with the context's pinned staging.
// ---------------------------------------------------------------------------

static bool scratch_view(lge_ctx *ctx, Workspace *v) {
  char *base = (char *)ctx->scratch;
  size_t cur = 0;
  auto take = [&](size_t bytes) -> void * {
    cur = (cur + 255) & ~(size_t)255;
    void *p = base + cur;
    cur += bytes;
    return p;
  };
  const int64_t cap = kNoAllocEdges;
  *v = Workspace();
  v->cap_edges = cap;
  for (int c = 0; c < kNumClasses; ++c) {
    v->bin_slot[c] = (int32_t *)take((size_t)cap * sizeof(int32_t));
    v->bin_a[c] = (int32_t *)take((size_t)cap * sizeof(int32_t));
    v->bin_b[c] = (int32_t *)take((size_t)cap * sizeof(int32_t));
  }
  v->items = (int64_t *)take((size_t)cap * sizeof(int64_t));
  v->item_pref = (int64_t *)take((size_t)cap * sizeof(int64_t));
  v->tcap = (int64_t *)take((size_t)cap * sizeof(int64_t));
  v->tbase = (int64_t *)take((size_t)cap * sizeof(int64_t));
  v->gacc = take((size_t)cap * gedge_bytes());
  v->scan_tmp_len = scan_tmp_size(cap);
  v->scan_tmp = (int64_t *)take((size_t)v->scan_tmp_len * sizeof(int64_t));
  v->sort_slot = (int32_t *)take((size_t)cap * sizeof(int32_t));
  v->sort_a = (int32_t *)take((size_t)cap * sizeof(int32_t));
  v->sort_b = (int32_t *)take((size_t)cap * sizeof(int32_t));
  v->cap_items = kNoAllocItems;
  v->item_edge = (int32_t *)take((size_t)kNoAllocItems * sizeof(int32_t));
  v->tmask = (unsigned long long *)take((size_t)kNoAllocItems * (kGlobalChunkMax / 64) * sizeof(unsigned long long));
  v->cap_tlist = kNoAllocTList;
  v->tlist = (int32_t *)take((size_t)3 * kNoAllocTList * sizeof(int32_t));
  v->tbw = (unsigned long long *)take((size_t)kNoAllocTList * sizeof(unsigned long long));
  v->tbi = (int16_t *)take((size_t)kNoAllocTList * sizeof(int16_t));
  v->cap_slots = kAccReplicas;  // one slot and its replicas
  v->cap_ranges = 1;
  v->ctl = (unsigned long long *)take((size_t)(kNumCtrs + (int64_t)kAccReplicas * kAccSlots * 2) *
                                      sizeof(unsigned long long));
  v->counters = v->ctl;
  v->acc = v->ctl + kNumCtrs;
  v->desc = take(sizeof(RangeDesc) + sizeof(SlotDesc));
  v->ranges = (RangeDesc *)v->desc;
  v->slots = (SlotDesc *)((char *)v->desc + sizeof(RangeDesc));
  // the sort histogram buffers and the pinned staging come from the context
  v->sort_hist = ctx->ws.sort_hist;
  v->sort_off = ctx->ws.sort_off;
  v->sort_tmp = ctx->ws.sort_tmp;
  v->h_desc = ctx->na_h_desc;
  v->h_ranges = (RangeDesc *)ctx->na_h_desc;
  v->h_slots = (SlotDesc *)((char *)ctx->na_h_desc + sizeof(RangeDesc));
  v->h_ctl = ctx->na_h_ctl;
  v->h_counters = ctx->na_h_ctl;
  v->h_acc = ctx->na_h_ctl + kNumCtrs;
  return cur <= kScratchBytes;
}

extern "C" int lge_estimate_noalloc(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, lge_result *out) {
  if (!p_ok(p)) return LGE_EINVAL;
  if (!ctx || !g || !out || g->ctx != ctx) return LGE_EINVAL;
  if (g->m > kNoAllocEdges) return LGE_ERANGE;
  if (!ctx->scratch || !ctx->na_h_desc || !ctx->na_h_ctl || !ctx->ws.sort_tmp) return LGE_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  Workspace v;
  if (!scratch_view(ctx, &v)) return LGE_EINTERNAL;  // the layout outgrew the array (a library bug)
  std::lock_guard<std::mutex> lk(scratch_lock(ctx->device));
  Job job{g, p, seed, 0, g->m, -1, -1, 0};
  const int rc = run_sequence(ctx, v, &job, 1, make_cfg(ctx, nullptr), false, INT64_MAX);
  if (rc != LGE_OK) return rc;
  lge_finalize(g->n, g->m, p, seed, v.h_acc, out);
  return LGE_OK;
}

extern "C" int lge_estimate_range(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, int64_t e0,
                                  int64_t e1, const lge_opts *opts, lge_result *out) {
  if (!p_ok(p)) return LGE_EINVAL;
  if (!ctx || !g || !out) return LGE_EINVAL;
  if (g->ctx != ctx || e0 < 0 || e1 < e0 || e1 > g->m) return LGE_EINVAL;
  Job job{g, p, seed, e0, e1, -1, -1, 0};
  int rc = lge_run_jobs(ctx, &job, 1, opts);
  if (rc != LGE_OK) return rc;
  lge_finalize(g->n, g->m, p, seed, ctx->ws.h_acc, out);
  return LGE_OK;
}

extern "C" int lge_estimate_async(lge_ctx *ctx, const lge_graph *g, double p, uint64_t seed, void *hip_stream,
                                  lge_result *out, lge_event **ev) {
  if (!p_ok(p)) return LGE_EINVAL;
  if (!ctx || !g || !out || !ev) return LGE_EINVAL;
  if (g->ctx != ctx) return LGE_EINVAL;
  *ev = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  // order after the work already queued on the caller's stream
  if (hip_stream) {
    hipEvent_t dep;
    LGE_HIP(hipEventCreateWithFlags(&dep, hipEventDisableTiming));
    hipError_t e = hipEventRecord(dep, (hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, dep, 0);
    (void)hipEventDestroy(dep);
    if (e != hipSuccess) return hip_err(e);
  }
  lge_event *E = new (std::nothrow) lge_event();
  if (!E) return LGE_ENOMEM;
  try {
    E->worker = std::thread([ctx, g, p, seed, out, E] {
      (void)hipSetDevice(ctx->device);
      Job job{g, p, seed, 0, g->m, -1, -1, 0};
      E->status = lge_run_jobs(ctx, &job, 1, nullptr);
      if (E->status == LGE_OK) lge_finalize(g->n, g->m, p, seed, ctx->ws.h_acc, out);
    });
  } catch (...) {
    delete E;
    return LGE_ENOMEM;
  }
  *ev = E;
  return LGE_OK;
}

extern "C" int lge_event_wait(lge_event *ev) {
  if (!ev) return LGE_EINVAL;
  if (ev->worker.joinable()) ev->worker.join();
  const int st = ev->status;
  delete ev;
  return st;
}

extern "C" int lge_last_timing(const lge_ctx *ctx, lge_timing *out) {
  if (!ctx || !out) return LGE_EINVAL;
  *out = ctx->timing;
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// batch: the graphs become one disjoint union (global vertex ids), each graph
// one slot over its own range of canonical edge ids
// ---------------------------------------------------------------------------

extern "C" int lge_count_batch(lge_ctx *ctx, const lge_batch *b, const lge_opts *opts, lge_result *outs) {
  if (!ctx || !b || !outs || b->count < 0) return LGE_EINVAL;
  if (b->count == 0) return LGE_OK;
  if (!b->vtx_off || !b->nnz_off || !b->row_ptr || !b->p || !b->seed) return LGE_EINVAL;
  const int G = b->count;
  for (int k = 0; k < G; ++k)
    if (!p_ok(b->p[k])) return LGE_EINVAL;
  const int64_t N = b->vtx_off[G];
  const int64_t NNZ = b->nnz_off[G];
  if (N < 0 || NNZ < 0 || (NNZ > 0 && !b->col)) return LGE_EINVAL;
  if (N >= kMaxVertices || NNZ > INT32_MAX) return LGE_ERANGE;
  // union CSR on the host
  std::vector<int32_t> rp((size_t)N + 1), cl((size_t)std::max<int64_t>(NNZ, 1));
  std::vector<int64_t> eoff((size_t)G + 1, 0);
  rp[0] = 0;
  for (int k = 0; k < G; ++k) {
    const int64_t v0 = b->vtx_off[k], v1 = b->vtx_off[k + 1];
    const int64_t z0 = b->nnz_off[k], z1 = b->nnz_off[k + 1];
    if (v1 < v0 || z1 < z0) return LGE_EINVAL;
    const int32_t *lrp = b->row_ptr + v0 + k;
    if (lrp[0] != 0 || lrp[v1 - v0] != z1 - z0) return LGE_EGRAPH;
    if (!(b->flags & LGE_FLAG_TRUSTED)) {
      int rc = lge_validate_csr_host(v1 - v0, lrp, b->col + z0);
      if (rc != LGE_OK) return rc;
    }
    for (int64_t u = 0; u < v1 - v0; ++u) rp[v0 + u + 1] = (int32_t)(z0 + lrp[u + 1]);
    for (int64_t j = z0; j < z1; ++j) cl[j] = (int32_t)(b->col[j] + v0);
    eoff[k + 1] = eoff[k] + (z1 - z0) / 2;
    if (!sizes_in_range(v1 - v0, (z1 - z0) / 2, host_max_deg(v1 - v0, lrp))) return LGE_ERANGE;
  }
  lge_graph *U = nullptr;
  int rc = create_host(ctx, N, rp.data(), cl.data(), LGE_FLAG_TRUSTED, false, &U);
  if (rc != LGE_OK) return rc;
  std::vector<Job> jobs((size_t)G);
  for (int k = 0; k < G; ++k) {
    const int64_t nk = b->vtx_off[k + 1] - b->vtx_off[k];
    jobs[k] = Job{U, b->p[k], b->seed[k], eoff[k], eoff[k + 1], nk, eoff[k + 1] - eoff[k], eoff[k]};
  }
  rc = lge_run_jobs(ctx, jobs.data(), G, opts);
  if (rc == LGE_OK) {
    for (int k = 0; k < G; ++k)
      lge_finalize(jobs[k].n_override, jobs[k].m_override, b->p[k], b->seed[k],
               ctx->ws.h_acc + (int64_t)k * kAccSlots * 2, &outs[k]);
  }
  lge_graph_destroy(U);
  return rc;
}

extern "C" int lge_estimate_many(lge_ctx *ctx, const lge_graph *const *graphs, const double *p,
                                 const uint64_t *seed, int32_t count, const lge_opts *opts, lge_result *outs) {
  if (!ctx || count < 0) return LGE_EINVAL;
  if (count == 0) return LGE_OK;
  if (!graphs || !p || !seed || !outs) return LGE_EINVAL;
  std::vector<Job> jobs((size_t)count);
  for (int32_t k = 0; k < count; ++k) {
    if (!p_ok(p[k]) || !graphs[k] || graphs[k]->ctx != ctx) return LGE_EINVAL;
    jobs[k] = Job{graphs[k], p[k], seed[k], 0, graphs[k]->m, -1, -1, 0};
  }
  int rc = lge_run_jobs(ctx, jobs.data(), count, opts);
  if (rc != LGE_OK) return rc;
  for (int32_t k = 0; k < count; ++k)
    lge_finalize(graphs[k]->n, graphs[k]->m, p[k], seed[k], ctx->ws.h_acc + (int64_t)k * kAccSlots * 2, &outs[k]);
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// Adaptive estimation (Sec. 4, Alg. 8).  Round t grows the sample by a
// fraction phi of the edges not yet sampled, p_t = p_{t-1} + phi (1 - p_{t-1}),
// then halves phi; because the sampler thresholds one uniform per edge, round
// t only counts the edges with p_{t-1} <= uniform < p_t and adds their exact
// sums, and its estimate is the plain Bernoulli(p_t) estimate.  The loop stops
// once the largest relative change of the 4-vertex estimates (G7..G17)
// between consecutive rounds is <= beta, or after t_max rounds.
// ---------------------------------------------------------------------------

extern "C" int lge_adaptive_cfg_default(lge_adaptive_cfg *c) {
  if (!c) return LGE_EINVAL;
  memset(c, 0, sizeof(*c));
  c->beta = 0.01;
  c->t_max = 20;
  c->phi0 = 0.0;
  return LGE_OK;
}

extern "C" int lge_estimate_adaptive(lge_ctx *ctx, const lge_graph *g, uint64_t seed, const lge_adaptive_cfg *cfg,
                                     lge_result *out, lge_adaptive_trace *trace) {
  if (!ctx || !g || !out) return LGE_EINVAL;
  if (g->ctx != ctx) return LGE_EINVAL;
  lge_adaptive_cfg c;
  lge_adaptive_cfg_default(&c);
  if (cfg) c = *cfg;
  if (!(c.beta >= 0.0) || c.t_max < 1 || c.t_max > LGE_ADAPTIVE_MAX_ROUNDS || !(c.phi0 >= 0.0) || c.phi0 > 1.0)
    return LGE_EINVAL;
  double phi = c.phi0 > 0.0 ? c.phi0 : (g->m > 0 ? 1.0 / sqrt((double)g->m) : 1.0);
  if (phi > 1.0) phi = 1.0;
  unsigned long long acc[kAccSlots * 2] = {};
  double p = 0.0;
  lge_result prev;
  bool have_prev = false;
  if (trace) memset(trace, 0, sizeof(*trace));
  for (int t = 0; t < c.t_max; ++t) {
    const double p_new = p + phi * (1.0 - p);
    Job job{g, p_new, seed, 0, g->m, -1, -1, 0};
    job.p_lo = p;
    const int rc = lge_run_jobs(ctx, &job, 1, nullptr);
    if (rc != LGE_OK) return rc;
    for (int k = 0; k < kAccSlots; ++k) {  // exact 128-bit accumulation
      const unsigned long long *src = ctx->ws.h_acc + 2 * k;
      const unsigned long long lo = acc[2 * k] + src[0];
      acc[2 * k + 1] += src[1] + (lo < acc[2 * k] ? 1ull : 0ull);
      acc[2 * k] = lo;
    }
    lge_finalize(g->n, g->m, p_new, seed, acc, out);
    double delta = -1.0;
    if (have_prev) {
      delta = 0.0;
      for (int i = 7; i <= 17; ++i) {
        const double x0 = prev.estimate[i], x1 = out->estimate[i];
        if (x0 != 0.0) delta = std::max(delta, fabs(x1 - x0) / fabs(x0));
        else if (x1 != 0.0) delta = std::max(delta, 1.0);
      }
    }
    if (trace) {
      trace->p[t] = p_new;
      trace->delta[t] = delta;
      trace->sampled[t] = out->sampled_edges;
      trace->rounds = t + 1;
    }
    prev = *out;
    have_prev = true;
    p = p_new;
    phi *= 0.5;
    if (delta >= 0.0 && delta <= c.beta) break;
  }
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// micro-level statistics
// ---------------------------------------------------------------------------

static int ensure_micro(lge_ctx *ctx, lge_graph *g) {
  if (g->mred) return LGE_OK;
  dev_free(g->t_arc);  // left over from a failed earlier attempt
  dev_free(g->tri);
  dev_free(g->t_slot);
  int rc;
  if ((rc = dev_alloc(&g->t_arc, std::max<int64_t>(2 * g->m, 1))) != LGE_OK) return rc;
  if ((rc = dev_alloc(&g->tri, std::max<int64_t>(g->n, 1))) != LGE_OK) return rc;
  if ((rc = dev_alloc(&g->t_slot, std::max<int64_t>(g->htab_len, 1))) != LGE_OK) return rc;
  hipStream_t s = ctx->stream;
  LGE_HIP(launch_micro_arc_tri(g->row_ptr, g->col, g->edges, g->hoff, g->htab, g->m, g->t_arc, s));
  LGE_HIP(launch_micro_vertex_tri(g->row_ptr, g->t_arc, g->n, g->tri, s));
  if (g->htab_len > 0)
    LGE_HIP(launch_micro_slot_tri(g->row_ptr, g->col, g->n, g->hoff, g->htab, g->t_arc, g->t_slot, s));
  LGE_HIP(hipStreamSynchronize(s));
  if ((rc = dev_alloc(&g->mred, 32)) != LGE_OK) return rc;  // last: marks the cache complete
  return LGE_OK;
}

extern "C" int lge_micro(lge_ctx *ctx, const lge_graph *gc, int64_t e0, int64_t e1, int64_t *out, int64_t *colmax) {
  if (!ctx || !gc) return LGE_EINVAL;
  if (gc->ctx != ctx || e0 < 0 || e1 < e0 || e1 > gc->m) return LGE_EINVAL;
  if (colmax)
    for (int i = 0; i < 18; ++i) colmax[i] = 0;
  if (e1 == e0) return LGE_OK;
  if (!out) return LGE_EINVAL;
  lge_graph *g = const_cast<lge_graph *>(gc);  // the cache is not part of the graph's value
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  int rc = ensure_micro(ctx, g);
  if (rc != LGE_OK) return rc;
  hipStream_t s = ctx->stream;
  long long *rows = reinterpret_cast<long long *>(out);
  LGE_HIP(launch_micro_mark(rows, e1 - e0, s));
  // t, k4 and cyc of every edge of the range from the counting kernels (p = 1)
  Job job{g, 1.0, 0, e0, e1, -1, -1, 0};
  job.micro = rows;
  if ((rc = lge_run_jobs(ctx, &job, 1, nullptr)) != LGE_OK) return rc;
  LGE_HIP(launch_zero_u64(g->mred, 32, s));
  int *err = reinterpret_cast<int *>(g->mred + 24);
  LGE_HIP(hipEventRecord(ctx->ev[6], s));
  LGE_HIP(launch_micro_rows(g->row_ptr, g->col, g->edges, g->vol2, g->hoff, g->htab, g->t_slot, g->vinfo, g->t_arc,
                            g->tri, g->n, g->m, e0, e1, rows, g->mred, err, ctx->num_cu * 8, s));
  LGE_HIP(hipEventRecord(ctx->ev[7], s));
  unsigned long long h[32];
  LGE_HIP(hipMemcpyAsync(h, g->mred, sizeof(h), hipMemcpyDeviceToHost, s));
  LGE_HIP(hipStreamSynchronize(s));
  int herr;
  memcpy(&herr, &h[24], sizeof(herr));
  if (herr != 0) return LGE_EINTERNAL;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]) == hipSuccess) ctx->timing.micro_ms = ms;
  ctx->timing.launches += 3;
  if (colmax)
    for (int i = 0; i < LGE_MICRO_COLS; ++i) colmax[i + 1] = (int64_t)h[i];
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// sampling designs: k-core weighted / degree weighted classes, fixed size
// ---------------------------------------------------------------------------

// k-core numbers by level-synchronous peeling; every level ends when no alive
// vertex has degree <= k, the next level starts at the smallest alive degree
static int ensure_core(lge_ctx *ctx, lge_graph *g) {
  if (g->max_core >= 0) return LGE_OK;
  const int64_t n = g->n;
  dev_free(g->core);
  int rc;
  if ((rc = dev_alloc(&g->core, std::max<int64_t>(n, 1))) != LGE_OK) return rc;
  if (n == 0) {
    g->max_core = 0;
    return LGE_OK;
  }
  int32_t *deg = nullptr, *state = nullptr, *fa = nullptr, *fb = nullptr;
  unsigned long long *cnt = nullptr;
  auto cleanup = [&] {
    dev_free(deg);
    dev_free(state);
    dev_free(fa);
    dev_free(fb);
    dev_free(cnt);
  };
  if ((rc = dev_alloc(&deg, n)) != LGE_OK || (rc = dev_alloc(&state, n)) != LGE_OK ||
      (rc = dev_alloc(&fa, n)) != LGE_OK || (rc = dev_alloc(&fb, n)) != LGE_OK || (rc = dev_alloc(&cnt, 4)) != LGE_OK) {
    cleanup();
    return rc;
  }
  hipStream_t s = ctx->stream;
  unsigned long long *h = ctx->ws.h_counters + kCtrHost;  // pinned staging (4 words)
  auto fail = [&](hipError_t e) {
    cleanup();
    return hip_err(e);
  };
  hipError_t e = launch_core_init(g->row_ptr, n, deg, state, s);
  if (e != hipSuccess) return fail(e);
  int64_t removed = 0;
  int32_t k = 0, kmax = 0;
  while (removed < n) {
    const unsigned long long init[2] = {0ull, ~0ull};
    if ((e = hipMemcpyAsync(cnt, init, sizeof(init), hipMemcpyHostToDevice, s)) != hipSuccess) return fail(e);
    if ((e = launch_core_scan(n, k, deg, state, fa, cnt, cnt + 1, s)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(h, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return fail(e);
    int64_t fn = (int64_t)h[0];
    if (fn == 0) {  // nothing left at this level: jump to the smallest alive degree
      if (h[1] == ~0ull) break;
      k = std::max<int32_t>(k + 1, (int32_t)h[1]);
      continue;
    }
    kmax = k;
    int32_t *front = fa, *next = fb;
    while (fn > 0) {
      if ((e = launch_zero_u64(cnt + 2, 1, s)) != hipSuccess) return fail(e);
      if ((e = launch_core_peel(g->row_ptr, g->col, front, fn, k, deg, state, g->core, next, cnt + 2, s)) !=
          hipSuccess)
        return fail(e);
      removed += fn;
      if ((e = hipMemcpyAsync(h + 2, cnt + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e);
      fn = (int64_t)h[2];
      std::swap(front, next);
    }
    ++k;
  }
  cleanup();
  if (removed != n) return LGE_EINTERNAL;
  g->max_core = kmax;
  return LGE_OK;
}

extern "C" int lge_core_numbers(lge_ctx *ctx, const lge_graph *gc, int32_t *core_out, int32_t *max_core) {
  if (!ctx || !gc || gc->ctx != ctx) return LGE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  lge_graph *g = const_cast<lge_graph *>(gc);  // the cache is not part of the graph's value
  const int rc = ensure_core(ctx, g);
  if (rc != LGE_OK) return rc;
  if (core_out && g->n > 0) {
    LGE_HIP(hipMemcpyAsync(core_out, g->core, (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    LGE_HIP(hipStreamSynchronize(ctx->stream));
  }
  if (max_core) *max_core = g->max_core;
  return LGE_OK;
}

static int ensure_levels(lge_ctx *ctx, lge_graph *g, int32_t mode) {
  uint8_t *&lv = g->wlevel[mode - 1];
  if (lv) return LGE_OK;
  int rc;
  if (mode == LGE_WEIGHT_KCORE && (rc = ensure_core(ctx, g)) != LGE_OK) return rc;
  uint8_t *buf = nullptr;
  unsigned long long *hist = nullptr;
  if ((rc = dev_alloc(&buf, std::max<int64_t>(g->m, 1))) != LGE_OK) return rc;
  if ((rc = dev_alloc(&hist, kWeightLevels)) != LGE_OK) {
    dev_free(buf);
    return rc;
  }
  hipStream_t s = ctx->stream;
  unsigned long long h[kWeightLevels];
  hipError_t e = launch_zero_u64(hist, kWeightLevels, s);
  if (e == hipSuccess) e = launch_weight_levels(mode, g->row_ptr, g->edges, g->core, g->m, buf, hist, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(hist);
  if (e != hipSuccess) {
    dev_free(buf);
    return hip_err(e);
  }
  for (int l = 0; l < kWeightLevels; ++l) g->whist[mode - 1][l] = h[l];
  lv = buf;
  return LGE_OK;
}

// Class probabilities p_l = min(1, c 2^l) with sum_l hist_l p_l = p_mean m:
// the classes from j up are saturated for the first j, counting down from
// kWeightLevels, whose c keeps every non-empty lower class below 1 and every
// non-empty saturated class at or above 1.
static bool plan_levels(const uint64_t *hist, double p_mean, int64_t m, double *pl) {
  if (p_mean >= 1.0) {
    for (int l = 0; l < kWeightLevels; ++l) pl[l] = 1.0;
    return true;
  }
  const double target = p_mean * (double)m;
  for (int j = kWeightLevels; j >= 1; --j) {
    uint64_t sat = 0, wsum = 0;
    for (int l = j; l < kWeightLevels; ++l) sat += hist[l];
    for (int l = 0; l < j; ++l) wsum += hist[l] << l;
    if (wsum == 0) continue;
    const double c = (target - (double)sat) / (double)wsum;
    if (c <= 0.0) continue;
    bool ok = true;
    for (int l = 0; l < kWeightLevels && ok; ++l) {
      if (!hist[l]) continue;
      const double q = c * ldexp(1.0, l);
      ok = l < j ? q < 1.0 : q >= 1.0;
    }
    if (!ok) continue;
    for (int l = 0; l < kWeightLevels; ++l) pl[l] = std::min(1.0, c * ldexp(1.0, l));
    return true;
  }
  return false;
}

extern "C" int lge_estimate_weighted(lge_ctx *ctx, const lge_graph *gc, int32_t mode, double p_mean, uint64_t seed,
                                     const lge_opts *opts, lge_result *out, lge_weight_info *info) {
  if (!ctx || !gc || !out || gc->ctx != ctx) return LGE_EINVAL;
  if (mode != LGE_WEIGHT_DEGREE && mode != LGE_WEIGHT_KCORE) return LGE_EINVAL;
  if (!(p_mean > 0.0 && p_mean <= 1.0)) return LGE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  lge_graph *g = const_cast<lge_graph *>(gc);
  int rc = ensure_levels(ctx, g, mode);
  if (rc != LGE_OK) return rc;
  const uint64_t *hist = g->whist[mode - 1];
  double pl[kWeightLevels];
  if (g->m == 0) {
    for (int l = 0; l < kWeightLevels; ++l) pl[l] = 1.0;
  } else if (!plan_levels(hist, p_mean, g->m, pl)) {
    return LGE_EINTERNAL;
  }
  Job job{g, p_mean, seed, 0, g->m, -1, -1, 0};
  job.design = kDesignWeighted;
  job.level = g->wlevel[mode - 1];
  job.plev = pl;
  if ((rc = lge_run_jobs(ctx, &job, 1, opts)) != LGE_OK) return rc;
  ExactSums lev[kWeightLevels], tot;
  memset(&tot, 0, sizeof(tot));
  bool full = true;
  for (int l = 0; l < kWeightLevels; ++l) {
    sums_from_acc(ctx->ws.h_acc + (int64_t)l * kAccSlots * 2, &lev[l]);
    sums_add(&tot, lev[l]);
    if (hist[l] && pl[l] != 1.0) full = false;
  }
  i128 K[18], E[18];
  fill_exact(g->n, g->m, p_mean, seed, tot, out, K, E);
  for (int i = 1; i <= 17; ++i) {
    if (i <= 2 || full) {
      set_xv(out, i, to_double(E[i]), 0.0);
      continue;
    }
    // Horvitz-Thompson over the classes, in class order
    double x = to_double(K[i]), v = 0.0;
    for (int l = 0; l < kWeightLevels; ++l) x += (to_double(lev[l].Z[i]) * (1.0 / pl[l])) / 12.0;
    for (int l = 0; l < kWeightLevels; ++l)
      v += (to_double((i128)lev[l].Q[i]) * ((1.0 - pl[l]) / (pl[l] * pl[l]))) / 144.0;
    set_xv(out, i, x, v);
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    for (int l = 0; l < kWeightLevels; ++l) {
      info->p_level[l] = pl[l];
      info->edges[l] = hist[l];
      info->sampled[l] = lev[l].count;
    }
    info->max_core = g->max_core;
  }
  return LGE_OK;
}


// K-th smallest composite key (Philox key << 64 | edge id) by 16 radix passes
static int select_kth(lge_ctx *ctx, int64_t m, uint64_t seed, uint64_t k, uint64_t *kkey, int64_t *keid) {
  hipStream_t s = ctx->stream;
  unsigned long long *hist = nullptr;
  int rc;
  if ((rc = dev_alloc(&hist, 256)) != LGE_OK) return rc;
  unsigned long long h[256];
  u128 chosen = 0;
  uint64_t r = k;  // 1-based rank among the keys matching the prefix
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 16 && e == hipSuccess; ++pass) {
    const int shift = 120 - 8 * pass, top = shift + 8;
    uint64_t pre_hi = 0, pre_lo = 0;
    if (top >= 128) {
    } else if (top >= 64) {
      pre_hi = (uint64_t)chosen;
    } else {
      const u128 full = chosen << top;
      pre_hi = (uint64_t)(full >> 64);
      pre_lo = (uint64_t)full >> top;
    }
    if ((e = launch_zero_u64(hist, 256, s)) != hipSuccess) break;
    if ((e = launch_select_hist(seed, m, shift, pre_hi, pre_lo, hist, s)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    int d = 0;
    while (d < 256 && h[d] < r) r -= h[d++];
    if (d == 256) {
      dev_free(hist);
      return LGE_EINTERNAL;
    }
    chosen = (chosen << 8) | (u128)d;
  }
  dev_free(hist);
  if (e != hipSuccess) return hip_err(e);
  *kkey = (uint64_t)(chosen >> 64);
  *keid = (int64_t)(uint64_t)chosen;
  return LGE_OK;
}

extern "C" int lge_estimate_fixed_k(lge_ctx *ctx, const lge_graph *g, uint64_t k, uint64_t seed,
                                    const lge_opts *opts, lge_result *out) {
  if (!ctx || !g || !out || g->ctx != ctx) return LGE_EINVAL;
  if (k < 1 || k > (uint64_t)g->m) return LGE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LGE_EDEVICE;
  const int64_t m = g->m;
  Job job{g, (double)k / (double)m, seed, 0, m, -1, -1, 0};
  job.design = kDesignFixedK;
  int rc = select_kth(ctx, m, seed, k, &job.kkey, &job.keid);
  if (rc != LGE_OK) return rc;
  if ((rc = lge_run_jobs(ctx, &job, 1, opts)) != LGE_OK) return rc;
  ExactSums t;
  sums_from_acc(ctx->ws.h_acc, &t);
  if (t.count != k) return LGE_EINTERNAL;
  i128 K[18], E[18];
  fill_exact(g->n, m, (double)k / (double)m, seed, t, out, K, E);
  const bool full = (int64_t)k == m;
  const double sigma = (double)m / (double)k;
  const double gfac = k >= 2 ? (double)m * (double)(m - (int64_t)k) / ((double)k * (double)k * (double)(k - 1)) : 0.0;
  for (int i = 1; i <= 17; ++i) {
    if (i <= 2 || full) {
      set_xv(out, i, to_double(E[i]), 0.0);
      continue;
    }
    const double x = to_double(K[i]) + (to_double(t.Z[i]) * sigma) / 12.0;
    double v = NAN;
    if (k >= 2) {
      // sample variance numerator K Q - Z^2 >= 0, exact in 256 bits
      const u128 az = t.Z[i] < 0 ? (u128)0 - (u128)t.Z[i] : (u128)t.Z[i];
      const U256 num = sub_u256(mul_u128((u128)k, t.Q[i]), mul_u128(az, az));
      v = (u256_to_double(num) * gfac) / 144.0;
    }
    set_xv(out, i, x, v);
  }
  return LGE_OK;
}

// ---------------------------------------------------------------------------
// autotuner: results never depend on the options, only the time does
// ---------------------------------------------------------------------------

static std::array<int32_t, 3> tune_class(const lge_graph *g, double p) {
  auto bits = [](uint64_t x) { int b = 0; for (; x; x >>= 1) ++b; return b; };
  return {bits((uint64_t)g->m), bits((uint64_t)std::max(g->max_deg, 0)), (int32_t)std::lround(4.0 * std::log2(p))};
}

extern "C" int lge_autotune(lge_ctx *ctx, const lge_graph *g, double p, lge_opts *out) {
  if (!p_ok(p)) return LGE_EINVAL;
  if (!ctx || !g || !out) return LGE_EINVAL;
  const auto key = tune_class(g, p);
  const auto hit = ctx->tuned.find(key);
  if (hit != ctx->tuned.end()) {
    *out = hit->second;
    return LGE_OK;
  }
  // coordinate descent over the class thresholds, the split-class work-item
  // size and layout flags, and the grid, starting from the defaults; each
  // candidate is timed on the device (sampling + counting), best of two
  // runs when one run is short
  lge_opts best;
  lge_opts_default(&best);
  lge_result r;
  int reps = 2;
  auto time_of = [&](const lge_opts &o, float *ms) -> int {
    float t_best = 1e30f;
    for (int rep = 0; rep < reps; ++rep) {
      const int rc = lge_estimate(ctx, g, p, 0x5eedull + (uint64_t)rep, &o, &r);
      if (rc != LGE_OK) return rc;
      const lge_timing &t = ctx->timing;
      t_best = std::min(t_best, t.sample_ms + t.count_ms[0] + t.count_ms[1] + t.global_prep_ms + t.count_ms[2]);
    }
    *ms = t_best;
    return LGE_OK;
  };
  float best_ms;
  int rc = time_of(best, &best_ms);
  if (rc != LGE_OK) return rc;
  if (best_ms > 50.0f) reps = 1;  // long runs vary by well under the gaps searched for
  auto knob = [&](int32_t lge_opts::*field, std::initializer_list<int32_t> vals) -> int {
    for (int32_t v : vals) {
      if (best.*field == v) continue;
      lge_opts o = best;
      o.*field = v;
      float ms;
      const int rc2 = time_of(o, &ms);
      if (rc2 != LGE_OK) return rc2;
      if (ms < best_ms) best_ms = ms, best = o;
    }
    return LGE_OK;
  };
  for (int pass = 0; pass < 2; ++pass) {
    const lge_opts start = best;
    if ((rc = knob(&lge_opts::wave_max_deg, {64, 128, 256, 512})) != LGE_OK) return rc;
    if ((rc = knob(&lge_opts::block_max_deg, {256, 512, 1024})) != LGE_OK) return rc;
    if ((rc = knob(&lge_opts::probe_ratio, {2, 4, 8})) != LGE_OK) return rc;
    if ((rc = knob(&lge_opts::global_chunk, {256, 512, 1024})) != LGE_OK) return rc;
    for (uint32_t f : {0u, LGE_OPT_SORT_HUB, LGE_OPT_XCD_LOCAL, LGE_OPT_SORT_HUB | LGE_OPT_XCD_LOCAL}) {
      if (best.flags == f) continue;
      lge_opts o = best;
      o.flags = f;
      float ms;
      if ((rc = time_of(o, &ms)) != LGE_OK) return rc;
      if (ms < best_ms) best_ms = ms, best = o;
    }
    if ((rc = knob(&lge_opts::grid_per_cu, {4, 8, 12})) != LGE_OK) return rc;
    if (memcmp(&start, &best, sizeof(best)) == 0) break;  // a pass changed nothing
  }
  ctx->tuned[key] = best;
  *out = best;
  return LGE_OK;
}

extern "C" int lge_autotune_reset(lge_ctx *ctx) {
  if (!ctx) return LGE_EINVAL;
  ctx->tuned.clear();
  return LGE_OK;
}

extern "C" int lge_set_table_budget(lge_ctx *ctx, uint64_t codeg_bytes, uint64_t rows_bytes) {
  if (!ctx) return LGE_EINVAL;
  ctx->codeg_budget = (int64_t)std::min<uint64_t>(codeg_bytes, (uint64_t)INT64_MAX);
  ctx->rows_budget = (int64_t)std::min<uint64_t>(rows_bytes, (uint64_t)INT64_MAX);
  return LGE_OK;
}

extern "C" int lge_set_build_scratch(lge_ctx *ctx, uint64_t bytes) {
  if (!ctx) return LGE_EINVAL;
  ctx->build_scratch = (int64_t)std::min<uint64_t>(bytes, (uint64_t)INT64_MAX);
  return LGE_OK;
}
