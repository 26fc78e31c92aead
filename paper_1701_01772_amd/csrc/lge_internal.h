// Internal interface between the host runtime (lge_host.cpp) and the device
// kernels (lge_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lge_layout.h"

namespace lge {

// Accumulator replicas per slot: kAccReplicas for a launch sequence of few
// slots, fewer as the slot count grows (kAccReplicaBudget replicas in all,
// at least one per slot).
constexpr int kAccReplicas = 32;
constexpr int kAccReplicaBudget = 2048;

// One estimate job as seen by the kernels.
struct SlotDesc {
  const int32_t *row_ptr;   // n+1
  const int32_t *col;       // 2m
  const uint64_t *edges;    // m canonical edges, (u << 32) | v with u < v
  const int64_t *vol2;      // n: sum of neighbour degrees
  const int64_t *hoff;      // n: offset of the vertex's hub table in htab (hubs only)
  const uint32_t *htab;     // hub tables (open addressing, 2^table_log(d) slots each)
  const int32_t *crank;     // n: rank in the co-degree table, -1 if absent
  const uint16_t *codeg;    // hc x hc, symmetric: |Gamma(x) n Gamma(y)| at [rank x][rank y], 16 bits
                            //     (pairs of two ranks >= codeg_sat are never read: they may not fit)
  int64_t hc;               // ranked vertices (0: no table)
  const unsigned long long *hbits;  // hc x hcw bit rows: bit ry of row rx = (x, y) adjacent
  int64_t hcw;              // 64-bit words per bit row, ceil(hc / 64) <= kBitsWords
  const int4 *vinfo;        // n: (row start, degree, rank or -1, co-degree row (ranked) or row column
                            //     (unranked), -1 if none)
  const uint32_t *arh;      // 2m, beside col: rank and row / column of the arc's head in 4 bytes,
                            //     ranked (rank + 1) | (row + 1) << 17, unranked 1 << 31 | (column + 1)
  const uint8_t *rows;      // rows x rows_stride entries of rows_w bytes: |Gamma(y) n Gamma(w)| at
                            // [row of ranked y][column of unranked w] (both from vinfo)
  int64_t rows_stride;
  int64_t n, m;
  double p;
  uint64_t seed;
  unsigned long long *acc;  // acc_reps replicas of kAccSlots x {lo, hi}; workgroup w adds into replica
                            // w % acc_reps (the host adds the replicas up), which spreads the atomics
                            // of many workgroups on one slot over several cache lines
  int32_t acc_reps;
  int32_t codeg_sat;        // first rank of degree >= 65535 (hc if none)
  double p_lo;              // sample edges with p_lo <= uniform < p (nested samples)
  // per-edge write-out (micro statistics; null otherwise): the counting
  // kernels store t, k4, cyc of edge id e in row e - micro_base of a
  // kMicroCols-wide int64 matrix, columns kMicroColT / K4 / Cyc
  long long *micro;
  int64_t micro_base, micro_len;
  // sampling design (kDesignBernoulli: p_lo <= uniform < p)
  int32_t design;
  int32_t rows_w;           // bytes per co-degree row entry: 1 when every unranked degree is
                            // <= kRowMaxDeg, else 2
  const uint8_t *level;     // kDesignWeighted: class of every edge id; class l is
                            //   kept iff uniform < plev[l] and binned to slot + l
  uint64_t kkey;            // kDesignFixedK: kept iff (Philox key, id) <= (kkey, keid)
  int64_t keid;
  double plev[16];
};

enum SampleDesign { kDesignBernoulli = 0, kDesignWeighted = 1, kDesignFixedK = 2 };
// weighted sampling: edge weights quantised to this many classes
constexpr int kWeightLevels = 16;

// micro statistics: one row of 17 int64 per edge, column i-1 = graphlet G_i
constexpr int kMicroCols = 17;
constexpr int kMicroColT = 2;    // G3 (triangles) = t
constexpr int kMicroColK4 = 6;   // G7 (4-cliques) = k4
constexpr int kMicroColCyc = 9;  // G10 (4-cycles) = cyc

// A contiguous range of canonical edge ids of one slot.
struct RangeDesc {
  int32_t slot;
  int32_t pad;
  int64_t e0, e1;  // [e0, e1)
  int64_t pref;    // exclusive prefix of range lengths over the range table
};

// Edge classes (who counts the edge).
enum EdgeClass { kClassWave = 0, kClassBlock = 1, kClassGlobal = 2, kNumClasses = 3 };

// Device counters of one launch sequence (unsigned long long each, zeroed
// at its start).  The kernels read every size they need from here, so the
// host enqueues the whole sequence without waiting for any of them.
// A device-scope atomic is carried out away from the XCD's L2, and the
// atomics of all XCDs on one 128-byte line queue behind each other.  So the
// counters and cursors that many workgroups touch come kXcds at a time
// (workgroup w uses copy w % kXcds), each copy on a line of its own (kLine
// words apart), and the host adds the copies up.
constexpr int kXcds = 8;
constexpr int kLine = 16;         // unsigned long long per 128-byte line
constexpr int kCtrCount = 0;      // sampled edges per class (kNumClasses)
constexpr int kCtrCursor = 3;     // work-queue cursors per class (split class without XCD-local order)
constexpr int kCtrItems = 6;      // split class: work items in all
constexpr int kCtrTList = 7;      // split class: T_e entries reserved in all
constexpr int kCtrHost = 8;       // 4 words of host-side staging (not written by the sequence)
constexpr int kCtrXcd = 16;       // XCD-local cursors of the split-class queue (kXcds lines)
constexpr int kCtrLdsXcd = kCtrXcd + kXcds * kLine;       // cursors of the wavefront and workgroup classes
constexpr int kCtrWords = kCtrLdsXcd + 2 * kXcds * kLine;  // 4-byte words read, per class and XCD
constexpr int kCtrAlg = kCtrWords + 3 * kXcds * kLine;     // neighbour-iteration bytes, per class and XCD
constexpr int kNumCtrs = kCtrAlg + 3 * kXcds * kLine;

// Binned work lists: structure of arrays, one per class, capacity `cap` each.
struct Bins {
  int32_t *slot[kNumClasses];
  int32_t *a[kNumClasses];  // side whose neighbours are iterated
  int32_t *b[kNumClasses];  // side held in the membership table
  unsigned long long *count;   // kNumClasses counters
  unsigned long long *cursor;  // kNumClasses work-queue cursors
  unsigned long long *words;   // kNumClasses x kXcds counters of 4-byte words read
  unsigned long long *alg;     // kNumClasses x kXcds counters of neighbour-iteration bytes of the sampled edges
  unsigned long long *xcd_cursor;  // kXcds cursors of the XCD-local split-class queue
  unsigned long long *lds_xcd;     // kXcds cursors per LDS class (wavefront, workgroup)
  unsigned long long *gtot;    // split class: [0] work items, [1] T_e entries (totals of the scans)
  int64_t cap;                 // entries of each class list
  int64_t cap_items;           // split class: work-item buffers (item -> edge map, T_e masks)
  int64_t cap_tlist;           // split class: T_e entry buffers
};

// The split class's work lists fit their buffers (the tail kernels of the
// class do nothing otherwise; the host grows the buffers and runs them again).
__host__ __device__ inline bool split_fits(const Bins &b, unsigned long long items, unsigned long long tl) {
  return (int64_t)items <= b.cap_items && (int64_t)tl <= b.cap_tlist;
}

struct KernelCfg {
  int32_t wave_max_deg;
  int32_t block_max_deg;
  int32_t probe_ratio;
  int32_t grid_wave, grid_block, grid_global;
  int32_t grid_sample;
  int32_t global_chunk;  // Gamma(a) positions per global-class work item
  uint32_t flags;        // LGE_OPT_* bits
  int64_t list_budget;   // bytes of split-class work lists one launch sequence may hold
};

// split-class edge ordering: key = rank of the table-side endpoint in the
// co-degree table, kSortKeys - 1 for unranked endpoints
constexpr int kSortKeys = kMaxRanked + 1;
constexpr uint32_t kOptSortHub = 1u;
constexpr uint32_t kOptXcdLocal = 2u;

// The allocation-free estimate keeps its whole workspace in one fixed device
// array per GPU (kScratchBytes, held until the process ends), laid out for a
// canonical edge-id range of at most kNoAllocEdges ids, at most
// kNoAllocItems split-class work items and kNoAllocTList T_e entries.
constexpr int64_t kNoAllocEdges = (int64_t)1 << 18;
constexpr int64_t kNoAllocItems = (int64_t)1 << 14;
constexpr int64_t kNoAllocTList = (int64_t)1 << 21;
constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;
// Device address of the array on `device` (which must be current), looked up
// once per device; scratch_lock(device) serialises its users in the process.
hipError_t scratch_address(int device, void **ptr);
std::mutex &scratch_lock(int device);

// ---- launchers (lge_kernels.hip) ----
hipError_t launch_graph_validate(const int32_t *row_ptr, const int32_t *col, int64_t n, int *err,
                                 hipStream_t s);
hipError_t launch_graph_upper(const int32_t *row_ptr, const int32_t *col, int64_t n, int32_t *up_start,
                              int64_t *cnt, hipStream_t s);
// exclusive scan; tmp must hold scan_tmp_size(len) entries
hipError_t launch_scan_i64(const int64_t *in, int64_t *out_excl, int64_t len, int64_t *tmp, hipStream_t s);
int64_t scan_tmp_size(int64_t len);
// exclusive scan of in[0, *len) with the length read on the device
// (*len <= cap); *total receives the sum; tmp holds ceil(cap / 1024) entries
hipError_t launch_scan_dev(const int64_t *in, int64_t *out_excl, const unsigned long long *len, int64_t cap,
                           int64_t *tmp, unsigned long long *total, hipStream_t s);
hipError_t launch_graph_edges(const int32_t *row_ptr, const int32_t *col, const int32_t *up_start,
                              const int64_t *eid_base, int64_t n, uint64_t *edges, hipStream_t s);
hipError_t launch_graph_vol2(const int32_t *row_ptr, const int32_t *col, int64_t n, int64_t *vol2,
                             hipStream_t s);
// per-block work estimate: blocks[k] = the cost of canonical edge ids
// [k kWorkBlock, (k + 1) kWorkBlock)
constexpr int64_t kWorkBlock = 4096;
hipError_t launch_graph_work(const int32_t *row_ptr, const uint64_t *edges, const int64_t *vol2, int64_t m,
                             unsigned long long *blocks, hipStream_t s);
hipError_t launch_hub_sizes(const int32_t *row_ptr, int64_t n, int64_t *size, hipStream_t s);
hipError_t launch_hub_build(const int32_t *row_ptr, const int32_t *col, int64_t n, const int64_t *hoff,
                            uint32_t *htab, hipStream_t s);
hipError_t launch_codeg_count(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n,
                              int64_t *cnt, hipStream_t s);
hipError_t launch_codeg_fill(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n,
                             const int64_t *off, const int64_t *cnt, int32_t *list, int32_t *nlo, hipStream_t s);
// per-vertex records (row start, degree, rank, row or column); crank, hrow,
// rcol may be null
hipError_t launch_vinfo(const int32_t *row_ptr, const int32_t *crank, const int32_t *hrow, const int32_t *rcol,
                        int64_t n, int4 *vinfo, hipStream_t s);
// packed rank words of every arc's head (after the vertex records)
hipError_t launch_arc_rank(const int32_t *col, const int4 *vinfo, int64_t nnz, uint32_t *arh, hipStream_t s);
// the neighbours of every vertex that have a column (arc word of an unranked
// head with a column), counted (cnt) and listed as columns at off (the
// exclusive scan of cnt), in adjacency order
hipError_t launch_col_count(const int32_t *row_ptr, const uint32_t *arh, int64_t n, int64_t *cnt, hipStream_t s);
hipError_t launch_col_fill(const int32_t *row_ptr, const uint32_t *arh, int64_t n, const int64_t *off, int32_t *clist,
                           hipStream_t s);
// co-degree rows of the vertices `hubs` at the ncol columns of the unranked
// vertices (coff / ccnt / clist: every vertex's column list), width bytes
// per entry, in tiles of rows_tile_entries(width) columns.  Every entry of
// the nh x stride rows is written (stride a multiple of 8).  toff: scratch
// of toff_len >= 2 n int32 for the segment ends of every column list at the
// tile bounds (the tiles go in passes of toff_len / n - 1).
int64_t rows_tile_entries(int width);
hipError_t launch_rows_fill(const int32_t *row_ptr, const int32_t *col, const int64_t *coff, const int64_t *ccnt,
                            const int32_t *clist, const int32_t *hubs, int64_t nh, int64_t ncol, int64_t stride,
                            int width, uint8_t *rows, int64_t n, int32_t *toff, int64_t toff_len, hipStream_t s);
// adjacency bit rows among the ranked vertices (bits zeroed by the caller)
hipError_t launch_codeg_bits(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n, int64_t hcw,
                             unsigned long long *bits, hipStream_t s);
// the whole hc x hc co-degree table, one row per ranked vertex (ranked[r] is
// the vertex of rank r; off / cnt / list: every vertex's ranked neighbours
// as ranks), every entry written (diagonal 0)
hipError_t launch_codeg_rows(const int32_t *row_ptr, const int32_t *col, const int32_t *ranked, const int64_t *off,
                             const int64_t *cnt, const int32_t *list, const int32_t *nlo, int64_t hc, uint16_t *tab,
                             hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int64_t len, hipStream_t s);
// clears p[0, len) and stores one range and one slot descriptor (passed by
// value) at rdst / sdst
hipError_t launch_seq_init(unsigned long long *p, int64_t len, RangeDesc *rdst, SlotDesc *sdst, const RangeDesc &r,
                           const SlotDesc &sd, hipStream_t s);
hipError_t launch_sample_bin(const SlotDesc *slots, const RangeDesc *ranges, int32_t nranges,
                             int64_t total, Bins bins, KernelCfg cfg, hipStream_t s);
// The counting launchers read each class's edge count from bins.count on the
// device; `bound` (>= that count, e.g. the length of the sampled ranges)
// only sizes the grids.
hipError_t launch_count_wave(const SlotDesc *slots, Bins bins, int64_t bound, KernelCfg cfg, hipStream_t s);
hipError_t launch_count_block(const SlotDesc *slots, Bins bins, int64_t bound, KernelCfg cfg, hipStream_t s);
// global class: per-edge work items and T_e capacities, T_e lists, counting
hipError_t launch_global_prep(const SlotDesc *slots, Bins bins, int64_t bound, int32_t chunk, int64_t *items,
                              int64_t *tcap, void *gacc, hipStream_t s);
// the per-edge first work items and T_e offsets (exclusive scans of items
// and tcap; totals into bins.gtot); tmp: scan scratch for bins.cap entries
hipError_t launch_global_scans(Bins bins, const int64_t *items, int64_t *item_pref, const int64_t *tcap,
                               int64_t *tbase, int64_t *tmp, hipStream_t s);
// work item -> edge map
hipError_t launch_item_fill(Bins bins, const int64_t *item_pref, const int64_t *items, const int64_t *tbase,
                            int64_t bound, int32_t *item_edge, void *gacc, hipStream_t s);
// T_e lists, and per work item the T_e membership of its positions of
// Gamma(a) (kGlobalChunkMax / 64 words per item)
hipError_t launch_global_classify(const SlotDesc *slots, Bins bins, const int64_t *item_pref,
                                  const int64_t *item_cnt, const int32_t *item_edge, const int64_t *tbase,
                                  int32_t *tlist, unsigned long long *tmask, void *gacc, KernelCfg cfg,
                                  hipStream_t s);
// counting sort of the split-class edges by key (see kSortKeys) into
// (slot2, a2, b2); hist, off: kSortKeys int64 each; tmp: scan scratch
hipError_t launch_sort_global(const SlotDesc *slots, Bins bins, int64_t bound, int32_t *slot2, int32_t *a2,
                              int32_t *b2, int64_t *hist, int64_t *off, int64_t *tmp, hipStream_t s);
// the compact ranked-member bit sets of every edge's T_e (non-zero words and
// their indices at the T_e offsets), then the counting
hipError_t launch_global_tbits(const SlotDesc *slots, Bins bins, int64_t bound, const int64_t *tbase,
                               const int32_t *tlist, unsigned long long *tbw, int16_t *tbi, void *gacc, hipStream_t s);
hipError_t launch_count_global(const SlotDesc *slots, Bins bins, const int64_t *item_pref,
                               const int64_t *item_cnt, const int32_t *item_edge, const int32_t *tlist, const unsigned long long *tbw, const int16_t *tbi,
                               const unsigned long long *tmask, void *gacc, KernelCfg cfg, hipStream_t s);
// folds the edges counted by several work items into their slots
hipError_t launch_global_finish(const SlotDesc *slots, Bins bins, int64_t bound, const int64_t *item_cnt,
                                const void *gacc, hipStream_t s);
size_t gedge_bytes();
// micro statistics: t of every arc (position j of col holds |Gamma(x) n
// Gamma(col[j])| for the row x owning j), vertex triangle counts, the
// per-edge sentinel fill, and the rows of edges [e0, e1)
// k-core peeling (one level k): scan pushes alive vertices of degree <= k
// (state 0 -> 2) and lowers *minalive to the smallest degree above k; peel
// assigns core = k to the frontier, decrements alive neighbours and pushes
// those that reach k, then retires the frontier (state 1)
hipError_t launch_core_init(const int32_t *row_ptr, int64_t n, int32_t *deg, int32_t *state, hipStream_t s);
hipError_t launch_core_scan(int64_t n, int32_t k, int32_t *deg, int32_t *state, int32_t *front,
                            unsigned long long *cnt, unsigned long long *minalive, hipStream_t s);
hipError_t launch_core_peel(const int32_t *row_ptr, const int32_t *col, const int32_t *front, int64_t fn, int32_t k,
                            int32_t *deg, int32_t *state, int32_t *core, int32_t *next, unsigned long long *ncnt,
                            hipStream_t s);
// weight classes of every edge (mode 1: d_u + d_v - 2, mode 2: min core) and
// their histogram (kWeightLevels counters, added to)
hipError_t launch_weight_levels(int32_t mode, const int32_t *row_ptr, const uint64_t *edges, const int32_t *core,
                                int64_t m, uint8_t *level, unsigned long long *hist, hipStream_t s);
// one radix-select pass over the composite keys (Philox key << 64 | id) of
// ids [0, m): histogram of the 8-bit digit at `shift` among the keys whose
// bits above `shift + 8` equal (pre_hi, pre_lo) there
hipError_t launch_select_hist(uint64_t seed, int64_t m, int32_t shift, uint64_t pre_hi, uint64_t pre_lo,
                              unsigned long long *hist, hipStream_t s);
hipError_t launch_micro_arc_tri(const int32_t *row_ptr, const int32_t *col, const uint64_t *edges,
                                const int64_t *hoff, const uint32_t *htab, int64_t m, int32_t *t_arc, hipStream_t s);
hipError_t launch_micro_vertex_tri(const int32_t *row_ptr, const int32_t *t_arc, int64_t n, int64_t *tri,
                                   hipStream_t s);
hipError_t launch_micro_mark(long long *out, int64_t rows, hipStream_t s);
// t_slot: t of every arc at its head's slot of the tail's hub table
// (k_micro_slot_tri), read for the tables hoff / htab
hipError_t launch_micro_slot_tri(const int32_t *row_ptr, const int32_t *col, int64_t n, const int64_t *hoff,
                                 const uint32_t *htab, const int32_t *t_arc, int32_t *t_slot, hipStream_t s);
hipError_t launch_micro_rows(const int32_t *row_ptr, const int32_t *col, const uint64_t *edges, const int64_t *vol2,
                             const int64_t *hoff, const uint32_t *htab, const int32_t *t_slot, const int4 *vinfo,
                             const int32_t *t_arc, const int64_t *tri, int64_t n, int64_t m, int64_t e0, int64_t e1,
                             long long *out, unsigned long long *colmax, int *err, int grid, hipStream_t s);

}  // namespace lge
