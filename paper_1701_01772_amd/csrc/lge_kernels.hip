// Device kernels of the edge-centric graphlet estimator for gfx950 (MI355X).
//
// Per sampled edge e = (a, b) the kernels compute the three quantities that
// need a neighbourhood search (Alg. 2-6 of "Estimation of Graphlet
// Statistics"):
//   t   = |T_e|, T_e = Gamma(a) n Gamma(b)                     (Alg. 2)
//   k4  = number of edges inside T_e                           (Alg. 3 / 5)
//   cyc = number of edges between S_a and S_b                  (Alg. 4 / 6)
// and fold them with the degrees into the unrestricted counts and the squared
// per-edge estimate numerators (closed forms of Sec. 2.3), accumulated as
// exact 128-bit integers per estimate slot.
//
// Membership tables: the side b is held in an open-addressing hash of vertex
// ids (bit 31 of a key tags "also in Gamma(a)", i.e. a member of T_e) —
// in LDS when d_b <= kHubDeg, else in the per-vertex global hub table built
// once per graph.  For every w in Gamma(a) \ {b} the kernel either scans
// Gamma(w) against the table (the neighbour iteration of Alg. 3/4) or, when
// Gamma(w) is much longer than the target set, looks each target up in
// Gamma(w) (the restricted searches of Alg. 5/6) by binary search or w's own
// hub table.  Both give the same integers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lge_internal.h"

namespace lge {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kTag = 0x80000000u;
constexpr uint32_t kProbe = 0x40000000u;
constexpr uint32_t kIdMask = 0x3FFFFFFFu;
constexpr int kWave = 64;

typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ceil_log2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// log2 of the slot count of a table holding `len` keys at load <= 1/2
__device__ __forceinline__ int table_log(int len) {
  int l = ceil_log2((uint32_t)(2 * (len > 0 ? len : 1)));
  return l < 6 ? 6 : l;
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t x, int logsz) {
  return (x * 2654435761u) >> (32 - logsz);
}

// Returns the slot holding x (key & kIdMask == x) or -1.  Works on LDS or
// global tables (generic pointer).
__device__ __forceinline__ int table_find(const uint32_t *tab, int logsz, uint32_t x) {
  const uint32_t mask = (1u << logsz) - 1u;
  uint32_t h = hash_slot(x, logsz);
  for (;;) {
    uint32_t k = tab[h];
    if (k == kEmpty) return -1;
    if ((k & kIdMask) == x) return (int)h;
    h = (h + 1u) & mask;
  }
}

__device__ __forceinline__ void lds_insert(uint32_t *tab, int logsz, uint32_t key) {
  const uint32_t mask = (1u << logsz) - 1u;
  uint32_t h = hash_slot(key & kIdMask, logsz);
  while (atomicCAS(&tab[h], kEmpty, key) != kEmpty) h = (h + 1u) & mask;
}

// binary search for x in the sorted list a[0, len); counts loads in *steps
__device__ __forceinline__ bool sorted_has(const int32_t *__restrict__ a, int len, int32_t x,
                                           uint32_t *steps) {
  int lo = 0, hi = len;
  uint32_t st = 0;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int32_t v = a[mid];
    ++st;
    if (v < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  bool found = false;
  if (lo < len) {
    found = a[lo] == x;
    ++st;
  }
  *steps += st;
  return found;
}

__device__ __forceinline__ void atomic_add_u128(unsigned long long *p, u128 v) {
  unsigned long long lo = (unsigned long long)v;
  unsigned long long hi = (unsigned long long)(v >> 64);
  if (lo) {
    unsigned long long old = atomicAdd(p, lo);
    if (old + lo < old) hi += 1ull;
  }
  if (hi) atomicAdd(p + 1, hi);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the Bernoulli edge test.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t philox_bits(uint64_t seed, uint64_t ctr) {
  uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = 0u, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return ((uint64_t)c1 << 32) | (uint64_t)c0;
}

__device__ __forceinline__ bool edge_taken(uint64_t seed, uint64_t eid, double p) {
  if (p >= 1.0) return true;  // the uniform is < 1 for every counter
  const uint64_t bits = philox_bits(seed, eid);
  return (double)(bits >> 11) * 0x1.0p-53 < p;
}

// ---------------------------------------------------------------------------
// Per-edge closed forms.  Term k of the slot accumulator for an edge with
// endpoint degrees da, db, |T| = t, k4 edges inside T, cyc edges between the
// two 2-star sets, in a graph of n vertices and m edges:
//   k = 0..12  C3, C4, C5, C7, C8, C9, C10, C11, C12, C13, C14, C15, C16
//   k = 13..27 (12 Y_i(e))^2 for i = 3..17
//   k = 28     1 (sampled edge count)
// ---------------------------------------------------------------------------

__device__ u128 edge_term(int k, int64_t n, int64_t m, int64_t da, int64_t db, int64_t t, int64_t k4,
                          int64_t cyc) {
  const int64_t sa = da - 1 - t, sb = db - 1 - t, s = sa + sb;
  const int64_t r = n - da - db + t;  // vertices adjacent to neither endpoint
  const int64_t f = m - da - db + 1;  // edges sharing no endpoint with e
  const int64_t c3 = t, c4 = s, c5 = r, c7 = k4, c8 = t * (t - 1) / 2, c9 = t * s, c10 = cyc;
  const int64_t c11 = sa * (sa - 1) / 2 + sb * (sb - 1) / 2, c12 = sa * sb, c13 = t * r, c14 = s * r;
  const int64_t c15 = f, c16 = r * (r - 1) / 2;
  if (k < 13) {
    int64_t c = 0;
    switch (k) {
      case 0: c = c3; break;
      case 1: c = c4; break;
      case 2: c = c5; break;
      case 3: c = c7; break;
      case 4: c = c8; break;
      case 5: c = c9; break;
      case 6: c = c10; break;
      case 7: c = c11; break;
      case 8: c = c12; break;
      case 9: c = c13; break;
      case 10: c = c14; break;
      case 11: c = c15; break;
      default: c = c16; break;
    }
    return (u128)(uint64_t)c;
  }
  if (k < 28) {
    // 12 * Y_i(e): the X equations with sigma = 1, constants dropped, times 12
    const int64_t z3 = 4 * c3, z4 = 6 * c4, z5 = 12 * c5, z6 = -(z3 + z4 + z5);
    const int64_t d87 = c8 - c7;
    const int64_t z7 = 2 * c7, z8 = 12 * d87, z9 = 6 * c9 - 24 * d87, z10 = 3 * c10;
    const int64_t z9_3 = 2 * c9 - 8 * d87;
    const int64_t z11 = 4 * c11 - z9_3, z12 = 12 * (c12 - c10), z13 = 4 * c13 - z9_3;
    const int64_t z14 = 6 * c14 - z12;
    const int64_t z15 = 6 * c15 - 3 * z7 - 2 * z8 - z9 - 2 * z10 - z12;
    const int64_t z16 = 12 * c16 - 2 * z15;
    const int64_t z17 = -(z7 + z8 + z9 + z10 + z11 + z12 + z13 + z14 + z15 + z16);
    int64_t z = 0;
    switch (k - 13) {
      case 0: z = z3; break;
      case 1: z = z4; break;
      case 2: z = z5; break;
      case 3: z = z6; break;
      case 4: z = z7; break;
      case 5: z = z8; break;
      case 6: z = z9; break;
      case 7: z = z10; break;
      case 8: z = z11; break;
      case 9: z = z12; break;
      case 10: z = z13; break;
      case 11: z = z14; break;
      case 12: z = z15; break;
      case 13: z = z16; break;
      default: z = z17; break;
    }
    const uint64_t az = (uint64_t)(z < 0 ? -z : z);
    return (u128)az * (u128)az;
  }
  if (k == kAccIdxCount) return 1;
  return 0;
}

// ---------------------------------------------------------------------------
// Graph preprocessing (once per resident graph)
// ---------------------------------------------------------------------------

// err bits: 1 bad row_ptr, 2 id out of range, 4 unsorted/duplicate,
//           8 self-loop, 16 asymmetric
__global__ __launch_bounds__(256) void k_graph_validate(const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, int64_t n,
                                                        int *err) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  int bad = 0;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    if (end < beg) {
      bad |= 1;
      continue;
    }
    for (int32_t j = beg + lane; j < end; j += kWave) {
      const int32_t v = col[j];
      if (v < 0 || v >= n) {
        bad |= 2;
        continue;
      }
      if (j > beg && col[j - 1] >= v) bad |= 4;
      if (v == u) bad |= 8;
      // symmetric: u must appear in Gamma(v)
      const int32_t vb = row_ptr[v], ve = row_ptr[v + 1];
      uint32_t st = 0;
      if (ve < vb || !sorted_has(col + vb, ve - vb, (int32_t)u, &st)) bad |= 16;
    }
  }
  if (bad) atomicOr(err, bad);
}

__global__ __launch_bounds__(256) void k_graph_upper(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, int64_t n,
                                                     int32_t *up_start, int64_t *cnt) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int lo = row_ptr[u], hi = row_ptr[u + 1];
    const int end = hi;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (col[mid] <= u)
        lo = mid + 1;
      else
        hi = mid;
    }
    up_start[u] = lo;
    cnt[u] = end - lo;
  }
}

__global__ __launch_bounds__(256) void k_graph_edges(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ up_start,
                                                     const int64_t *__restrict__ eid_base, int64_t n,
                                                     uint64_t *edges) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int32_t beg = up_start[u], end = row_ptr[u + 1];
    const int64_t base = eid_base[u];
    for (int32_t j = beg + lane; j < end; j += kWave)
      edges[base + (j - beg)] = ((uint64_t)(uint32_t)u << 32) | (uint64_t)(uint32_t)col[j];
  }
}

__global__ __launch_bounds__(256) void k_graph_vol2(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, int64_t n,
                                                    int64_t *vol2) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    unsigned long long s = 0;
    for (int32_t j = beg + lane; j < end; j += kWave) {
      const int32_t w = col[j];
      s += (unsigned long long)(row_ptr[w + 1] - row_ptr[w]);
    }
    s = wave_sum_u64(s);
    if (lane == 0) vol2[u] = (int64_t)s;
  }
}

// slot count (power of two) of each vertex's hub table; 0 for non-hubs
__global__ __launch_bounds__(256) void k_hub_sizes(const int32_t *__restrict__ row_ptr, int64_t n,
                                                   int64_t *size) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int d = row_ptr[u + 1] - row_ptr[u];
    size[u] = d > kHubDeg ? ((int64_t)1 << table_log(d)) : 0;
  }
}

__global__ __launch_bounds__(256) void k_hub_build(const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, int64_t n,
                                                   const int64_t *__restrict__ hoff, uint32_t *htab) {
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    const int d = end - beg;
    if (d <= kHubDeg) continue;  // uniform per block
    const int lg = table_log(d);
    uint32_t *tab = htab + hoff[u];
    for (int j = threadIdx.x; j < (1 << lg); j += blockDim.x) tab[j] = kEmpty;
    __syncthreads();
    const uint32_t mask = (1u << lg) - 1u;
    for (int32_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
      const uint32_t x = (uint32_t)col[j];
      uint32_t h = hash_slot(x, lg);
      while (atomicCAS(&tab[h], kEmpty, x) != kEmpty) h = (h + 1u) & mask;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (three-phase, 1024 elements per block)
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 1024;

__device__ int64_t block_exclusive_scan_256x4(int64_t v[4], int64_t *sh /* >= 256 */) {
  // v: 4 consecutive elements of this thread; returns the block total
  int64_t s = v[0] + v[1] + v[2] + v[3];
  const int tid = threadIdx.x;
  sh[tid] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t x = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  const int64_t incl = sh[tid];
  const int64_t total = sh[255];
  int64_t run = incl - s;
  for (int i = 0; i < 4; ++i) {
    const int64_t x = v[i];
    v[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(256) void k_scan_blocks(const int64_t *__restrict__ in, int64_t *out,
                                                     int64_t len, int64_t *block_sums) {
  __shared__ int64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int64_t v[4];
  for (int i = 0; i < 4; ++i) v[i] = base + i < len ? in[base + i] : 0;
  const int64_t total = block_exclusive_scan_256x4(v, sh);
  for (int i = 0; i < 4; ++i)
    if (base + i < len) out[base + i] = v[i];
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t *out, int64_t len,
                                                  const int64_t *__restrict__ offsets) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  const int64_t off = offsets[blockIdx.x];
  for (int i = 0; i < 4; ++i)
    if (base + i < len) out[base + i] += off;
}

// ---------------------------------------------------------------------------
// Sampling and binning (a pass over the canonical edge ids of every range)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_sample_bin(const SlotDesc *__restrict__ slots,
                                                    const RangeDesc *__restrict__ ranges, int32_t nranges,
                                                    int64_t total, Bins bins, KernelCfg cfg) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += stride) {
    const int64_t i = base + threadIdx.x;
    int cls = -1;
    int32_t slot = 0, a = 0, b = 0;
    if (i < total) {
      int lo = 0, hi = nranges - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ranges[mid].pref <= i)
          lo = mid;
        else
          hi = mid - 1;
      }
      const RangeDesc R = ranges[lo];
      slot = R.slot;
      const SlotDesc &S = slots[slot];
      const int64_t eid = R.e0 + (i - R.pref);
      if (edge_taken(S.seed, (uint64_t)eid, S.p)) {
        const uint64_t e = S.edges[eid];
        const int32_t u = (int32_t)(e >> 32), v = (int32_t)(uint32_t)e;
        const int32_t du = S.row_ptr[u + 1] - S.row_ptr[u];
        const int32_t dv = S.row_ptr[v + 1] - S.row_ptr[v];
        const int64_t wu = S.vol2[u], wv = S.vol2[v];
        // iterate the side whose neighbours have the smaller total degree
        const bool ua = wu < wv || (wu == wv && (du < dv || (du == dv && u < v)));
        a = ua ? u : v;
        b = ua ? v : u;
        const int32_t dmax = du > dv ? du : dv;
        cls = dmax <= cfg.wave_max_deg ? kClassWave : (dmax <= kHubDeg ? kClassBlock : kClassGlobal);
      }
    }
    for (int c = 0; c < kNumClasses; ++c) {
      const uint64_t msk = __ballot(cls == c);
      if (msk == 0ull) continue;
      const int leader = __ffsll((unsigned long long)msk) - 1;
      unsigned long long pos0 = 0;
      if (lane == leader) pos0 = atomicAdd(&bins.count[c], (unsigned long long)__popcll(msk));
      pos0 = __shfl(pos0, leader);
      if (cls == c) {
        const int64_t pos = (int64_t)pos0 + __popcll(msk & lt_mask);
        bins.slot[c][pos] = slot;
        bins.a[c][pos] = a;
        bins.b[c][pos] = b;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Block-level helpers for the counting kernels
// ---------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *red) {
  v = wave_sum_u64(v);
  if constexpr (NT == kWave) {
    return v;
  } else {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    unsigned long long s = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) s += red[i];
    __syncthreads();
    return s;
  }
}

// exclusive scan of x[0, len) in LDS by NT threads; returns the total
template <int NT>
__device__ int32_t block_scan_lds(int32_t *x, int len, int32_t *carry_sh) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int32_t carry = 0;
  for (int base = 0; base < len; base += NT) {
    const int i = base + (int)threadIdx.x;
    int32_t v = i < len ? x[i] : 0;
    // inclusive wave scan
    int32_t s = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int32_t y = __shfl_up(s, off);
      if (lane >= off) s += y;
    }
    int32_t wave_off = 0, chunk_total = 0;
    if constexpr (NT == kWave) {
      chunk_total = __shfl(s, kWave - 1);
    } else {
      __syncthreads();
      if (lane == kWave - 1) carry_sh[w] = s;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NT / kWave; ++k) {
        const int32_t t = carry_sh[k];
        if (k < w) wave_off += t;
        chunk_total += t;
      }
    }
    if (i < len) x[i] = carry + wave_off + s - v;
    carry += chunk_total;
    if constexpr (NT != kWave) __syncthreads();
  }
  return carry;
}

// Accumulates one edge's terms into the 32-lane register accumulator of wave 0
// of the block; flushes to the slot when the slot changes.
struct SlotAcc {
  u128 acc;
  int32_t slot;
  __device__ void init() {
    acc = 0;
    slot = -1;
  }
  __device__ void flush(const SlotDesc *__restrict__ slots) {
    const int lane = threadIdx.x & 63;
    if (slot >= 0 && lane < kAccSlots && acc != 0) atomic_add_u128(slots[slot].acc + 2 * lane, acc);
    acc = 0;
  }
  __device__ void add(const SlotDesc *__restrict__ slots, int32_t s, int64_t n, int64_t m, int64_t da,
                      int64_t db, int64_t t, int64_t k4, int64_t cyc) {
    const int lane = threadIdx.x & 63;
    if (s != slot) {
      flush(slots);
      slot = s;
    }
    if (lane <= kAccIdxCount) acc += edge_term(lane, n, m, da, db, t, k4, cyc);
  }
};

// ---------------------------------------------------------------------------
// LDS counting kernel: one edge per workgroup of NT threads, both endpoint
// degrees <= CAP.  LDS: hash of Gamma(b)\{a} (tag = member of T_e), the list
// of w in Gamma(a)\{b} with per-w unit prefix, and the target list
// (T_e at the front, S_b at the back) for restricted searches.
// ---------------------------------------------------------------------------

template <int NT, int CAP>
__global__ __launch_bounds__(NT) void k_count_lds(const SlotDesc *__restrict__ slots,
                                                  const int32_t *__restrict__ bslot,
                                                  const int32_t *__restrict__ ba,
                                                  const int32_t *__restrict__ bb, int64_t nedges,
                                                  unsigned long long *cursor, unsigned long long *words_out,
                                                  int32_t probe_ratio, int32_t chunk) {
  constexpr int HS = 2 * CAP;  // max hash slots
  __shared__ uint32_t htab[HS];
  __shared__ uint32_t wl_v[CAP];
  __shared__ int32_t wl_beg[CAP];
  __shared__ int32_t wl_deg[CAP];
  __shared__ int32_t wl_pref[CAP + 1];
  __shared__ int32_t tgt[CAP];
  __shared__ int32_t sh_cnt[4];
  __shared__ int32_t carry_sh[NT / kWave + 1];
  __shared__ unsigned long long red[NT / kWave];
  __shared__ unsigned long long sh_e;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  SlotAcc acc;
  acc.init();
  unsigned long long words = 0;

  for (;;) {
    if (tid == 0) sh_e = atomicAdd(cursor, (unsigned long long)chunk);
    __syncthreads();
    const int64_t e0 = (int64_t)sh_e;
    __syncthreads();
    if (e0 >= nedges) break;
    const int64_t e1 = e0 + chunk < nedges ? e0 + chunk : nedges;
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t slot = bslot[e];
      const int32_t a = ba[e], b = bb[e];
      const SlotDesc &S = slots[slot];
      const int32_t *__restrict__ rp = S.row_ptr;
      const int32_t *__restrict__ col = S.col;
      const int32_t abeg = rp[a], aend = rp[a + 1], bbeg = rp[b], bend = rp[b + 1];
      const int da = aend - abeg, db = bend - bbeg;
      const int lg = table_log(db);
      const int hs = 1 << lg;
      for (int i = tid; i < hs; i += NT) htab[i] = kEmpty;
      if (tid < 4) sh_cnt[tid] = 0;
      __syncthreads();
      // Gamma(b) \ {a} into the hash
      for (int i = tid; i < db; i += NT) {
        const int32_t x = col[bbeg + i];
        if (x != a) lds_insert(htab, lg, (uint32_t)x);
      }
      words += (unsigned long long)(db + 4);
      __syncthreads();
      // classify Gamma(a) \ {b}: in the hash -> T_e (tag it), else S_a
      for (int base = 0; base < da; base += NT) {
        const int i = base + tid;
        bool valid = i < da;
        int32_t x = valid ? col[abeg + i] : -1;
        valid = valid && x != b;
        bool isT = false;
        if (valid) {
          const int sl = table_find(htab, lg, (uint32_t)x);
          if (sl >= 0) {
            isT = true;
            htab[sl] = (uint32_t)x | kTag;
          }
        }
        const uint64_t vm = __ballot(valid);
        const int wcount = __popcll(vm);
        int pos0 = 0;
        if (lane == 0 && wcount) pos0 = atomicAdd(&sh_cnt[0], wcount);
        pos0 = __shfl(pos0, 0);
        if (valid) {
          const int pos = pos0 + __popcll(vm & lt_mask);
          const int32_t wb = rp[x], we = rp[x + 1];
          wl_v[pos] = (uint32_t)x | (isT ? kTag : 0u);
          wl_beg[pos] = wb;
          wl_deg[pos] = we - wb;
        }
      }
      words += (unsigned long long)da + 2ull * (unsigned long long)(da > 0 ? da - 1 : 0);
      __syncthreads();
      // target lists from the hash: T_e at the front, S_b at the back
      for (int i = tid; i < hs; i += NT) {
        const uint32_t k = htab[i];
        if (k == kEmpty) continue;
        if (k & kTag)
          tgt[atomicAdd(&sh_cnt[1], 1)] = (int32_t)(k & kIdMask);
        else
          tgt[CAP - 1 - atomicAdd(&sh_cnt[2], 1)] = (int32_t)(k & kIdMask);
      }
      __syncthreads();
      const int L = sh_cnt[0];
      const int t = sh_cnt[1];
      const int sbn = sh_cnt[2];
      // per-w strategy and unit counts
      for (int i = tid; i < L; i += NT) {
        const uint32_t v = wl_v[i];
        const int dw = wl_deg[i];
        const int tl = (v & kTag) ? t : sbn;
        int units = dw;
        if (probe_ratio > 0) {
          const int cost = dw > kHubDeg ? 3 : ceil_log2((uint32_t)dw + 1u) + 1;
          const long long pc = (long long)tl * (long long)cost * probe_ratio;
          if (pc < dw) {
            units = tl;
            wl_v[i] = v | kProbe;
          }
        }
        wl_pref[i] = units;
      }
      __syncthreads();
      const int32_t total = block_scan_lds<NT>(wl_pref, L, carry_sh);
      if (tid == 0) wl_pref[L] = total;
      __syncthreads();
      // flattened (w, unit) loop
      unsigned long long k4 = 0, cyc = 0;
      int cur = 0;
      uint32_t steps = 0;
      for (int base = 0; base < total; base += NT) {
        const int idx = base + tid;
        if (idx < total) {
          // largest i with wl_pref[i] <= idx, searching upward from cur
          int lo = cur, hi = L - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (wl_pref[mid] <= idx)
              lo = mid;
            else
              hi = mid - 1;
          }
          cur = lo;
          const uint32_t v = wl_v[lo];
          const int off = idx - wl_pref[lo];
          const bool isT = (v & kTag) != 0;
          if (v & kProbe) {
            const int32_t x = isT ? tgt[off] : tgt[CAP - sbn + off];
            const int32_t w = (int32_t)(v & kIdMask);
            const int dw = wl_deg[lo];
            bool found;
            if (dw > kHubDeg) {
              found = table_find(S.htab + S.hoff[w], table_log(dw), (uint32_t)x) >= 0;
              steps += 2;
            } else {
              found = sorted_has(col + wl_beg[lo], dw, x, &steps);
            }
            if (found) {
              if (isT)
                ++k4;
              else
                ++cyc;
            }
          } else {
            const int32_t r = col[wl_beg[lo] + off];
            ++steps;
            const int sl = table_find(htab, lg, (uint32_t)r);
            if (sl >= 0) {
              const bool rT = (htab[sl] & kTag) != 0;
              if (isT && rT) ++k4;
              if (!isT && !rT) ++cyc;
            }
          }
        }
      }
      words += steps;
      k4 = block_sum_u64<NT>(k4, red);
      cyc = block_sum_u64<NT>(cyc, red);
      if (tid < kWave) acc.add(slots, slot, S.n, S.m, da, db, t, (int64_t)(k4 / 2), (int64_t)cyc);
      __syncthreads();
    }
  }
  if (tid < kWave) acc.flush(slots);
  const unsigned long long wsum = block_sum_u64<NT>(words, red);
  if (tid == 0 && wsum) atomicAdd(words_out, wsum);
}

// ---------------------------------------------------------------------------
// Global-class counting: edges with an endpoint of degree > kHubDeg.
// Work item = (edge, chunk of kGlobalChunk positions of Gamma(a)).  Hub
// endpoints use their global hub table; a non-hub endpoint is hashed into
// LDS per item.  Per-edge partial sums meet in gacc; the item that completes
// an edge folds it into the slot.
// ---------------------------------------------------------------------------

constexpr int kGlobalNT = 256;

struct GEdge {
  unsigned long long t, k4, cyc, done;
};

__global__ __launch_bounds__(256) void k_global_prep(const SlotDesc *__restrict__ slots,
                                                     const int32_t *__restrict__ bslot,
                                                     const int32_t *__restrict__ ba, int64_t nedges,
                                                     int32_t chunk, int64_t *items, GEdge *gacc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges;
       e += (int64_t)gridDim.x * blockDim.x) {
    const SlotDesc &S = slots[bslot[e]];
    const int32_t a = ba[e];
    const int da = S.row_ptr[a + 1] - S.row_ptr[a];
    items[e] = (da + chunk - 1) / chunk;
    gacc[e].t = gacc[e].k4 = gacc[e].cyc = gacc[e].done = 0ull;
  }
}

__device__ __forceinline__ bool side_has(bool hub, const uint32_t *lds_tab, int lds_lg, const uint32_t *htab,
                                         int64_t off, int hlg, uint32_t x) {
  if (hub) return table_find(htab + off, hlg, x) >= 0;
  return table_find(lds_tab, lds_lg, x) >= 0;
}

__global__ __launch_bounds__(kGlobalNT) void k_count_global(
    const SlotDesc *__restrict__ slots, const int32_t *__restrict__ bslot, const int32_t *__restrict__ ba,
    const int32_t *__restrict__ bb, int64_t nedges, const int64_t *__restrict__ item_pref,
    const int64_t *__restrict__ item_cnt, GEdge *gacc, unsigned long long *cursor,
    unsigned long long *words_out, int32_t probe_ratio, int32_t chunk) {
  constexpr int NT = kGlobalNT;
  constexpr int CH = kGlobalChunkMax;
  constexpr int HS = 2 * kHubDeg;
  __shared__ uint32_t hA[HS];
  __shared__ uint32_t hB[HS];
  __shared__ uint32_t wl_v[CH];
  __shared__ int32_t wl_beg[CH];
  __shared__ int32_t wl_deg[CH];
  __shared__ int32_t wl_pref[CH + 1];
  __shared__ int32_t sh_cnt[4];
  __shared__ int32_t carry_sh[NT / kWave + 1];
  __shared__ unsigned long long red[NT / kWave];
  __shared__ long long sh_item;
  __shared__ int sh_last;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long words = 0;
  const int64_t total_items = nedges > 0 ? item_pref[nedges - 1] + item_cnt[nedges - 1] : 0;

  for (;;) {
    if (tid == 0) sh_item = (long long)atomicAdd(cursor, 1ull);
    __syncthreads();
    const int64_t item = sh_item;
    __syncthreads();
    if (item >= total_items) break;
    // edge of this item
    int64_t lo = 0, hi = nedges - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (item_pref[mid] <= item)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t e = lo;
    const int64_t c = item - item_pref[e];
    const int32_t slot = bslot[e];
    const SlotDesc &S = slots[slot];
    const int32_t *__restrict__ rp = S.row_ptr;
    const int32_t *__restrict__ col = S.col;
    const int64_t *__restrict__ hoff = S.hoff;
    const uint32_t *__restrict__ htab = S.htab;
    const int32_t a = ba[e], b = bb[e];
    const int32_t abeg = rp[a], aend = rp[a + 1], bbeg = rp[b], bend = rp[b + 1];
    const int da = aend - abeg, db = bend - bbeg;
    const bool ha = da > kHubDeg, hb = db > kHubDeg;
    const int alg = table_log(da), blg = table_log(db);
    const int64_t aoff = ha ? hoff[a] : 0, boff = hb ? hoff[b] : 0;
    if (tid < 4) sh_cnt[tid] = 0;
    // LDS tables for non-hub endpoints
    if (!hb) {
      for (int i = tid; i < (1 << blg); i += NT) hB[i] = kEmpty;
    }
    if (!ha) {
      for (int i = tid; i < (1 << alg); i += NT) hA[i] = kEmpty;
    }
    __syncthreads();
    if (!hb) {
      for (int i = tid; i < db; i += NT) {
        const int32_t x = col[bbeg + i];
        if (x != a) lds_insert(hB, blg, (uint32_t)x);
      }
      words += (unsigned long long)db;
    }
    if (!ha) {
      for (int i = tid; i < da; i += NT) {
        const int32_t x = col[abeg + i];
        if (x != b) lds_insert(hA, alg, (uint32_t)x);
      }
      words += (unsigned long long)da;
    }
    __syncthreads();
    // classify this chunk's w
    const int p0 = (int)(c * chunk);
    const int p1 = p0 + chunk < da ? p0 + chunk : da;
    for (int base = p0; base < p1; base += NT) {
      const int i = base + tid;
      bool valid = i < p1;
      const int32_t x = valid ? col[abeg + i] : -1;
      valid = valid && x != b;
      bool isT = false;
      if (valid) isT = side_has(hb, hB, blg, htab, boff, blg, (uint32_t)x);
      const uint64_t vm = __ballot(valid);
      const uint64_t tm = __ballot(isT);
      int pos0 = 0;
      if (lane == 0 && vm) {
        pos0 = atomicAdd(&sh_cnt[0], __popcll(vm));
        atomicAdd(&sh_cnt[1], __popcll(tm));
      }
      pos0 = __shfl(pos0, 0);
      if (valid) {
        const int pos = pos0 + __popcll(vm & lt_mask);
        const int32_t wb = rp[x], we = rp[x + 1];
        wl_v[pos] = (uint32_t)x | (isT ? kTag : 0u);
        wl_beg[pos] = wb;
        wl_deg[pos] = we - wb;
      }
    }
    words += (unsigned long long)(3 * (p1 - p0) + 4);
    __syncthreads();
    const int L = sh_cnt[0];
    const int tchunk = sh_cnt[1];
    // per-w strategy: scan Gamma(w), or walk the target source list (T_e from
    // the shorter of Gamma(a), Gamma(b); S_b from Gamma(b)) and look each
    // member up in Gamma(w)
    const int tsrc = da < db ? da : db;
    for (int i = tid; i < L; i += NT) {
      const uint32_t v = wl_v[i];
      const int dw = wl_deg[i];
      const int srcn = (v & kTag) ? tsrc : db;
      int units = dw;
      if (probe_ratio > 0) {
        const int cost = dw > kHubDeg ? 3 : ceil_log2((uint32_t)dw + 1u) + 1;
        const long long pc = (long long)srcn * (long long)cost * probe_ratio;
        if (pc < dw) {
          units = srcn;
          wl_v[i] = v | kProbe;
        }
      }
      wl_pref[i] = units;
    }
    __syncthreads();
    const int32_t total = block_scan_lds<NT>(wl_pref, L, carry_sh);
    if (tid == 0) wl_pref[L] = total;
    __syncthreads();
    unsigned long long k4 = 0, cyc = 0;
    uint32_t steps = 0;
    int cur = 0;
    for (int base = 0; base < total; base += NT) {
      const int idx = base + tid;
      if (idx < total) {
        int l2 = cur, h2 = L - 1;
        while (l2 < h2) {
          const int mid = (l2 + h2 + 1) >> 1;
          if (wl_pref[mid] <= idx)
            l2 = mid;
          else
            h2 = mid - 1;
        }
        cur = l2;
        const uint32_t v = wl_v[l2];
        const int off = idx - wl_pref[l2];
        const bool isT = (v & kTag) != 0;
        if (v & kProbe) {
          // candidate x from the source list, kept only if it is a target
          int32_t x;
          bool keep;
          if (isT) {
            if (da < db) {
              x = col[abeg + off];
              keep = x != b && side_has(hb, hB, blg, htab, boff, blg, (uint32_t)x);
            } else {
              x = col[bbeg + off];
              keep = x != a && side_has(ha, hA, alg, htab, aoff, alg, (uint32_t)x);
            }
          } else {
            x = col[bbeg + off];
            keep = x != a && !side_has(ha, hA, alg, htab, aoff, alg, (uint32_t)x);
          }
          ++steps;
          if (keep) {
            const int32_t w = (int32_t)(v & kIdMask);
            const int dw = wl_deg[l2];
            bool found;
            if (dw > kHubDeg) {
              found = table_find(htab + hoff[w], table_log(dw), (uint32_t)x) >= 0;
              steps += 2;
            } else {
              found = sorted_has(col + wl_beg[l2], dw, x, &steps);
            }
            if (found) {
              if (isT)
                ++k4;
              else
                ++cyc;
            }
          }
        } else {
          const int32_t r = col[wl_beg[l2] + off];
          ++steps;
          if (side_has(hb, hB, blg, htab, boff, blg, (uint32_t)r)) {
            // r in Gamma(b) \ {a}; in T_e iff also in Gamma(a)
            const bool rA = side_has(ha, hA, alg, htab, aoff, alg, (uint32_t)r);
            if (isT && rA) ++k4;
            if (!isT && !rA && r != a) ++cyc;
          }
        }
      }
    }
    words += steps;
    k4 = block_sum_u64<NT>(k4, red);
    cyc = block_sum_u64<NT>(cyc, red);
    if (tid == 0) {
      GEdge *g = gacc + e;
      if (tchunk) atomicAdd(&g->t, (unsigned long long)tchunk);
      if (k4) atomicAdd(&g->k4, k4);
      if (cyc) atomicAdd(&g->cyc, cyc);
      __threadfence();
      const unsigned long long d = atomicAdd(&g->done, 1ull);
      sh_last = (d + 1ull == (unsigned long long)item_cnt[e]) ? 1 : 0;
    }
    __syncthreads();
    if (sh_last && tid < kWave) {
      GEdge *g = gacc + e;
      __threadfence();
      const int64_t tt = (int64_t)atomicAdd(&g->t, 0ull);
      const int64_t kk = (int64_t)atomicAdd(&g->k4, 0ull);
      const int64_t cc = (int64_t)atomicAdd(&g->cyc, 0ull);
      if (lane <= kAccIdxCount) {
        const u128 v = edge_term(lane, S.n, S.m, da, db, tt, kk / 2, cc);
        if (v != 0) atomic_add_u128(S.acc + 2 * lane, v);
      }
    }
    __syncthreads();
  }
  const unsigned long long wsum = block_sum_u64<NT>(words, red);
  if (tid == 0 && wsum) atomicAdd(words_out, wsum);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_graph_validate(const int32_t *row_ptr, const int32_t *col, int64_t n, int *err,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_validate, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, n, err);
  return hipGetLastError();
}

hipError_t launch_graph_upper(const int32_t *row_ptr, const int32_t *col, int64_t n, int32_t *up_start,
                              int64_t *cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_upper, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, row_ptr, col, n,
                     up_start, cnt);
  return hipGetLastError();
}

hipError_t launch_scan_i64(const int64_t *in, int64_t *out, int64_t len, int64_t *tmp, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int64_t nb = (len + kScanBlock - 1) / kScanBlock;
  int64_t *sums = tmp;
  int64_t *sums_scanned = tmp + nb;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, in, out, len, sums);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || nb == 1) return err;
  err = launch_scan_i64(sums, sums_scanned, nb, tmp + 2 * nb, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, out, len, sums_scanned);
  return hipGetLastError();
}

int64_t scan_tmp_size(int64_t len) {
  int64_t need = 0;
  while (len > 1) {
    const int64_t nb = (len + kScanBlock - 1) / kScanBlock;
    need += 2 * nb;
    if (nb == 1) break;
    len = nb;
  }
  return need + 2;
}

hipError_t launch_graph_edges(const int32_t *row_ptr, const int32_t *col, const int32_t *up_start,
                              const int64_t *eid_base, int64_t n, uint64_t *edges, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_edges, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, up_start,
                     eid_base, n, edges);
  return hipGetLastError();
}

hipError_t launch_graph_vol2(const int32_t *row_ptr, const int32_t *col, int64_t n, int64_t *vol2,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_vol2, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, n, vol2);
  return hipGetLastError();
}

hipError_t launch_hub_sizes(const int32_t *row_ptr, int64_t n, int64_t *size, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hub_sizes, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, row_ptr, n, size);
  return hipGetLastError();
}

hipError_t launch_hub_build(const int32_t *row_ptr, const int32_t *col, int64_t n, const int64_t *hoff,
                            uint32_t *htab, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hub_build, dim3(grid_for(n, 64, 8192)), dim3(256), 0, s, row_ptr, col, n, hoff, htab);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t len, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(len, 256, 4096)), dim3(256), 0, s, p, len);
  return hipGetLastError();
}

hipError_t launch_sample_bin(const SlotDesc *slots, const RangeDesc *ranges, int32_t nranges, int64_t total,
                             Bins bins, KernelCfg cfg, hipStream_t s) {
  if (total <= 0 || nranges <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_bin, dim3(grid_for(total, 256, cfg.grid_sample)), dim3(256), 0, s, slots, ranges,
                     nranges, total, bins, cfg);
  return hipGetLastError();
}

template <int NT, int CAP>
static hipError_t launch_lds(const SlotDesc *slots, Bins bins, int cls, int64_t nedges, int grid_cap,
                             int32_t probe_ratio, hipStream_t s) {
  const int chunk = NT == kWave ? 4 : 1;
  const int grid = grid_for(nedges, chunk, grid_cap);
  hipLaunchKernelGGL((k_count_lds<NT, CAP>), dim3(grid), dim3(NT), 0, s, slots, bins.slot[cls], bins.a[cls],
                     bins.b[cls], nedges, bins.cursor + cls, bins.words + cls, probe_ratio, chunk);
  return hipGetLastError();
}

hipError_t launch_count_wave(const SlotDesc *slots, Bins bins, int64_t nedges, KernelCfg cfg, hipStream_t s) {
  if (nedges <= 0) return hipSuccess;
  const int d = cfg.wave_max_deg;
  if (d <= 64) return launch_lds<kWave, 64>(slots, bins, kClassWave, nedges, cfg.grid_wave, cfg.probe_ratio, s);
  if (d <= 128) return launch_lds<kWave, 128>(slots, bins, kClassWave, nedges, cfg.grid_wave, cfg.probe_ratio, s);
  if (d <= 256) return launch_lds<kWave, 256>(slots, bins, kClassWave, nedges, cfg.grid_wave, cfg.probe_ratio, s);
  return launch_lds<kWave, 512>(slots, bins, kClassWave, nedges, cfg.grid_wave, cfg.probe_ratio, s);
}

hipError_t launch_count_block(const SlotDesc *slots, Bins bins, int64_t nedges, KernelCfg cfg, hipStream_t s) {
  if (nedges <= 0) return hipSuccess;
  return launch_lds<256, kHubDeg>(slots, bins, kClassBlock, nedges, cfg.grid_block, cfg.probe_ratio, s);
}

hipError_t launch_global_prep(const SlotDesc *slots, Bins bins, int64_t nedges, int32_t chunk, int64_t *items,
                              void *gacc, hipStream_t s) {
  if (nedges <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_global_prep, dim3(grid_for(nedges, 256, 8192)), dim3(256), 0, s, slots,
                     bins.slot[kClassGlobal], bins.a[kClassGlobal], nedges, chunk, items, (GEdge *)gacc);
  return hipGetLastError();
}

hipError_t launch_count_global(const SlotDesc *slots, Bins bins, int64_t nedges, const int64_t *item_pref,
                               const int64_t *item_cnt, void *gacc, KernelCfg cfg, hipStream_t s) {
  if (nedges <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_global, dim3(cfg.grid_global), dim3(kGlobalNT), 0, s, slots,
                     bins.slot[kClassGlobal], bins.a[kClassGlobal], bins.b[kClassGlobal], nedges, item_pref,
                     item_cnt, (GEdge *)gacc, bins.cursor + kClassGlobal, bins.words + kClassGlobal,
                     cfg.probe_ratio, cfg.global_chunk);
  return hipGetLastError();
}

size_t gedge_bytes() { return sizeof(GEdge); }

}  // namespace lge
