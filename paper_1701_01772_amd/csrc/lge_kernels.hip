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
// in LDS for the edges counted by one workgroup, else in the per-vertex global
// hub table (every vertex of degree > kTableDeg has one) built
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
constexpr uint32_t kIdMask = 0x1FFFFFFFu;  // vertex ids < 2^29; bits 29..31 carry tags
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

// whether a vertex of degree d owns a global hub table (the single rule used
// by the table sizing, the table build and every lookup)
__device__ __forceinline__ bool has_table(int d) { return d > kHashDeg; }

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

// edge eid is taken iff p_lo <= uniform < p (p_lo = 0 is the plain Bernoulli(p)
// sample; thresholds of one uniform give nested samples)
__device__ __forceinline__ bool edge_taken(uint64_t seed, uint64_t eid, double p_lo, double p) {
  if (p >= 1.0 && p_lo <= 0.0) return true;  // the uniform is < 1 for every counter
  const uint64_t bits = philox_bits(seed, eid);
  const double u = (double)(bits >> 11) * 0x1.0p-53;
  return u >= p_lo && u < p;
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

// Per-edge write-out of (t, k4, cyc) for the micro statistics: the canonical
// edge list is sorted by (u << 32 | v), so a binary search over the requested
// id range gives the row.
__device__ __forceinline__ void micro_put(const SlotDesc &S, int32_t a, int32_t b, int64_t t, int64_t k4,
                                          int64_t cyc) {
  if (!S.micro) return;
  const uint64_t key = a < b ? (((uint64_t)(uint32_t)a << 32) | (uint32_t)b)
                             : (((uint64_t)(uint32_t)b << 32) | (uint32_t)a);
  int64_t lo = S.micro_base, hi = S.micro_base + S.micro_len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (S.edges[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < S.micro_base + S.micro_len && S.edges[lo] == key) {
    long long *row = S.micro + (lo - S.micro_base) * kMicroCols;
    row[kMicroColT] = t;
    row[kMicroColK4] = k4;
    row[kMicroColCyc] = cyc;
  }
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

// Scheduling weight of a graph: sum over canonical edges of
// d_u + d_v + min(vol2(u), vol2(v)), the neighbour-iteration cost of the
// cheaper orientation (an upper bound on the counting work per edge), summed
// over each block of kWorkBlock consecutive canonical edge ids: one
// wavefront per block.
__global__ __launch_bounds__(256) void k_graph_work(const int32_t *__restrict__ row_ptr,
                                                    const uint64_t *__restrict__ edges,
                                                    const int64_t *__restrict__ vol2, int64_t m,
                                                    unsigned long long *__restrict__ blocks) {
  const int lane = threadIdx.x & 63;
  const int64_t nb = (m + kWorkBlock - 1) / kWorkBlock;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t blk = w0; blk < nb; blk += nw) {
    const int64_t e1 = (blk + 1) * kWorkBlock < m ? (blk + 1) * kWorkBlock : m;
    unsigned long long acc = 0;
    for (int64_t e = blk * kWorkBlock + lane; e < e1; e += kWave) {
      const uint64_t x = edges[e];
      const int32_t u = (int32_t)(x >> 32), v = (int32_t)(uint32_t)x;
      const int64_t du = row_ptr[u + 1] - row_ptr[u], dv = row_ptr[v + 1] - row_ptr[v];
      const int64_t w = vol2[u] < vol2[v] ? vol2[u] : vol2[v];
      acc += (unsigned long long)(du + dv + w);
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) blocks[blk] = acc;
  }
}

// slot count (power of two) of each vertex's hub table; 0 for non-hubs
__global__ __launch_bounds__(256) void k_hub_sizes(const int32_t *__restrict__ row_ptr, int64_t n,
                                                   int64_t *size) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int d = row_ptr[u + 1] - row_ptr[u];
    size[u] = has_table(d) ? ((int64_t)1 << table_log(d)) : 0;
  }
}

__global__ __launch_bounds__(256) void k_hub_build(const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, int64_t n,
                                                   const int64_t *__restrict__ hoff, uint32_t *htab) {
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    const int d = end - beg;
    if (!has_table(d)) continue;  // uniform per block
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

// The same scan with the length read on the device (the work lists of a
// launch sequence are sized by earlier kernels of the sequence): grid-stride
// blocks of kScanBlock elements, one workgroup turning the block sums into
// block offsets (and writing the total), then the add.
__global__ __launch_bounds__(256) void k_scan_dev_blocks(const int64_t *__restrict__ in, int64_t *out,
                                                         const unsigned long long *__restrict__ len_p,
                                                         int64_t *block_sums) {
  __shared__ int64_t sh[256];
  const int64_t len = (int64_t)*len_p;
  const int64_t nb = (len + kScanBlock - 1) / kScanBlock;
  for (int64_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {  // uniform per block
    const int64_t base = bi * kScanBlock + threadIdx.x * 4;
    int64_t v[4];
    for (int i = 0; i < 4; ++i) v[i] = base + i < len ? in[base + i] : 0;
    const int64_t total = block_exclusive_scan_256x4(v, sh);
    for (int i = 0; i < 4; ++i)
      if (base + i < len) out[base + i] = v[i];
    if (threadIdx.x == 0) block_sums[bi] = total;
  }
}

__global__ __launch_bounds__(256) void k_scan_dev_sums(int64_t *block_sums, const unsigned long long *__restrict__ len_p,
                                                       unsigned long long *total) {
  __shared__ int64_t sh[256];
  const int64_t len = (int64_t)*len_p;
  const int64_t nb = (len + kScanBlock - 1) / kScanBlock;
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {  // uniform
    const int64_t base = b0 + threadIdx.x * 4;
    int64_t v[4];
    for (int i = 0; i < 4; ++i) v[i] = base + i < nb ? block_sums[base + i] : 0;
    const int64_t t = block_exclusive_scan_256x4(v, sh);
    for (int i = 0; i < 4; ++i)
      if (base + i < nb) block_sums[base + i] = carry + v[i];
    carry += t;
  }
  if (threadIdx.x == 0 && total) *total = (unsigned long long)carry;
}

__global__ __launch_bounds__(256) void k_scan_dev_add(int64_t *out, const unsigned long long *__restrict__ len_p,
                                                      const int64_t *__restrict__ offsets) {
  const int64_t len = (int64_t)*len_p;
  const int64_t nb = (len + kScanBlock - 1) / kScanBlock;
  for (int64_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int64_t off = offsets[bi];
    const int64_t base = bi * kScanBlock + threadIdx.x * 4;
    for (int i = 0; i < 4; ++i)
      if (base + i < len) out[base + i] += off;
  }
}

// ---------------------------------------------------------------------------
// Sampling and binning (a pass over the canonical edge ids of every range)
// ---------------------------------------------------------------------------

constexpr int kSamplePer = 4;  // edges per thread per round of the sampling kernel
// edges whose scan side has at most this degree (and whose other end owns a
// hub table) are counted by one wavefront (the wavefront class) instead of a
// workgroup or a split-class work item
constexpr int kSmallScan = 64;

__global__ __launch_bounds__(256) void k_sample_bin(const SlotDesc *__restrict__ slots,
                                                    const RangeDesc *__restrict__ ranges, int32_t nranges,
                                                    int64_t total, Bins bins, KernelCfg cfg) {
  constexpr int NT = 256, NW = NT / kWave;
  __shared__ int wcnt[kNumClasses][NW];
  __shared__ unsigned long long bbase[kNumClasses];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long algc[kNumClasses];
#pragma unroll
  for (int c = 0; c < kNumClasses; ++c) algc[c] = 0ull;
  // one round: NT * kSamplePer consecutive edge positions per workgroup; the
  // workgroup claims its positions in each class list with one atomic
  const int64_t span = (int64_t)NT * kSamplePer;
  for (int64_t base = (int64_t)blockIdx.x * span; base < total; base += (int64_t)gridDim.x * span) {
    int cls[kSamplePer];
    int32_t sl[kSamplePer], av[kSamplePer], bv[kSamplePer];
#pragma unroll
    for (int k = 0; k < kSamplePer; ++k) {
      const int64_t i = base + (int64_t)k * NT + threadIdx.x;
      cls[k] = -1;
      sl[k] = 0;
      av[k] = 0;
      bv[k] = 0;
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
        int32_t slot = R.slot;
        const SlotDesc &S = slots[slot];
        const int64_t eid = R.e0 + (i - R.pref);
        bool take;
        if (S.design == kDesignBernoulli) {
          take = edge_taken(S.seed, (uint64_t)eid, S.p_lo, S.p);
        } else if (S.design == kDesignWeighted) {
          const int l = S.level[eid];
          take = edge_taken(S.seed, (uint64_t)eid, 0.0, S.plev[l]);
          slot += l;
        } else {
          const uint64_t key = philox_bits(S.seed, (uint64_t)eid);
          take = key < S.kkey || (key == S.kkey && eid <= S.keid);
        }
        if (take) {
          const uint64_t e = S.edges[eid];
          const int32_t u = (int32_t)(e >> 32), v = (int32_t)(uint32_t)e;
          const int32_t du = S.row_ptr[u + 1] - S.row_ptr[u];
          const int32_t dv = S.row_ptr[v + 1] - S.row_ptr[v];
          const int64_t wu = S.vol2[u], wv = S.vol2[v];
          // iterate the side whose neighbours have the smaller total degree
          const bool ua = wu < wv || (wu == wv && (du < dv || (du == dv && u < v)));
          av[k] = ua ? u : v;
          bv[k] = ua ? v : u;
          sl[k] = slot;
          const int32_t dmax = du > dv ? du : dv;
          const int64_t da = ua ? du : dv, db = ua ? dv : du, wa = ua ? wu : wv;
          // an edge with a small scan side and b owning a hub table is
          // counted by one wavefront (using b's hub table) whatever b's degree
          const bool small_scan = cfg.probe_ratio > 0 && da <= kSmallScan && db > kTableDeg;
          const int c = (dmax <= cfg.wave_max_deg || small_scan) ? kClassWave
                        : dmax <= cfg.block_max_deg               ? kClassBlock
                                                                  : kClassGlobal;
          cls[k] = c;
          // bytes the neighbour iteration of Alg. 2-4 reads for this edge:
          // both row_ptr pairs, both rows, and for every w in Gamma(a) \ {b}
          // its row_ptr pair and row
          const unsigned long long alg = 16ull + 4ull * (unsigned long long)(du + dv) +
                                         8ull * (unsigned long long)(da - 1) + 4ull * (unsigned long long)(wa - db);
#pragma unroll
          for (int q = 0; q < kNumClasses; ++q)
            if (c == q) algc[q] += alg;
        }
      }
    }
    int wc[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
      int nc = 0;
#pragma unroll
      for (int k = 0; k < kSamplePer; ++k) nc += __popcll(__ballot(cls[k] == c));
      wc[c] = nc;
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kNumClasses; ++c) wcnt[c][wid] = wc[c];
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += wcnt[threadIdx.x][w];
      bbase[threadIdx.x] = tot ? atomicAdd(&bins.count[threadIdx.x], (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
      if (wc[c] == 0) continue;  // uniform per wavefront
      int64_t pos = (int64_t)bbase[c];
      for (int w = 0; w < wid; ++w) pos += wcnt[c][w];
#pragma unroll
      for (int k = 0; k < kSamplePer; ++k) {
        const uint64_t msk = __ballot(cls[k] == c);
        if (cls[k] == c) {
          const int64_t at = pos + __popcll(msk & lt_mask);
          bins.slot[c][at] = sl[k];
          bins.a[c][at] = av[k];
          bins.b[c][at] = bv[k];
        }
        pos += __popcll(msk);
      }
    }
    __syncthreads();  // wcnt and bbase are rewritten next round
  }
#pragma unroll
  for (int c = 0; c < kNumClasses; ++c) {
    const unsigned long long v = wave_sum_u64(algc[c]);
    if (lane == 0 && v) atomicAdd(&bins.alg[(c * kXcds + blockIdx.x % kXcds) * kLine], v);
  }
}

// ---------------------------------------------------------------------------
// Co-degree table of the high-degree vertices: codeg[i][j] = |Gamma(x) n
// Gamma(y)| for the vertices x, y of ranks i, j among those with degree > tau.
// Built once per graph: every vertex's ranked neighbours as a list of ranks,
// then one LDS-counted row per ranked vertex (each common neighbour w of x
// and y is seen once, from w's list, while walking Gamma(x)).
// ---------------------------------------------------------------------------

// number of ranked neighbours of every vertex
__global__ __launch_bounds__(256) void k_codeg_count(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ crank, int64_t n, int64_t *cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    unsigned long long c = 0;
    for (int32_t j = row_ptr[u] + lane; j < row_ptr[u + 1]; j += kWave) c += crank[col[j]] >= 0 ? 1ull : 0ull;
    c = wave_sum_u64(c);
    if (lane == 0) cnt[u] = (int64_t)c;
  }
}

// every vertex's ranked neighbours as ranks, those below kRankSplit first
// (in adjacency order) and the others after them (in reverse), with the
// number of the first kind in nlo: a pass of the row builder over a range
// of ranks reads only its part
constexpr int32_t kRankSplit = 65536;
__global__ __launch_bounds__(256) void k_codeg_fill(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ crank, int64_t n,
                                                    const int64_t *__restrict__ off, const int64_t *__restrict__ cnt,
                                                    int32_t *list, int32_t *__restrict__ nlo) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int64_t o = off[u];
    int64_t lo = o, hi = o + cnt[u];  // next low slot; one past the next high slot
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    for (int32_t base = beg; base < end; base += kWave) {
      const int32_t j = base + lane;
      const int32_t r = j < end ? crank[col[j]] : -1;
      const uint64_t ml = __ballot(r >= 0 && r < kRankSplit);
      const uint64_t mh = __ballot(r >= kRankSplit);
      if (r >= 0 && r < kRankSplit) list[lo + __popcll(ml & lt_mask)] = r;
      if (r >= kRankSplit) list[hi - 1 - __popcll(mh & lt_mask)] = r;
      lo += __popcll(ml);
      hi -= __popcll(mh);
    }
    if (lane == 0) nlo[u] = (int32_t)(lo - o);
  }
}

// Co-degree rows counted in LDS: one workgroup per ranked vertex x of rank
// rx.  For every w in Gamma(x), every ranked neighbour of w (w's rank list)
// adds 1 at its rank's column, so the row ends up holding
// |Gamma(x) n Gamma(y)| for every ranked y; it is then written once,
// coalesced, diagonal 0, as 16-bit entries.  A co-degree never exceeds
// deg(x): rows of x with deg(x) < 2^16 count in the 16-bit halves of the LDS
// words (2 * kRowWords ranks per pass), the others in 32-bit words
// (kRowWords ranks per pass).  A wave loads 64 of the w at once (coalesced)
// and walks the short lists each in its own lane, the long ones one after
// another, lanes striding each.
constexpr int kRowNT = 1024;
constexpr int kRowWords = 32768;  // 128 KB of LDS counters
constexpr int kOwnSeg = 16;       // longest list (segment) a lane walks by itself
constexpr int kCoopUnroll = 8;    // reads per lane in flight when a wave walks a long list
constexpr int kRankUnroll = 16;   // the same for the rank lists of the co-degree table
__global__ __launch_bounds__(kRowNT) void k_codeg_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ ranked,
                                                        const int64_t *__restrict__ off,
                                                        const int64_t *__restrict__ cnt,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ nlo, int64_t hc,
                                                        uint16_t *__restrict__ tab) {
  __shared__ uint32_t c[kRowWords];
  const int64_t rx = blockIdx.x;
  const int32_t x = ranked[rx];
  const int32_t beg = rp[x], d = rp[x + 1] - beg;
  const bool narrow = d < 65536;
  const int64_t span = narrow ? 2 * (int64_t)kRowWords : (int64_t)kRowWords;  // ranks per pass
  const int passes = (int)((hc + span - 1) / span);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int kWaves = kRowNT / kWave;
  uint16_t *row = tab + rx * hc;
  for (int pass = 0; pass < passes; ++pass) {
    const int64_t c0 = (int64_t)pass * span;
    const int64_t c1 = c0 + span < hc ? c0 + span : hc;
    const int64_t words = narrow ? (c1 - c0 + 1) / 2 : c1 - c0;
    // the part of each rank list this pass needs: ranks below kRankSplit
    // sit first, the others after them
    const bool low_only = c1 <= kRankSplit, high_only = c0 >= kRankSplit;
    for (int64_t i = threadIdx.x; i < words; i += kRowNT) c[i] = 0u;
    __syncthreads();
    for (int32_t g0 = wid * kWave; g0 < d; g0 += kWaves * kWave) {
      const int32_t j = g0 + lane;
      const int32_t w = j < d ? col[beg + j] : -1;
      long long o = w >= 0 ? (long long)off[w] : 0ll;
      int k = w >= 0 ? (int)cnt[w] : 0;
      if (w >= 0 && (low_only || high_only)) {
        const int kl = nlo[w];
        if (low_only) {
          k = kl;
        } else {
          o += kl;
          k -= kl;
        }
      }
      auto add = [&](int32_t y) {
        if (y < c0 || y >= c1) return;
        const int32_t yy = y - (int32_t)c0;
        if (narrow)
          atomicAdd(&c[yy >> 1], 1u << ((yy & 1) << 4));
        else
          atomicAdd(&c[yy], 1u);
      };
      // a short list is walked by its own lane, from a lane-dependent start
      // (lists share their hub ranks, and lanes adding at one counter at
      // once serialise); the wave walks the long ones one after another
      const bool own = k <= kOwnSeg;
      if (own && k > 0) {
        const int st = lane % k;
        for (int s0 = 0; s0 < k; s0 += 4) {
          int32_t ys[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            int idx = st + s0 + u;
            if (idx >= k) idx -= k;
            ys[u] = s0 + u < k ? list[o + idx] : -1;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) add(ys[u]);
        }
      }
      uint64_t lm = __ballot(!own);
      while (lm) {  // uniform per wave
        const int q = __ffsll((long long)lm) - 1;
        lm &= lm - 1;
        const long long oq = __shfl(o, q);
        const int kq = __shfl(k, q);
        for (int i0 = lane; i0 < kq; i0 += kRankUnroll * kWave) {  // kRankUnroll reads in flight
          int32_t ys[kRankUnroll];
#pragma unroll
          for (int u = 0; u < kRankUnroll; ++u) ys[u] = i0 + u * kWave < kq ? list[oq + i0 + u * kWave] : -1;
#pragma unroll
          for (int u = 0; u < kRankUnroll; ++u) add(ys[u]);
        }
      }
    }
    __syncthreads();
    // one 16-bit entry per rank; a count of 65535 or more (both ends of
    // degree >= 65535, never read) is clamped
    for (int64_t y = c0 + threadIdx.x; y < c1; y += kRowNT) {
      const int64_t yy = y - c0;
      const uint32_t v = narrow ? (c[yy >> 1] >> ((yy & 1) << 4)) & 0xFFFFu : c[yy];
      row[y] = y == rx ? (uint16_t)0 : (uint16_t)(v < 0xFFFFu ? v : 0xFFFFu);
    }
    __syncthreads();
  }
}

// Co-degree rows over the unranked columns, one workgroup per (row h,
// column tile t): the row's hub y, every x in Gamma(y), and x's neighbours w
// with a column in the tile, counted in LDS (each w once per x, so the entry
// ends as |Gamma(y) n Gamma(w)|).  Every vertex's neighbours that have a
// column are first listed as columns, in increasing order (columns go by
// vertex id, and the adjacency lists are sorted); the tile's part of x's list
// is then one segment, whose ends a separate pass finds once per (x, tile)
// (k_rows_offsets).  Two 16-bit LDS counters per word, so a tile spans
// 65,536 columns (an entry never exceeds the unranked vertex's degree, at
// most 65,535; one counter per word took 20 % longer on Chung-Lu 1M, four
// byte counters per word 30 % longer); the tile is then written out once as
// entries of `width` bytes.  A wave reads the segment ends of 64 x at once; a lane
// walks its own x's segment when it is short, and the wave walks the long
// ones one after another, lanes striding each.
constexpr int kTileNT = 1024;
constexpr int kTileWords = 32768;        // 128 KB of LDS counters
constexpr int kTileCols = 2 * kTileWords;  // columns per tile: 16-bit halves

__device__ __forceinline__ int64_t lower_pos(const int32_t *__restrict__ a, int64_t lo, int64_t hi, int32_t v) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// column of an arc's head from its packed word (-1: ranked, or no column)
__device__ __forceinline__ int32_t arc_column(uint32_t r) {
  return (r >> 31) ? (int32_t)(r & 0x7FFFFFFFu) - 1 : -1;
}

// number of every vertex's neighbours that have a column
__global__ __launch_bounds__(256) void k_col_count(const int32_t *__restrict__ rp, const uint32_t *__restrict__ arh,
                                                   int64_t n, int64_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    unsigned long long c = 0;
    for (int32_t j = rp[u] + lane; j < rp[u + 1]; j += kWave) c += arc_column(arh[j]) >= 0 ? 1ull : 0ull;
    c = wave_sum_u64(c);
    if (lane == 0) cnt[u] = (int64_t)c;
  }
}

// the columns of every vertex's neighbours, in adjacency order, at off[u]
__global__ __launch_bounds__(256) void k_col_fill(const int32_t *__restrict__ rp, const uint32_t *__restrict__ arh,
                                                  int64_t n, const int64_t *__restrict__ off,
                                                  int32_t *__restrict__ clist) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwaves) {
    int64_t at = off[u];
    const int32_t end = rp[u + 1];
    for (int32_t base = rp[u]; base < end; base += kWave) {
      const int32_t j = base + lane;
      const int32_t cc = j < end ? arc_column(arh[j]) : -1;
      const uint64_t m = __ballot(cc >= 0);
      if (cc >= 0) clist[at + __popcll(m & lt_mask)] = cc;
      at += __popcll(m);
    }
  }
}

// toff[x * (nb + 1) + i] = first position of x's column list at or above
// column (t0 + i) * kTileCols, for every vertex x and i in [0, nb]
__global__ __launch_bounds__(256) void k_rows_offsets(const int64_t *__restrict__ off, const int64_t *__restrict__ cnt,
                                                      const int32_t *__restrict__ clist, int64_t n, int64_t t0,
                                                      int64_t nb, int32_t *__restrict__ toff) {
  const int64_t per = nb + 1, total = n * per;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = i / per, k = i - x * per;
    const int64_t lo = off[x];
    toff[i] = (int32_t)lower_pos(clist, lo, lo + cnt[x], (int32_t)((t0 + k) * kTileCols));
  }
}

// tiles [t0, t0 + nb) of every row; toff from k_rows_offsets over the same
// tiles
__global__ __launch_bounds__(kTileNT) void k_rows_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ clist,
                                                       const int32_t *__restrict__ hubs, int64_t nh,
                                                       const int32_t *__restrict__ toff, int64_t t0, int64_t nb,
                                                       int64_t ncol, int64_t stride, int width,
                                                       uint8_t *__restrict__ rows) {
  __shared__ uint32_t c[kTileWords];
  const int64_t T = kTileCols;
  // column q of the tile: the 16-bit half q & 1 of word q >> 1
  auto bump = [&](int32_t q) { atomicAdd(&c[q >> 1], 1u << ((q & 1) << 4)); };
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int kWaves = kTileNT / kWave;
  const int64_t per = nb + 1;
  for (int64_t wi = blockIdx.x; wi < nh * nb; wi += gridDim.x) {  // uniform per block
    const int64_t h = wi / nb, tt = wi % nb, t = t0 + tt;
    const int32_t y = hubs[h];
    const int64_t c0 = t * T, c1 = c0 + T < ncol ? c0 + T : ncol;
    const int64_t cols = c1 - c0;
    const int64_t words = (cols + 1) >> 1;
    const int32_t base = (int32_t)c0;
    for (int64_t i = threadIdx.x; i < words; i += kTileNT) c[i] = 0u;
    __syncthreads();
    const int32_t ybeg = rp[y], dy = rp[y + 1] - ybeg;
    for (int32_t g0 = wid * kWave; g0 < dy; g0 += kWaves * kWave) {
      const int32_t j = g0 + lane;
      int32_t lo = 0, hi = 0;
      if (j < dy) {
        const int64_t x = col[ybeg + j];
        lo = toff[x * per + tt];
        hi = toff[x * per + tt + 1];
      }
      const bool own = hi - lo <= kOwnSeg;
      for (int32_t k = own ? lo : hi; k < hi; k += 4) {
        int32_t cs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cs[u] = k + u < hi ? clist[k + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (cs[u] >= 0) bump(cs[u] - base);
      }
      uint64_t lm = __ballot(!own);
      while (lm) {  // uniform per wave
        const int q = __ffsll((long long)lm) - 1;
        lm &= lm - 1;
        const int32_t lq = __shfl(lo, q), hq = __shfl(hi, q);
        for (int32_t k0 = lq + lane; k0 < hq; k0 += kCoopUnroll * kWave) {  // kCoopUnroll reads in flight
          int32_t cs[kCoopUnroll];
#pragma unroll
          for (int u = 0; u < kCoopUnroll; ++u) cs[u] = k0 + u * kWave < hq ? clist[k0 + u * kWave] : -1;
#pragma unroll
          for (int u = 0; u < kCoopUnroll; ++u)
            if (cs[u] >= 0) bump(cs[u] - base);
        }
      }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < cols; i += kTileNT) {
      const uint32_t v = (c[i >> 1] >> ((i & 1) << 4)) & 0xFFFFu;
      if (width == 1)
        rows[h * stride + c0 + i] = (uint8_t)v;
      else
        reinterpret_cast<uint16_t *>(rows)[h * stride + c0 + i] = (uint16_t)v;
    }
    __syncthreads();
  }
}

// column c of co-degree row r
__device__ __forceinline__ uint32_t row_at(const SlotDesc &S, int64_t r, int64_t x) {
  const int64_t i = r * S.rows_stride + x;
  return S.rows_w == 1 ? (uint32_t)S.rows[i] : (uint32_t)reinterpret_cast<const uint16_t *>(S.rows)[i];
}

// (row start, degree, rank or -1, co-degree row of a ranked vertex or row
// column of an unranked one, -1 if none) of every vertex
__global__ __launch_bounds__(256) void k_vinfo(const int32_t *__restrict__ rp, const int32_t *__restrict__ crank,
                                               const int32_t *__restrict__ hrow, const int32_t *__restrict__ rcol,
                                               int64_t n, int4 *__restrict__ vinfo) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = crank ? crank[v] : -1;
    const int32_t h = r >= 0 ? (hrow ? hrow[v] : -1) : (rcol ? rcol[v] : -1);
    vinfo[v] = make_int4(rp[v], rp[v + 1] - rp[v], r, h);
  }
}

// the rank and row / column of every arc's head, packed into one word and
// stored beside the adjacency lists (read with them, coalesced): ranked
// (rank + 1) | (row + 1) << 17, unranked 1 << 31 | (column + 1)
__global__ __launch_bounds__(256) void k_arc_rank(const int32_t *__restrict__ col, const int4 *__restrict__ vinfo,
                                                  int64_t nnz, uint32_t *__restrict__ arh) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x) {
    const int4 v = vinfo[col[j]];
    arh[j] = v.z >= 0 ? (uint32_t)(v.z + 1) | ((uint32_t)(v.w + 1) << 17) : (0x80000000u | (uint32_t)(v.w + 1));
  }
}

__global__ __launch_bounds__(256) void k_codeg_bits(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ crank, int64_t n, int64_t hcw,
                                                    unsigned long long *bits) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t x = w0; x < n; x += nw) {
    const int32_t rx = crank[x];
    if (rx < 0) continue;  // uniform per wavefront
    unsigned long long *row = bits + (int64_t)rx * hcw;
    for (int32_t j = rp[x] + lane; j < rp[x + 1]; j += 64) {
      const int32_t ry = crank[col[j]];
      if (ry >= 0) atomicOr(row + (ry >> 6), 1ull << (ry & 63));
    }
  }
}

// |Gamma(x) n Gamma(y)| when tabulated: both ranked (the symmetric table,
// y's row), or one end unranked with a row column and the other ranked with
// a co-degree row.  rhx is the packed rank word of an arc ending at x (rank
// + 1 and co-degree row + 1 when ranked, else bit 31 and column + 1); vy is
// y's vertex record.
__device__ __forceinline__ bool codeg_pair(const SlotDesc &S, uint32_t rhx, int4 vy, uint32_t *val) {
  if (S.hc <= 0) return false;
  const bool xr = (rhx >> 31) == 0u;
  const int32_t xrank = xr ? (int32_t)(rhx & 0x1FFFFu) - 1 : -1;
  const int32_t xw = xr ? (int32_t)(rhx >> 17) - 1 : (int32_t)(rhx & 0x7FFFFFFFu) - 1;
  if (xrank >= 0 && vy.z >= 0) {
    if (xrank >= S.codeg_sat && vy.z >= S.codeg_sat) return false;  // may exceed 16 bits
    *val = S.codeg[(int64_t)vy.z * S.hc + xrank];
    return true;
  }
  if (xrank < 0 && xw >= 0 && vy.z >= 0 && vy.w >= 0) {  // x's column of y's row
    *val = row_at(S, vy.w, xw);
    return true;
  }
  if (vy.z < 0 && vy.w >= 0 && xrank >= 0 && xw >= 0) {  // y's column of x's row
    *val = row_at(S, xw, vy.w);
    return true;
  }
  return false;
}

// ---------------------------------------------------------------------------
// Block-level helpers for the counting kernels
// ---------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long *red) {
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

// two block sums with one round of barriers (red holds 2 * NT / kWave words)
template <int NT>
__device__ __forceinline__ void block_sum2_u64(unsigned long long &x, unsigned long long &y,
                                               unsigned long long *red) {
  x = wave_sum_u64(x);
  y = wave_sum_u64(y);
  if constexpr (NT != kWave) {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[w] = x;
      red[NT / kWave + w] = y;
    }
    __syncthreads();
    unsigned long long sx = 0, sy = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
      sx += red[i];
      sy += red[NT / kWave + i];
    }
    __syncthreads();
    x = sx;
    y = sy;
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

// Accumulates one edge's terms in the registers of wave 0 (lane k holds
// accumulator k) and flushes them into the slot when the slot changes.
struct SlotAcc {
  u128 acc;
  int32_t slot;
  __device__ void init() {
    acc = 0;
    slot = -1;
  }
  __device__ void flush(const SlotDesc *__restrict__ slots) {
    const int lane = threadIdx.x & 63;
    if (slot >= 0 && lane < kAccSlots && acc != 0) {
      const SlotDesc &S = slots[slot];
      const int64_t r = (int64_t)(blockIdx.x % (unsigned)S.acc_reps);
      atomic_add_u128(S.acc + r * (kAccSlots * 2) + 2 * lane, acc);
    }
    acc = 0;
  }
  __device__ void add(const SlotDesc *__restrict__ slots, int32_t s, int64_t n, int64_t m, int64_t da, int64_t db,
                      int64_t t, int64_t k4, int64_t cyc) {
    const int lane = threadIdx.x & 63;
    if (s != slot) {
      flush(slots);
      slot = s;
    }
    if (lane <= kAccIdxCount) acc += edge_term(lane, n, m, da, db, t, k4, cyc);
  }
};

// ---------------------------------------------------------------------------
// Per-neighbour work of the workgroup classes.  With probe_ratio > 0 they
// count in the aggregate form the split class uses,
//   cyc = sum_{w in S_a} cbx(w) - sum_{x in T_e} cax(x) + sum_{x in T_e} degT(x),
// cbx(w) = |Gamma(w) n Gamma(b)\{a}|, cax(x) = |Gamma(x) n Gamma(a)\{b}|,
// degT(x) = |Gamma(x) n T_e|, k4 = sum degT / 2, and pick per w the cheapest
// way to each term:
//   w in S_a : cbx = codeg(w,b) - 1 when tabulated (no units); else scan
//              Gamma(w) against the table of Gamma(b)\{a}        units = d_w
//              or look each of Gamma(b)\{a} up in Gamma(w)       units = d_b - 1
//   x in T_e : degT by scan (T-tagged hits)                      units = d_x
//              or by looking T_e up in Gamma(x) (Alg. 5)         units = t
//              cax = codeg(x,a) - 1 when tabulated, else look each of
//              Gamma(a)\{b} up in Gamma(x)                       units = d_a - 1
// With probe_ratio <= 0 every w scans Gamma(w) (neighbour iteration,
// Alg. 3/4): S_a members count their neighbours in S_b, T_e members theirs
// in T_e.  "Look up x in Gamma(w)" uses w's hub table when d_w > kHashDeg,
// else a binary search of the sorted list.  Costs are in quarter units: a
// scanned entry costs 8 (a coalesced load and a table probe), a look-up
// 4*(2 + probe cost) scaled by probe_ratio / 4.
// ---------------------------------------------------------------------------

// workgroups per XCD that take blocks from the other XCDs' queues
constexpr int kLdsStealers = 16;

// One claim from the XCD-local queues of the LDS counting kernels (see
// there): the next block [*e0, *e1) of the class list, *e0 = -1 when this
// workgroup is done.  *qpos holds the workgroup's place in its queue order
// (0: its own XCD's queue).  Not inlined and recomputing its parameters from
// the launch shape each time, so it holds no registers across the edge loop.
__device__ __noinline__ void lds_claim(unsigned long long *xcd_cursor, int64_t nedges, int max_chunk, int stealers,
                                       int *qpos, long long *e0, long long *e1) {
  const int nseg = gridDim.x % kXcds == 0 ? kXcds : 1;
  const int my_seg = (int)(blockIdx.x % (unsigned)nseg);
  int64_t run = nedges / (4 * (int64_t)gridDim.x);
  run = run < 1 ? 1 : (run > max_chunk ? max_chunk : run);
  const int64_t nblk = (nedges + run - 1) / run;
  const bool stealer = (int64_t)(blockIdx.x / (unsigned)nseg) < (int64_t)stealers;
  int seg_off = *qpos;
  long long b0 = -1, b1 = -1;
  while (seg_off < nseg && (seg_off == 0 || stealer)) {
    const int sg = (my_seg + seg_off) % nseg;
    const int64_t j = (int64_t)atomicAdd(&xcd_cursor[sg * kLine], 1ull) * nseg + sg;
    if (j < nblk) {
      b0 = j * run;
      b1 = b0 + run < nedges ? b0 + run : nedges;
      break;
    }
    ++seg_off;
  }
  *qpos = seg_off;
  *e0 = b0;
  *e1 = b1;
}

constexpr uint32_t kModeLook = 0x40000000u;  // S_a: look Gamma(b)\{a} up; T_e: degT by looking T_e up
constexpr uint32_t kModeAux = 0x20000000u;   // S_a: cbx tabulated (no units); T_e: cax by look-ups

__device__ __forceinline__ int64_t look_cost(int dw, int probe_ratio) {
  return (int64_t)((has_table(dw) ? 1 : ceil_log2((uint32_t)dw + 1u)) + 2) * probe_ratio;
}

// is x in Gamma(w)?  (w's hub table, or binary search of its sorted list)
__device__ __forceinline__ bool w_has(const SlotDesc &S, int32_t w, int32_t wbeg, int dw, int32_t x,
                                      uint32_t *steps) {
  if (has_table(dw)) {
    *steps += 2;
    return table_find(S.htab + S.hoff[w], table_log(dw), (uint32_t)x) >= 0;
  }
  return sorted_has(S.col + wbeg, dw, x, steps);
}

// ---------------------------------------------------------------------------
// LDS counting kernel: one edge per workgroup of NT threads, both endpoint
// degrees <= CAP.  LDS holds the hash of Gamma(b) \ {a} (bit 31 tags members
// of T_e), the list of w in Gamma(a) \ {b} with their modes and unit prefix,
// and the target list (T_e at the front, S_b at the back).
// ---------------------------------------------------------------------------

template <int NT, int CAP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_count_lds(const SlotDesc *__restrict__ slots, const int32_t *__restrict__ bslot,
                                                  const int32_t *__restrict__ ba, const int32_t *__restrict__ bb,
                                                  const unsigned long long *__restrict__ ncount,
                                                  unsigned long long *xcd_cursor,
                                                  unsigned long long *words_out, int32_t probe_ratio, int32_t max_chunk,
                                                  int32_t stealers) {
  constexpr int HS = 2 * CAP;
  __shared__ uint32_t htab[HS];
  __shared__ uint32_t wl_v[CAP];
  __shared__ int32_t wl_beg[CAP];
  __shared__ uint16_t wl_dg[CAP];  // degrees, 0xFFFF standing for 65535 or more
  __shared__ int32_t wl_pref[CAP + 1];
  __shared__ int32_t tgt[CAP];
  __shared__ int32_t sh_cnt[4];
  __shared__ int32_t carry_sh[NT / kWave + 1];
  __shared__ unsigned long long red[NT / kWave];
  __shared__ long long sh_e0, sh_e1;
  __shared__ int sh_qpos;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const SlotDesc *cur_slot = nullptr;  // the slot of the edge being counted
  // degree of w-list entry i (a saturated entry is read from its record)
  auto deg_of = [&](int i) -> int {
    const int d = wl_dg[i];
    return d < 0xFFFF ? d : cur_slot->vinfo[wl_v[i] & kIdMask].y;
  };
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t nedges = (int64_t)*ncount;  // the class's edges, binned by the sampling kernel
  if (nedges == 0) return;  // uniform
  SlotAcc acc;
  acc.init();
  unsigned long long words = 0;
  // XCD-local queues: the class list is cut into blocks of `run` consecutive
  // edges, block j in queue j % kXcds (one queue when the grid is not a
  // multiple of kXcds), so every queue sees the same mix of light and heavy
  // edges (heavy ones cluster: the rows of hubs).  The workgroups of XCD x
  // (blockIdx % kXcds) take blocks from queue x, each claim one atomic on
  // that queue's own cache line; once it is empty `stealers` of them per XCD
  // go on to the other queues (few for light edges, which keeps the failed
  // claims at the end few).  A block mostly keeps one slot (the register sums
  // are flushed when it changes); about four blocks per workgroup keep the
  // tail short.
  if (tid == 0) sh_qpos = 0;

  for (;;) {
    if (tid == 0) lds_claim(xcd_cursor, nedges, max_chunk, stealers, &sh_qpos, &sh_e0, &sh_e1);
    __syncthreads();
    const int64_t e0 = sh_e0, e1 = sh_e1;
    __syncthreads();
    if (e0 < 0) break;
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t slot = bslot[e];
      const int32_t a = ba[e], b = bb[e];
      const SlotDesc &S = slots[slot];
      cur_slot = &S;
      const int32_t *__restrict__ col = S.col;
      // endpoint records (row start, degree, rank, co-degree row / column);
      // the rank fields count only when co-degrees are read
      int4 va = S.vinfo[a], vb = S.vinfo[b];
      const int32_t abeg = va.x, bbeg = vb.x;
      const int da = va.y, db = vb.y;
      const bool has_ranks = probe_ratio > 0 && S.hc > 0;
      if (!has_ranks) va.z = va.w = vb.z = vb.w = -1;
      // an edge with a small scan side and a large b (binned here by the
      // sampling kernel): Gamma(b) stays in b's hub table, the LDS table holds T_e
      const bool bhub = db > CAP;
      const uint32_t *__restrict__ btab = bhub ? S.htab + S.hoff[b] : nullptr;
      const int blg = bhub ? table_log(db) : 0;
      const int lg = table_log(bhub ? da : db);
      const int hs = 1 << lg;
      for (int i = tid; i < hs; i += NT) htab[i] = kEmpty;
      if (tid < 4) sh_cnt[tid] = 0;
      __syncthreads();
      if (!bhub) {
        for (int i = tid; i < db; i += NT) {
          const int32_t x = col[bbeg + i];
          if (x != a) lds_insert(htab, lg, (uint32_t)x);
        }
      }
      if (tid == 0) words += (unsigned long long)((bhub ? 0 : db) + 4);  // per-edge terms counted once
      __syncthreads();
      // classify Gamma(a) \ {b}: in the hash -> T_e (tag it), else S_a
      for (int base = 0; base < da; base += NT) {
        const int i = base + tid;
        bool valid = i < da;
        const int32_t x = valid ? col[abeg + i] : -1;
        // the arc's packed rank word, read coalesced beside Gamma(a)
        const uint32_t rh = valid && has_ranks ? S.arh[abeg + i] : 0x80000000u;
        valid = valid && x != b;
        bool isT = false;
        if (valid && bhub) {
          isT = table_find(btab, blg, (uint32_t)x) >= 0;
          if (isT) lds_insert(htab, lg, (uint32_t)x | kTag);
        } else if (valid) {
          const int sl = table_find(htab, lg, (uint32_t)x);
          if (sl >= 0) {
            isT = true;
            htab[sl] = (uint32_t)x | kTag;
          }
        }
        const uint64_t vm = __ballot(valid);
        int pos0 = 0;
        if (lane == 0 && vm) pos0 = atomicAdd(&sh_cnt[0], __popcll(vm));
        pos0 = __shfl(pos0, 0);
        if (valid) {
          const int pos = pos0 + __popcll(vm & lt_mask);
          const int4 vx = S.vinfo[x];
          wl_v[pos] = (uint32_t)x | (isT ? kTag : 0u);
          wl_beg[pos] = vx.x;
          wl_dg[pos] = (uint16_t)(vx.y < 0xFFFF ? vx.y : 0xFFFF);
          wl_pref[pos] = (int32_t)rh;  // until the mode pass turns it into the unit count
        }
      }
      if (tid == 0) words += (unsigned long long)(3 * da);
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
      // per-w modes under both schemes; the edge takes the cheaper one
      const bool may_look = probe_ratio > 0;
      long long cyc_base = 0;
      unsigned long long c_plain = 0, c_agg = 0;
      for (int i = tid; i < L; i += NT) {
        const uint32_t v = wl_v[i];
        const bool isT = (v & kTag) != 0;
        const uint32_t rh = (uint32_t)wl_pref[i];
        const int dw = deg_of(i);
        const int64_t scan = 8ll * dw;
        if (!may_look) {
          c_plain += (unsigned long long)scan;
          continue;
        }
        const int64_t lk = look_cost(dw, probe_ratio);
        const int64_t lt = (int64_t)t * lk;
        c_plain += (unsigned long long)(isT ? (lt < scan ? lt : scan)
                                             : ((int64_t)sbn * lk < scan ? (int64_t)sbn * lk : scan));
        uint32_t cdeg = 0;
        const bool cok = codeg_pair(S, rh, isT ? va : vb, &cdeg);
        uint32_t fl = 0;
        int32_t units = dw;
        int64_t cost = scan;
        if (!isT) {
          if (cok) {
            fl = kModeAux;
            units = 0;
            cost = 0;
            cyc_base += (long long)cdeg - 1;
          } else if ((int64_t)(bhub ? db : db - 1) * lk < scan) {
            fl = kModeLook;
            units = bhub ? db : db - 1;  // a hub's list is read from its row (a skipped)
            cost = (int64_t)units * lk;
          }
        } else {
          if (lt < scan) {
            fl = kModeLook;
            units = t;
            cost = lt;
          }
          if (cok) {
            cyc_base -= (long long)cdeg - 1;
          } else {
            fl |= kModeAux;
            units += L;  // Gamma(a) \ {b} is the w-list (x itself is never found)
            cost += (int64_t)L * lk;
          }
        }
        c_agg += (unsigned long long)cost;
        wl_v[i] = v | fl;
        wl_pref[i] = units;
      }
      c_plain = block_sum_u64<NT>(c_plain, red);
      c_agg = block_sum_u64<NT>(c_agg, red);
      // a hub edge has no S_b list for the plain scheme
      const bool agg = may_look && (bhub || c_agg < c_plain);
      if (!agg) {  // plain scheme: S_a members count |Gamma(w) n S_b|, T_e members degT
        cyc_base = 0;
        for (int i = tid; i < L; i += NT) {
          const uint32_t v = wl_v[i] & ~(kModeLook | kModeAux);
          const bool isT = (v & kTag) != 0;
          const int dw = deg_of(i);
          uint32_t fl = 0;
          int32_t units = dw;
          if (may_look) {
            const int64_t lk = look_cost(dw, probe_ratio);
            const int32_t src = isT ? t : sbn;
            if ((int64_t)src * lk < 8ll * dw) {
              fl = kModeLook;
              units = src;
            }
          }
          wl_v[i] = v | fl;
          wl_pref[i] = units;
        }
      }
      __syncthreads();
      const int32_t total = block_scan_lds<NT>(wl_pref, L, carry_sh);
      if (tid == 0) wl_pref[L] = total;
      __syncthreads();
      // flattened (w, unit) loop
      unsigned long long kt = 0, cs = (unsigned long long)cyc_base;
      int cur = 0;
      uint32_t steps = 0;
      for (int base = 0; base < total; base += NT) {
        const int idx = base + tid;
        if (idx < total) {
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
          const int32_t w = (int32_t)(v & kIdMask);
          if (!isT) {
            if (v & kModeLook) {  // look up Gamma(b) \ {a} (T_e, then S_b) for cbx, else S_b
              const int32_t x = bhub  ? col[bbeg + off]
                                : agg ? (off < t ? tgt[off] : tgt[CAP - sbn + (off - t)])
                                      : tgt[CAP - sbn + off];
              if (x != a && w_has(S, w, wl_beg[lo], deg_of(lo), x, &steps)) ++cs;
            } else {  // scan: cbx (any hit), or |Gamma(w) n S_b| without the aggregate form
              const int32_t r = col[wl_beg[lo] + off];
              ++steps;
              if (bhub) {
                if (r != a && table_find(btab, blg, (uint32_t)r) >= 0) ++cs;
              } else {
                const int sl = table_find(htab, lg, (uint32_t)r);
                if (sl >= 0 && (agg || !(htab[sl] & kTag))) ++cs;
              }
            }
          } else {
            const bool lt = (v & kModeLook) != 0;
            const int part1 = lt ? t : deg_of(lo);
            if (off < part1) {  // degT
              if (lt) {
                if (w_has(S, w, wl_beg[lo], deg_of(lo), tgt[off], &steps)) ++kt;
              } else {
                const int32_t r = col[wl_beg[lo] + off];
                ++steps;
                const int sl = table_find(htab, lg, (uint32_t)r);
                if (sl >= 0 && (htab[sl] & kTag)) ++kt;
              }
            } else {  // cax: look Gamma(a) \ {b} up in Gamma(x)
              const int32_t y = (int32_t)(wl_v[off - part1] & kIdMask);
              if (w_has(S, w, wl_beg[lo], deg_of(lo), y, &steps)) --cs;
            }
          }
        }
      }
      words += steps + (tid == 0 ? 2ull * (unsigned long long)L : 0ull);
      kt = block_sum_u64<NT>(kt, red);
      cs = block_sum_u64<NT>(cs, red);
      const unsigned long long cyc = agg ? cs + kt : cs;
      if (tid < kWave) acc.add(slots, slot, S.n, S.m, da, db, t, (int64_t)(kt / 2), (int64_t)cyc);
      if (tid == 0) micro_put(S, a, b, t, (int64_t)(kt / 2), (int64_t)cyc);
      __syncthreads();
    }
  }
  if (tid < kWave) acc.flush(slots);
  const unsigned long long wsum = block_sum_u64<NT>(words, red);
  if (tid == 0 && wsum) atomicAdd(words_out + (blockIdx.x % kXcds) * kLine, wsum);
}

// ---------------------------------------------------------------------------
// Global class: edges with an endpoint of degree > kHubDeg whose scan side has
// degree > kSmallScan (the others go to the wavefront kernel).  Work item =
// (edge, chunk of up to kGlobalChunkMax Gamma(a) positions).  Kernels:
//   prep     : items and T_e capacity per edge, partial sums cleared
//   classify : T_e of every edge into a global list (membership in Gamma(b)
//              by b's hub table or binary search)
//   count    : the per-w modes above over each chunk; per-edge partial sums
//              meet in GEdge and the item that completes an edge folds it
//              into its slot
// Tables in LDS per item: Gamma(b) \ {a} when b is not a hub, T_e when
// t <= kTHashCap (otherwise a's hub table serves).
// ---------------------------------------------------------------------------

constexpr int kGlobalNT = 512;  // counting kernel: one pass over a work item's positions
constexpr int kPrepNT = 256;    // classify and bit-set kernels
constexpr int kTHashCap = 512;
constexpr int kMaskWords = kGlobalChunkMax / 64;  // T_e membership words per work item
static_assert(kGlobalChunkMax % kGlobalNT == 0 && kGlobalChunkMax % kPrepNT == 0,
              "an item's positions take whole passes of the workgroups");

// Per split-class edge: counters (t by classify, nzw by the bit-set kernel,
// k4 / cyc summed by the counting items of edges with several) and the
// edge's descriptor, written once per launch so a work item finds
// everything in one 128-byte record.
struct GEdge {
  unsigned long long t, k4, cyc, spare, nzw;
  int32_t a, b, slot, da, db, abeg, bbeg, ra;  // ra / rb: ranks (-1 when unranked)
  int32_t rb, hra, hrb, pad;                   // hra / hrb: co-degree row (ranked) or row column (unranked), -1 none
  int64_t hoffa, hoffb;                        // hub-table offsets (-1 when no table)
  int64_t tbase, ipref, icnt;                  // T_e offset, first work item, work items
};
static_assert(sizeof(GEdge) == 128, "one GEdge per 128 bytes");

__global__ __launch_bounds__(256) void k_global_prep(const SlotDesc *__restrict__ slots,
                                                     const int32_t *__restrict__ bslot, const int32_t *__restrict__ ba,
                                                     const int32_t *__restrict__ bb,
                                                     const unsigned long long *__restrict__ ncount, int32_t chunk,
                                                     int64_t *items, int64_t *tcap, GEdge *gacc) {
  const int64_t nedges = (int64_t)*ncount;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t slot = bslot[e];
    const SlotDesc &S = slots[slot];
    const int32_t a = ba[e], b = bb[e];
    const int32_t abeg = S.row_ptr[a], bbeg = S.row_ptr[b];
    const int da = S.row_ptr[a + 1] - abeg;
    const int db = S.row_ptr[b + 1] - bbeg;
    const int4 va = S.vinfo[a], vb = S.vinfo[b];
    items[e] = (da + chunk - 1) / chunk;
    // room for T_e = Gamma(a) n Gamma(b): its exact size when the co-degree
    // table or rows hold the pair, else the smaller degree
    const uint32_t rha = va.z >= 0 ? (uint32_t)(va.z + 1) | ((uint32_t)(va.w + 1) << 17)
                                   : (0x80000000u | (uint32_t)(va.w + 1));
    uint32_t te;
    tcap[e] = codeg_pair(S, rha, vb, &te) ? (int64_t)te : (int64_t)(da < db ? da : db);
    GEdge &G = gacc[e];
    G.t = G.k4 = G.cyc = G.spare = G.nzw = 0ull;
    G.a = a;
    G.b = b;
    G.slot = slot;
    G.da = da;
    G.db = db;
    G.abeg = abeg;
    G.bbeg = bbeg;
    G.ra = va.z;
    G.rb = vb.z;
    G.hra = va.w;
    G.hrb = vb.w;
    G.pad = 0;
    // hub-table offsets of the sides too large for the LDS tables
    G.hoffa = da > kTableDeg ? S.hoff[a] : -1;
    G.hoffb = db > kTableDeg ? S.hoff[b] : -1;
  }
}

// the work item -> edge map: item_pref[e] .. item_pref[e] + items[e] - 1 -> e
__global__ __launch_bounds__(256) void k_item_fill(Bins bins, const int64_t *__restrict__ item_pref,
                                                   const int64_t *__restrict__ items,
                                                   const int64_t *__restrict__ tbase,
                                                   int32_t *__restrict__ item_edge, GEdge *gacc) {
  if (!split_fits(bins, bins.gtot[0], bins.gtot[1])) return;  // the host grows the buffers and runs again
  const int64_t nedges = (int64_t)bins.count[kClassGlobal];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = item_pref[e], k = items[e];
    for (int64_t i = 0; i < k; ++i) item_edge[b + i] = (int32_t)e;
    gacc[e].tbase = tbase[e];
    gacc[e].ipref = b;
    gacc[e].icnt = k;
  }
}

__global__ __launch_bounds__(kPrepNT) void k_global_classify(
    const SlotDesc *__restrict__ slots, Bins bins, const int64_t *__restrict__ item_pref,
    const int64_t *__restrict__ item_cnt, const int32_t *__restrict__ item_edge, int32_t *tlist,
    unsigned long long *__restrict__ tmask, GEdge *gacc, int32_t chunk, int32_t xcd_local) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t total_items = (int64_t)bins.gtot[0];
  if (!split_fits(bins, bins.gtot[0], bins.gtot[1])) return;
  // XCD-local mapping: the workgroups of XCD x = blockIdx % kXcds take
  // segment x of the items, so the items of one table-side endpoint b
  // (adjacent after the hub ordering) probe b's hub table through one L2
  int64_t first = blockIdx.x, hi = total_items, stride = gridDim.x;
  if (xcd_local && gridDim.x % kXcds == 0) {
    const int64_t sg = blockIdx.x % kXcds;
    first = total_items * sg / kXcds + blockIdx.x / kXcds;
    hi = total_items * (sg + 1) / kXcds;
    stride = gridDim.x / kXcds;
  }
  constexpr int kPass = kGlobalChunkMax / kPrepNT;  // passes over an item's positions
  constexpr int kNW = kPrepNT / kWave;
  __shared__ int wcnt[kNW];
  __shared__ unsigned long long sbase;
  const int wv = threadIdx.x >> 6;
  for (int64_t item = first; item < hi; item += stride) {
    // the edge's record (written by the preparation kernels)
    const int64_t e = item_edge[item];
    const GEdge &G = gacc[e];
    const SlotDesc &S = slots[G.slot];
    const int32_t *__restrict__ col = S.col;
    const int32_t b = G.b, abeg = G.abeg, bbeg = G.bbeg, da = G.da, db = G.db;
    const int64_t c = item - G.ipref, tb0 = G.tbase;
    const bool hb = has_table(db);
    const uint32_t *__restrict__ btab = hb ? S.htab + S.hoff[b] : nullptr;
    // a ranked b tests ranked x in its adjacency bit row (hcw words, shared
    // by the adjacent items of the same b), other x in b's table or list
    const unsigned long long *__restrict__ brow = G.rb >= 0 ? S.hbits + (int64_t)G.rb * S.hcw : nullptr;
    const int p0 = (int)(c * chunk);
    const int p1 = p0 + chunk < da ? p0 + chunk : da;
    // every read of the item's positions goes out before any is used
    int32_t xs[kPass];
    uint32_t rhs[kPass];
#pragma unroll
    for (int q = 0; q < kPass; ++q) {
      const int i = p0 + q * kPrepNT + (int)threadIdx.x;
      xs[q] = i < p1 ? col[abeg + i] : -1;
      rhs[q] = (i < p1 && brow) ? S.arh[abeg + i] : 0x80000000u;
    }
    bool ts[kPass];
#pragma unroll
    for (int q = 0; q < kPass; ++q) {
      const int32_t x = xs[q];
      ts[q] = false;
      if (x >= 0) {
        if (brow && !(rhs[q] >> 31)) {  // x ranked: its rank + 1 in the low bits
          const int32_t rx = (int32_t)(rhs[q] & 0x1FFFFu) - 1;
          ts[q] = ((brow[rx >> 6] >> (rx & 63)) & 1ull) != 0;
        } else if (x != b) {
          uint32_t st = 0;
          ts[q] = hb ? table_find(btab, table_log(db), (uint32_t)x) >= 0 : sorted_has(col + bbeg, db, x, &st);
        }
      }
    }
    // membership words for the counting items, and one claim of T_e slots
    // per item
    uint64_t tms[kPass];
    int wc = 0;
#pragma unroll
    for (int q = 0; q < kPass; ++q) {
      tms[q] = __ballot(ts[q]);
      wc += __popcll(tms[q]);
      if (lane == 0 && p0 + q * kPrepNT < p1) tmask[item * kMaskWords + q * kNW + wv] = tms[q];
    }
    if (lane == 0) wcnt[wv] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < kNW; ++w) tot += wcnt[w];
      sbase = tot ? atomicAdd(&gacc[e].t, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    int64_t pos = tb0 + (int64_t)sbase;
    for (int w = 0; w < wv; ++w) pos += wcnt[w];
#pragma unroll
    for (int q = 0; q < kPass; ++q) {
      if (ts[q]) {  // (id, degree, rank) triples; rank -1 when not ranked
        const int4 vi = S.vinfo[xs[q]];
        const int64_t at = pos + __popcll(tms[q] & lt_mask);
        tlist[3 * at] = xs[q];
        tlist[3 * at + 1] = vi.y;
        tlist[3 * at + 2] = vi.z;
      }
      pos += __popcll(tms[q]);
    }
    __syncthreads();  // wcnt and sbase are rewritten by the next item
  }
}

// The ranked members of every split-class edge's T_e as a bit set over the
// ranks, stored compactly (non-zero words and their indices, in increasing
// word order) at the edge's T_e offset; one workgroup per edge, once per
// launch.
__global__ __launch_bounds__(kPrepNT) void k_global_tbits(const SlotDesc *__restrict__ slots,
                                                            const int32_t *__restrict__ bslot, Bins bins,
                                                            const int64_t *__restrict__ tbase,
                                                            const int32_t *__restrict__ tlist, GEdge *gacc,
                                                            unsigned long long *__restrict__ tbw,
                                                            int16_t *__restrict__ tbi) {
  if (!split_fits(bins, bins.gtot[0], bins.gtot[1])) return;
  const int64_t nedges = (int64_t)bins.count[kClassGlobal];
  __shared__ unsigned long long bits[kBitsWords];
  __shared__ int wcnt[kPrepNT / kWave];
  const int lane = threadIdx.x & 63;
  const int wv_id = threadIdx.x >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int64_t e = blockIdx.x; e < nedges; e += gridDim.x) {
    const SlotDesc &S = slots[bslot[e]];
    const int hcw = S.hc > 0 ? (int)S.hcw : 0;
    const int t = (int)gacc[e].t;
    if (hcw == 0 || t == 0) continue;  // uniform per block; nzw stays 0
    for (int i = threadIdx.x; i < hcw; i += kPrepNT) bits[i] = 0ull;
    __syncthreads();
    const int32_t *T = tlist + 3 * tbase[e];
    for (int i = threadIdx.x; i < t; i += kPrepNT) {
      const int32_t r = T[3 * i + 2];
      if (r >= 0) atomicOr(&bits[r >> 6], 1ull << (r & 63));
    }
    __syncthreads();
    int cnt = 0;  // non-zero words so far (uniform)
    for (int i0 = 0; i0 < hcw; i0 += kPrepNT) {
      const int i = i0 + (int)threadIdx.x;
      const unsigned long long wv = i < hcw ? bits[i] : 0ull;
      const uint64_t m = __ballot(wv != 0ull);
      if (lane == 0) wcnt[wv_id] = __popcll(m);
      __syncthreads();
      int off = cnt, tot = 0;
      for (int q = 0; q < kPrepNT / kWave; ++q) {
        if (q < wv_id) off += wcnt[q];
        tot += wcnt[q];
      }
      if (wv) {
        const int k = off + __popcll(m & lt_mask);
        tbw[tbase[e] + k] = wv;
        tbi[tbase[e] + k] = (int16_t)i;
      }
      cnt += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) gacc[e].nzw = (unsigned long long)cnt;
  }
}

// Split-class counting in aggregate form.  With
//   cbx(w) = |Gamma(w) n (Gamma(b) \ {a})|   for w in S_a,
//   cax(x) = |Gamma(x) n (Gamma(a) \ {b})|   for x in T_e,
//   degT(x) = |Gamma(x) n T_e|              for x in T_e,
// the edges between S_a and S_b number
//   cyc = sum_{w in S_a} cbx(w) - sum_{x in T_e} cax(x) + sum_{x in T_e} degT(x)
// (each w in S_a is adjacent to a, and a's other neighbours split into T_e and
// S_a), and the edges inside T_e number k4 = sum degT / 2.  cbx and cax are
// pair co-degrees: one read when tabulated (both ranked: the co-degree table;
// one unranked: the other's co-degree row).  Per vertex the kernel picks the
// cheapest way to get its terms:
//   w in S_a : codeg(w,b) - 1 | walk Gamma(w) testing Gamma(b) | look Gamma(b) up in Gamma(w)
//   x in T_e : degT from the bit rows (ranked x: its ranked partners above
//              its rank, weight 2), by walking Gamma(x) against T_e or by
//              looking T_e up in Gamma(x); cax from the tables, or by walking
//              Gamma(x) against Gamma(a), or by looking Gamma(a) up in Gamma(x)
// A pair of unranked T_e members that both look up is tested once, by the one
// of smaller id, with weight 2, and an unranked member counts a ranked
// partner with weight 2 (the choices depend only on (d_x, t) and the edge's
// bit-set size, so every workgroup of the edge agrees on them).  Costs are in
// quarter units of one coalesced load.
__device__ __forceinline__ int64_t lookup_cost(int dw) {
  return has_table(dw) ? 16 : 8ll * (ceil_log2((uint32_t)dw + 1u) + 1);
}

__device__ __forceinline__ bool t_looks(int dx, int t, int64_t mT, int probe_ratio) {
  if (probe_ratio <= 0) return false;
  return (int64_t)t * (((4 + lookup_cost(dx)) * probe_ratio) / 4) < (int64_t)dx * (4 + mT);
}

constexpr uint8_t kFLookT = 1;   // degT by look-ups of T_e
constexpr uint8_t kFLookA = 2;   // cax by look-ups of Gamma(a)
constexpr uint8_t kFCodeg = 4;   // co-degree from the table
constexpr uint8_t kFLookB = 8;   // w in S_a: cbx by look-ups of Gamma(b)
constexpr uint8_t kFBits = 16;   // ranked w in T_e: degT over ranked members from bit rows
constexpr uint32_t kRTag = 0x40000000u;  // T_e hash key tag: member is ranked
// words of an edge's ranked-member set held in LDS (larger sets are read
// from the global lists): 10 KB, which keeps four workgroups per CU
constexpr int kBitsLds = 1024;

__global__ __launch_bounds__(kGlobalNT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_count_global(
    const SlotDesc *__restrict__ slots, Bins bins, const int64_t *__restrict__ item_pref,
    const int64_t *__restrict__ item_cnt, const int32_t *__restrict__ item_edge, const int32_t *__restrict__ tlist, const unsigned long long *__restrict__ tbw, const int16_t *__restrict__ tbi,
    const unsigned long long *__restrict__ tmask, GEdge *gacc,
    unsigned long long *cursor, unsigned long long *xcd_cursor, unsigned long long *words_out, int32_t probe_ratio,
    int32_t chunk, uint32_t flags) {
  constexpr int NT = kGlobalNT;
  constexpr int CH = kGlobalChunkMax;
  constexpr int HB = 2 * kTableDeg;
  constexpr int HT = 2 * kTHashCap;
  __shared__ uint32_t hA[HB];
  __shared__ uint32_t hB[HB];
  __shared__ uint32_t hT[HT];
  __shared__ uint32_t wl_v[CH];
  __shared__ uint8_t wl_f[CH];
  __shared__ int32_t wl_beg[CH];
  __shared__ int32_t wl_deg[CH];
  __shared__ int32_t wl_pref[CH + 1];
  __shared__ int32_t sh_cnt[4];
  __shared__ int32_t carry_sh[NT / kWave + 1];
  __shared__ unsigned long long red[2 * NT / kWave];
  __shared__ long long sh_item;
  __shared__ unsigned long long tbits[kBitsLds];  // non-zero words of the ranked members of T_e
  __shared__ int16_t twidx[kBitsLds];            // and their indices
  __shared__ int32_t bx_rank[CH];  // ranked members of T_e in this chunk

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (!split_fits(bins, bins.gtot[0], bins.gtot[1])) return;  // uniform
  unsigned long long words = 0;
  SlotAcc acc;
  acc.init();
  const int64_t total_items = (int64_t)bins.gtot[0];
  // XCD-local queue: workgroups of XCD x = blockIdx % kXcds drain segment x
  // of the item range first, then the following segments
  const bool xcd_local = (flags & kOptXcdLocal) != 0;
  const int my_seg = (int)(blockIdx.x % kXcds);
  int seg_off = 0;
  // the next work item (-1: none left); thread 0 asks for item k+1 while the
  // workgroup counts item k
  auto next_item = [&]() -> long long {
    if (!xcd_local) {
      const long long it = (long long)atomicAdd(cursor, 1ull);
      return it < total_items ? it : -1;
    }
    while (seg_off < kXcds) {
      const int sg = (my_seg + seg_off) % kXcds;
      const int64_t lo = total_items * sg / kXcds, hi = total_items * (sg + 1) / kXcds;
      const long long k = (long long)atomicAdd(&xcd_cursor[sg * kLine], 1ull);
      if (lo + k < hi) return lo + k;
      ++seg_off;
    }
    return -1;
  };
  if (tid == 0) sh_item = next_item();
  __syncthreads();

  for (;;) {
    const int64_t item = sh_item;
    __syncthreads();
    if (item < 0) break;
    long long upcoming = -1;
    if (tid == 0) upcoming = next_item();
    const int64_t e = item_edge[item];
    const GEdge &G = gacc[e];
    const int32_t a = G.a, b = G.b, slot = G.slot, da = G.da, db = G.db, abeg = G.abeg, bbeg = G.bbeg;
    const int32_t ra = G.ra, rb = G.rb, hra = G.hra, hrb = G.hrb;
    const int64_t hoffa = G.hoffa, hoffb = G.hoffb, tb0 = G.tbase, icnt = G.icnt;
    const int64_t c = item - G.ipref;
    const int t = (int)G.t;
    const SlotDesc &S = slots[slot];
    const int32_t *__restrict__ col = S.col;
    const bool ha = hoffa >= 0, hb = hoffb >= 0;
    static_assert(2 * kTableDeg <= (1 << 9), "LDS tables of the split kernel hold degree <= kTableDeg");
    const int blg = table_log(db), alg = table_log(da);
    const uint32_t *__restrict__ btab = hb ? S.htab + hoffb : hB;
    const uint32_t *__restrict__ atab = ha ? S.htab + hoffa : hA;
    const int32_t *__restrict__ T = tlist + 3 * tb0;  // (id, degree, rank) triples
    const bool tl = t <= kTHashCap;
    const int tlg = table_log(t);
    const int hcw = S.hc > 0 ? (int)S.hcw : 0;  // 0: no ranked vertices, no bit rows
    // every edge of a graph with ranked vertices counts its ranked pairs
    // from the bit rows; the ranked-member set is copied to LDS when it has
    // at most kBitsLds non-zero words, larger sets are read from the global
    // lists the bit-set kernel wrote
    const bool ubits = hcw > 0;
    const int nzw = ubits ? (int)G.nzw : 0;
    const bool bits_lds = nzw <= kBitsLds;
    const int nzw_lds = bits_lds ? nzw : 0;
    if (tid < 4) sh_cnt[tid] = 0;
    if (!hb)
      for (int i = tid; i < (1 << blg); i += NT) hB[i] = kEmpty;
    if (!ha)
      for (int i = tid; i < (1 << alg); i += NT) hA[i] = kEmpty;
    if (tl)
      for (int i = tid; i < (1 << tlg); i += NT) hT[i] = kEmpty;
    __syncthreads();
    {  // the LDS tables: Gamma(b) \ {a}, Gamma(a) \ {b} (non-hub sides), T_e (small)
      const int nB = hb ? 0 : db, nA = ha ? 0 : da, nT = tl ? t : 0;
      int nmax = nB > nA ? (nB > nT ? nB : nT) : (nA > nT ? nA : nT);
      nmax = nmax > nzw_lds ? nmax : nzw_lds;
      for (int i = tid; i < nmax; i += NT) {  // all loads first, then the LDS writes
        const int32_t xb = i < nB ? col[bbeg + i] : -1;
        const int32_t xa = i < nA ? col[abeg + i] : -1;
        const int32_t ty = i < nT ? T[3 * i] : -1;
        const int32_t tr = i < nT ? T[3 * i + 2] : -1;
        const unsigned long long bw = i < nzw_lds ? tbw[tb0 + i] : 0ull;
        const int16_t bi = i < nzw_lds ? tbi[tb0 + i] : (int16_t)0;
        if (i < nzw_lds) {
          tbits[i] = bw;
          twidx[i] = bi;
        }
        if (xb >= 0 && xb != a) lds_insert(hB, blg, (uint32_t)xb);
        if (xa >= 0 && xa != b) lds_insert(hA, alg, (uint32_t)xa);
        if (ty >= 0) lds_insert(hT, tlg, (uint32_t)ty | (ubits && tr >= 0 ? kRTag : 0u));
      }
      if (tid == 0) words += (unsigned long long)(nB + nA + 2 * nT + 3 * nzw_lds + 32);  // per-item terms once
    }
    __syncthreads();
    // r in Gamma(b) \ {a}; r in Gamma(a) \ {b}; r in T_e (the LDS tables
    // exclude a and b already, the hub tables do not)
    auto inBx = [&](uint32_t r) -> bool { return r != (uint32_t)a && table_find(btab, blg, r) >= 0; };
    auto inAx = [&](uint32_t r) -> bool { return r != (uint32_t)b && table_find(atab, alg, r) >= 0; };
    // 0: r not in T_e; 1: unranked member; 2: ranked member.  The weight is
    // the pair's share of the edges inside T_e counted from this side: a
    // ranked member counts only its ranked partners (bit rows), so the
    // unranked side counts a mixed pair twice.
    auto tmemb = [&](uint32_t r) -> int {
      if (tl) {
        const int sl = table_find(hT, tlg, r);
        return sl < 0 ? 0 : ((hT[sl] & kRTag) ? 2 : 1);
      }
      if (table_find(atab, alg, r) < 0 || table_find(btab, blg, r) < 0) return 0;
      return (ubits && S.crank[r] >= 0) ? 2 : 1;
    };
    const int64_t mB = hb ? 16 : 4, mA = ha ? 16 : 4, mT = tl ? 4 : 32;
    // this chunk's vertices w of Gamma(a) \ {b}, each with its mode: the loads
    // that depend only on w (row, rank, membership in Gamma(b)) go out
    // together, then the co-degree read
    const int p0 = (int)(c * chunk);
    const int p1 = p0 + chunk < da ? p0 + chunk : da;
    long long cyc_base = 0;
    const bool may_look = probe_ratio > 0;
    for (int base = p0; base < p1; base += NT) {
      const int i = base + tid;
      bool valid = i < p1;
      const int32_t x = valid ? col[abeg + i] : -1;
      valid = valid && x != b;
      int32_t wb = 0, dw = 0, rw = -1, hw = -1;
      bool isT = false;
      if (valid) {
        // rank and co-degree row (ranked) or row column (unranked): the arc's
        // packed word, read coalesced beside Gamma(a)
        const uint32_t rh = S.arh[abeg + i];
        if (rh >> 31) {
          hw = (int32_t)(rh & 0x7FFFFFFFu) - 1;
        } else {
          rw = (int32_t)(rh & 0x1FFFFu) - 1;
          hw = (int32_t)(rh >> 17) - 1;
        }
        // x in Gamma(a) is in T_e iff in Gamma(b): the classify pass's bit
        isT = ((tmask[item * kMaskWords + ((i - p0) >> 6)] >> ((i - p0) & 63)) & 1ull) != 0;
      }
      // |Gamma(x) n Gamma(y)|, y = a for T_e members, b otherwise: the table
      // for ranked pairs; a ranked end's co-degree row at the unranked end's
      // column
      int tab = 0;
      const int32_t ry = isT ? ra : rb, hy = isT ? hra : hrb;
      if (valid && may_look && hcw) {
        tab = (rw >= 0 && ry >= 0 && (rw < S.codeg_sat || ry < S.codeg_sat)) ? 1
              : (rw < 0 && hw >= 0 && ry >= 0 && hy >= 0) ? 2
              : (ry < 0 && hy >= 0 && rw >= 0 && hw >= 0) ? 3
                                                          : 0;
      }
      // row start and degree unless x has no units: a tabulated S_a member,
      // or a tabulated T_e member whose degT comes from the bit rows; issued
      // together with the co-degree read
      if (valid && (tab == 0 || (isT && !(ubits && rw >= 0)))) {
        const int4 vi = S.vinfo[x];
        wb = vi.x;
        dw = vi.y;
      }
      uint32_t cdeg = 0;
      if (tab == 1) cdeg = S.codeg[(int64_t)ry * S.hc + rw];  // symmetric: the fixed end's row
      else if (tab == 2) cdeg = row_at(S, hy, hw);
      else if (tab == 3) cdeg = row_at(S, hw, hy);
      const bool cok = tab != 0;
      uint8_t fl = 0;
      int32_t units = 0;
      if (valid) {
        const int64_t look = may_look ? ((4 + lookup_cost(dw)) * probe_ratio) / 4 : 0;
        if (!isT) {
          if (cok) {
            fl = kFCodeg;
            cyc_base += (long long)cdeg - 1;
          } else if (may_look && (int64_t)db * look < (int64_t)dw * (4 + mB)) {
            fl = kFLookB;
            units = db;
          } else {
            units = dw;
          }
        } else {
          const bool bits = ubits && rw >= 0;
          const bool lt = !bits && t_looks(dw, t, mT, probe_ratio);
          if (lt) fl |= kFLookT;
          if (bits) {  // degT over ranked partners in the bit-row phase below
            fl |= kFBits;
            bx_rank[atomicAdd(&sh_cnt[2], 1)] = rw;
          }
          const int part1 = bits ? 0 : (lt ? t : dw);
          if (cok) {
            fl |= kFCodeg;
            cyc_base -= (long long)cdeg - 1;
            units = part1;
          } else {
            const bool la = may_look && (int64_t)da * look < (int64_t)dw * (4 + mA);
            if (la) fl |= kFLookA;
            // one walk of Gamma(w) serves both terms when nothing else is used
            units = (!bits && !lt && !la) ? dw : part1 + (la ? da : dw);
          }
        }
      }
      const uint64_t vm = __ballot(valid);
      int pos0 = 0;
      if (lane == 0 && vm) pos0 = atomicAdd(&sh_cnt[0], __popcll(vm));
      pos0 = __shfl(pos0, 0);
      if (valid) {
        const int pos = pos0 + __popcll(vm & lt_mask);
        wl_v[pos] = (uint32_t)x | (isT ? kTag : 0u);
        wl_beg[pos] = wb;
        wl_deg[pos] = dw;
        wl_f[pos] = fl;
        wl_pref[pos] = units;
      }
    }
    if (tid == 0) words += (unsigned long long)(6 * (p1 - p0));
    __syncthreads();
    const int L = sh_cnt[0];
    __syncthreads();
    const int32_t total = block_scan_lds<NT>(wl_pref, L, carry_sh);
    if (tid == 0) wl_pref[L] = total;
    __syncthreads();
    unsigned long long kt = 0;                              // sum of degT over T_e members
    unsigned long long cs = (unsigned long long)cyc_base;  // sum cbx - sum cax (mod 2^64)
    uint32_t steps = 0;
    int cur = 0;
    for (int base = 0; base < total; base += NT) {
      const int idx = base + tid;
      if (idx < total) {
        int l2 = cur;
        if (wl_pref[l2 + 1] <= idx) {
          int h2 = L - 1;
          while (l2 < h2) {
            const int mid = (l2 + h2 + 1) >> 1;
            if (wl_pref[mid] <= idx)
              l2 = mid;
            else
              h2 = mid - 1;
          }
        }
        cur = l2;
        const uint32_t v = wl_v[l2];
        const uint8_t fl = wl_f[l2];
        const int off = idx - wl_pref[l2];
        const bool isT = (v & kTag) != 0;
        const int32_t w = (int32_t)(v & kIdMask);
        const int dw = wl_deg[l2];
        ++steps;
        if (!isT) {
          if (fl & kFLookB) {  // cbx by looking Gamma(b) up in Gamma(w)
            const int32_t x = col[bbeg + off];
            if (x != a && w_has(S, w, wl_beg[l2], dw, x, &steps)) ++cs;
          } else {  // cbx by walking Gamma(w)
            if (inBx((uint32_t)col[wl_beg[l2] + off])) ++cs;
          }
        } else {
          const bool lt = (fl & kFLookT) != 0;
          const bool bits = (fl & kFBits) != 0;
          const bool both = !(fl & (kFCodeg | kFLookT | kFLookA | kFBits));
          const int part1 = bits ? 0 : (lt ? t : dw);
          if (both) {  // one walk of Gamma(w): degT and cax
            const uint32_t r = (uint32_t)col[wl_beg[l2] + off];
            kt += (unsigned long long)tmemb(r);
            if (inAx(r)) --cs;
          } else if (off < part1) {  // degT
            if (lt) {
              const int32_t y = T[3 * off];
              const int dy = T[3 * off + 1];
              // ranked members count only ranked partners; pairs of unranked
              // look-up members are tested by the smaller id only
              const int wgt =
                  (ubits && T[3 * off + 2] >= 0) ? 2 : (t_looks(dy, t, mT, probe_ratio) ? (y > w ? 2 : 0) : 1);
              if (wgt && w_has(S, w, wl_beg[l2], dw, y, &steps)) kt += (unsigned long long)wgt;
            } else {
              kt += (unsigned long long)tmemb((uint32_t)col[wl_beg[l2] + off]);
            }
          } else {  // cax
            const int o2 = off - part1;
            if (fl & kFLookA) {
              const int32_t y = col[abeg + o2];
              if (y != b && w_has(S, w, wl_beg[l2], dw, y, &steps)) --cs;
            } else {
              if (inAx((uint32_t)col[wl_beg[l2] + o2])) --cs;
            }
          }
        }
      }
    }
    words += steps + (tid == 0 ? 2ull * (unsigned long long)L : 0ull);
    // bit-row phase: the edges between ranked members of T_e, each counted
    // once, from its lower-rank end x in this chunk, with weight 2: the
    // popcount of x's bit row AND the ranked-member set over the non-zero
    // words from x's own word on (bits above x's rank only).  Ranks grow
    // with degree, so the common high-degree members read few words.  The
    // (member, word) pairs are spread over the whole workgroup.
    __syncthreads();  // wl_pref and wl_beg are reused below
    if (sh_cnt[2] > 0 && nzw > 0) {  // uniform: skipped without ranked members in this chunk
      const int nb = sh_cnt[2];
      int32_t *const bk0 = wl_beg;   // first word index of member j
      int32_t *const bpref = wl_pref;  // pairs before member j
      // the set's word indices and words: the LDS copy, or the global lists
      const int16_t *__restrict__ gti = tbi + tb0;
      const unsigned long long *__restrict__ gtw = tbw + tb0;
      for (int j = tid; j < nb; j += NT) {
        const int wx = bx_rank[j] >> 6;
        int lo = 0, hi = nzw;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((bits_lds ? twidx[mid] : gti[mid]) < wx)
            lo = mid + 1;
          else
            hi = mid;
        }
        bk0[j] = lo;
        bpref[j] = nzw - lo;
      }
      __syncthreads();
      const int32_t P = block_scan_lds<NT>(bpref, nb, carry_sh);
      if (tid == 0) bpref[nb] = P;
      __syncthreads();
      unsigned long long bsum = 0;
      int jc = 0;
      for (int q = tid; q < P; q += NT) {
        int lo = jc;
        if (bpref[lo + 1] <= q) {
          int hi = nb - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bpref[mid] <= q)
              lo = mid;
            else
              hi = mid - 1;
          }
        }
        jc = lo;
        const int rx = bx_rank[jc];
        const int k = bk0[jc] + (q - bpref[jc]);
        const int wk = bits_lds ? twidx[k] : gti[k];
        unsigned long long v = S.hbits[(int64_t)rx * S.hcw + wk] & (bits_lds ? tbits[k] : gtw[k]);
        if (wk == (rx >> 6)) v &= (rx & 63) == 63 ? 0ull : (~0ull << ((rx & 63) + 1));
        bsum += (unsigned long long)__popcll(v);
        words += 2;
      }
      kt += 2ull * bsum;
    }
    block_sum2_u64<NT>(kt, cs, red);
    if (icnt == 1) {  // the edge's only item: no partial sums to meet
      if (tid < kWave) {
        // per-lane register sums, flushed into the slot when it changes
        acc.add(slots, slot, S.n, S.m, da, db, t, (int64_t)(kt / 2), (int64_t)(cs + kt));
        if (lane == 0) micro_put(S, a, b, t, (int64_t)(kt / 2), (int64_t)(cs + kt));
      }
    } else if (tid == 0) {  // partial sums; k_global_finish folds the edge
      GEdge *g = gacc + e;
      if (kt) atomicAdd(&g->k4, kt);
      if (cs) atomicAdd(&g->cyc, cs);
    }
    if (tid == 0) sh_item = upcoming;
    __syncthreads();
  }
  if (tid < kWave) acc.flush(slots);
  const unsigned long long wsum = block_sum_u64<NT>(words, red);
  if (tid == 0 && wsum) atomicAdd(words_out + (blockIdx.x % kXcds) * kLine, wsum);
}

// Edges counted by several work items: their items left k4 (twice the
// edges inside T_e) and the rest of cyc in the edge's counters; one
// wavefront per edge turns them into the edge's terms (Alg. 2) and folds
// them into its slot.
__global__ __launch_bounds__(256) void k_global_finish(const SlotDesc *__restrict__ slots, Bins bins,
                                                       const GEdge *__restrict__ gacc,
                                                       const int64_t *__restrict__ item_cnt) {
  if (!split_fits(bins, bins.gtot[0], bins.gtot[1])) return;
  const int64_t nedges = (int64_t)bins.count[kClassGlobal];
  SlotAcc acc;
  acc.init();
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  // 64 edges per wavefront and round: their item counts in one coalesced
  // read, then the multi-item ones one after another
  for (int64_t base = w0 * kWave; base < nedges; base += nw * kWave) {
    const int64_t e = base + lane;
    uint64_t m = __ballot(e < nedges && item_cnt[e] > 1);
    while (m) {  // uniform per wavefront
      const int k = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const GEdge &G = gacc[base + k];
      const SlotDesc &S = slots[G.slot];
      const unsigned long long kk = G.k4, cc = G.cyc + kk;
      acc.add(slots, G.slot, S.n, S.m, G.da, G.db, (int64_t)G.t, (int64_t)(kk / 2), (int64_t)cc);
      if (lane == 0) micro_put(S, G.a, G.b, (int64_t)G.t, (int64_t)(kk / 2), (int64_t)cc);
    }
  }
  acc.flush(slots);
}

// ---------------------------------------------------------------------------
// Micro-level statistics (Sec. 3, Alg. 7 with p_e = 1): for every edge of a
// range, the number of induced k-vertex subgraphs of each type G_i that hold
// both ends of the edge.  The searches that need the neighbourhoods of the
// neighbours (k4, cyc) come from the counting kernels above through
// micro_put; everything else follows from per-arc triangle counts:
//   tau_a   = sum over w in T_e of t(a, w)    (arcs a-w of the T_e members)
//   omega   = edges T_e - (S_a u S_b)        = tau_a + tau_b - 2t - 4 k4
//   e(S_a)  = edges inside S_a               = tri(a) - tau_a + k4
//   RT      = edges T_e - R                  = sum_T d_w - 2t - 2k4 - omega
//   RS      = edges (S_a u S_b) - R          = sum_S d_w - s - omega
//                                               - 2(e(S_a) + e(S_b)) - 2 cyc
//   e(R)    = edges inside R = f - (k4 + omega + e(S_a) + e(S_b) + cyc) - RT - RS
// with R the vertices adjacent to neither end, f the edges that share no end
// with e, tri(x) the triangles at x and sum_S d_w = vol2(a) + vol2(b)
// - d_a - d_b - 2 sum_T d_w.  The row then reads
//   G1 1, G3 t, G4 s, G5 r, G7 k4, G8 C(t,2) - k4 + omega,
//   G9 e(S_a) + e(S_b) + t s - omega + RT, G10 cyc,
//   G11 C(s_a,2) - e(S_a) + C(s_b,2) - e(S_b), G12 s_a s_b - cyc + RS,
//   G13 t r - RT, G14 s r - RS, G15 e(R), G16 C(r,2) - e(R), G2 = G6 = G17 = 0.
// ---------------------------------------------------------------------------

// first position in the sorted list a[0, len) holding a value >= x
__device__ __forceinline__ int row_lower(const int32_t *__restrict__ a, int len, int32_t x) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

constexpr int kMicroGroup = 16;  // lanes per edge
constexpr int kMicroUnroll = 4;  // positions a lane of the micro rows reads at a time

template <typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = kMicroGroup / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kMicroGroup);
  return v;
}

// t(u, v) of every edge, stored at both arcs
__global__ __launch_bounds__(256) void k_micro_arc_tri(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const uint64_t *__restrict__ edges,
                                                       const int64_t *__restrict__ hoff,
                                                       const uint32_t *__restrict__ htab, int64_t m,
                                                       int32_t *__restrict__ t_arc) {
  const int gl = threadIdx.x & (kMicroGroup - 1);
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kMicroGroup;
  const int64_t ng = ((int64_t)gridDim.x * blockDim.x) / kMicroGroup;
  for (int64_t e = g0; e < m; e += ng) {
    const uint64_t key = edges[e];
    const int32_t u = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
    const int32_t ub = rp[u], du = rp[u + 1] - ub, vb = rp[v], dv = rp[v + 1] - vb;
    const bool us = du <= dv;
    const int32_t abeg = us ? ub : vb, da = us ? du : dv, b = us ? v : u;
    const int32_t bbeg = us ? vb : ub, db = us ? dv : du;
    const bool hb = has_table(db);
    const uint32_t *btab = hb ? htab + hoff[b] : nullptr;
    const int blg = table_log(db);
    int cnt = 0;
    for (int i = gl; i < da; i += kMicroGroup) {
      const int32_t x = col[abeg + i];
      if (x == b) continue;
      bool in;
      if (hb) {
        in = table_find(btab, blg, (uint32_t)x) >= 0;
      } else {
        const int k = row_lower(col + bbeg, db, x);
        in = k < db && col[bbeg + k] == x;
      }
      cnt += in ? 1 : 0;
    }
    cnt = group_sum(cnt);
    if (gl == 0) {
      const int pu = row_lower(col + ub, du, v), pv = row_lower(col + vb, dv, u);
      if (pu < du) t_arc[ub + pu] = cnt;
      if (pv < dv) t_arc[vb + pv] = cnt;
    }
  }
}

// tri(x) = half the sum of t over the arcs of x; one wavefront per vertex
__global__ __launch_bounds__(256) void k_micro_vertex_tri(const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ t_arc, int64_t n,
                                                          int64_t *__restrict__ tri) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t x = w0; x < n; x += nw) {
    unsigned long long acc = 0;
    const int32_t end = rp[x + 1];
    for (int32_t j = rp[x] + lane; j < end; j += 64) acc += (unsigned long long)t_arc[j];
    acc = wave_sum_u64(acc);
    if (lane == 0) tri[x] = (int64_t)(acc / 2);
  }
}

// t of every arc (u, x) of a vertex u with a hub table, stored at x's slot
// of that table: the micro rows read t(b, x) with the membership test of x
// in Gamma(b) (one probe instead of a binary search for x's position)
__global__ __launch_bounds__(256) void k_micro_slot_tri(const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, int64_t n,
                                                        const int64_t *__restrict__ hoff,
                                                        const uint32_t *__restrict__ htab,
                                                        const int32_t *__restrict__ t_arc,
                                                        int32_t *__restrict__ t_slot) {
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
    const int d = end - beg;
    if (!has_table(d)) continue;  // uniform per block
    const int lg = table_log(d);
    const uint32_t *tab = htab + hoff[u];
    int32_t *ts = t_slot + hoff[u];
    for (int32_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
      const int sl = table_find(tab, lg, (uint32_t)col[j]);
      if (sl >= 0) ts[sl] = t_arc[j];
    }
  }
}

// sentinel -1 in the columns the counting kernels fill
__global__ __launch_bounds__(256) void k_micro_mark(long long *__restrict__ out, int64_t rows) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
    long long *row = out + r * kMicroCols;
    row[kMicroColT] = -1;
    row[kMicroColK4] = -1;
    row[kMicroColCyc] = -1;
  }
}

__device__ __forceinline__ long long micro_pick(int c, const long long *y) {
  long long v = 0;
#pragma unroll
  for (int i = 0; i < kMicroGroup; ++i)
    if (c == i) v = y[i];
  return v;
}

// the rows of edges [e0, e1); one group of kMicroGroup lanes per edge, lane c
// writes column c (lane 0 also column 16); column maxima reduced per block
__global__ __launch_bounds__(256) void k_micro_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const uint64_t *__restrict__ edges,
                                                   const int64_t *__restrict__ vol2,
                                                   const int64_t *__restrict__ hoff,
                                                   const uint32_t *__restrict__ htab,
                                                   const int32_t *__restrict__ t_slot,
                                                   const int4 *__restrict__ vinfo,
                                                   const int32_t *__restrict__ t_arc,
                                                   const int64_t *__restrict__ tri, int64_t n, int64_t m, int64_t e0,
                                                   int64_t e1, long long *__restrict__ out,
                                                   unsigned long long *__restrict__ colmax, int *__restrict__ err) {
  __shared__ unsigned long long smax[kMicroCols];
  if (threadIdx.x < kMicroCols) smax[threadIdx.x] = 0;
  __syncthreads();
  const int gl = threadIdx.x & (kMicroGroup - 1);
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kMicroGroup;
  const int64_t ng = ((int64_t)gridDim.x * blockDim.x) / kMicroGroup;
  unsigned long long mx = 0;
  for (int64_t e = e0 + g0; e < e1; e += ng) {
    const uint64_t key = edges[e];
    const int32_t u = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
    const int32_t ub = rp[u], du = rp[u + 1] - ub, vb = rp[v], dv = rp[v + 1] - vb;
    const bool us = du <= dv;
    const int32_t a = us ? u : v, b = us ? v : u;
    const int32_t abeg = us ? ub : vb, da = us ? du : dv;
    const int32_t bbeg = us ? vb : ub, db = us ? dv : du;
    // x in Gamma(a) n Gamma(b) with t(a, x), t(b, x) and d_x: b's hub table
    // and the t stored at its slots, else a binary search of b's list.  A
    // lane takes kMicroUnroll positions at a time, each step's reads of all
    // of them in flight together (positions, first probes, then t and the
    // degrees)
    const bool hb = has_table(db);
    const uint32_t *btab = hb ? htab + hoff[b] : nullptr;
    const int32_t *bts = hb ? t_slot + hoff[b] : nullptr;
    const int blg = table_log(db);
    const uint32_t bmask = (1u << blg) - 1u;
    long long st = 0, sdt = 0, ta = 0, tb = 0;
    for (int i0 = gl; i0 < da; i0 += kMicroUnroll * kMicroGroup) {
      int32_t xs[kMicroUnroll], tas[kMicroUnroll], tbx[kMicroUnroll];
#pragma unroll
      for (int u = 0; u < kMicroUnroll; ++u) {
        const int i = i0 + u * kMicroGroup;
        const int32_t x = i < da ? col[abeg + i] : -1;
        xs[u] = x == b ? -1 : x;
        tas[u] = i < da ? t_arc[abeg + i] : 0;
      }
      if (hb) {
        uint32_t h[kMicroUnroll], k[kMicroUnroll];
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u) {
          h[u] = xs[u] >= 0 ? hash_slot((uint32_t)xs[u], blg) : 0u;
          k[u] = xs[u] >= 0 ? btab[h[u]] : kEmpty;
        }
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u) {
          while (k[u] != kEmpty && (k[u] & kIdMask) != (uint32_t)xs[u]) {  // linear probing
            h[u] = (h[u] + 1u) & bmask;
            k[u] = btab[h[u]];
          }
          tbx[u] = k[u] != kEmpty ? bts[h[u]] : -1;
        }
      } else {
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u) {
          tbx[u] = -1;
          if (xs[u] >= 0) {
            const int kk = row_lower(col + bbeg, db, xs[u]);
            if (kk < db && col[bbeg + kk] == xs[u]) tbx[u] = t_arc[bbeg + kk];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kMicroUnroll; ++u) {
        if (tbx[u] >= 0) {
          st += 1;
          sdt += vinfo[xs[u]].y;
          ta += tas[u];
          tb += tbx[u];
        }
      }
    }
    st = group_sum(st);
    sdt = group_sum(sdt);
    ta = group_sum(ta);
    tb = group_sum(tb);
    long long *row = out + (e - e0) * kMicroCols;
    const long long t = row[kMicroColT], k4 = row[kMicroColK4], cyc = row[kMicroColCyc];
    if (t != st || k4 < 0 || cyc < 0) {  // the counting pass missed this edge
      if (gl == 0) atomicOr(err, 1);
      continue;
    }
    const long long DA = da, DB = db;
    const long long sa = DA - 1 - t, sb = DB - 1 - t, s = sa + sb;
    const long long r = (long long)n - DA - DB + t;
    const long long f = (long long)m - DA - DB + 1;
    const long long omega = ta + tb - 2 * t - 4 * k4;
    const long long esa = tri[a] - ta + k4, esb = tri[b] - tb + k4;
    const long long rt = sdt - 2 * t - 2 * k4 - omega;
    const long long sds = vol2[a] + vol2[b] - DA - DB - 2 * sdt;
    const long long rs = sds - s - omega - 2 * (esa + esb) - 2 * cyc;
    const long long er = f - (k4 + omega + esa + esb + cyc) - rt - rs;
    long long y[kMicroGroup];
    y[0] = 1;
    y[1] = 0;
    y[2] = t;
    y[3] = s;
    y[4] = r;
    y[5] = 0;
    y[6] = k4;
    y[7] = t * (t - 1) / 2 - k4 + omega;
    y[8] = esa + esb + t * s - omega + rt;
    y[9] = cyc;
    y[10] = sa * (sa - 1) / 2 - esa + sb * (sb - 1) / 2 - esb;
    y[11] = sa * sb - cyc + rs;
    y[12] = t * r - rt;
    y[13] = s * r - rs;
    y[14] = er;
    y[15] = r * (r - 1) / 2 - er;
    const long long val = micro_pick(gl, y);
    row[gl] = val;
    mx = (unsigned long long)val > mx ? (unsigned long long)val : mx;
    if (gl == 0) row[16] = 0;  // G17: no independent set holds an edge
  }
  atomicMax(&smax[gl], mx);  // column 16 (G17) stays 0
  __syncthreads();
  if (threadIdx.x < kMicroCols && smax[threadIdx.x]) atomicMax(colmax + threadIdx.x, smax[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// k-core numbers by level-synchronous peeling (once per graph), edge weight
// classes, and the radix select of fixed-size samples
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_core_init(const int32_t *__restrict__ rp, int64_t n, int32_t *deg,
                                                   int32_t *state) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    deg[v] = rp[v + 1] - rp[v];
    state[v] = 0;
  }
}

__global__ __launch_bounds__(256) void k_core_scan(int64_t n, int32_t k, int32_t *deg, int32_t *state,
                                                   int32_t *front, unsigned long long *cnt,
                                                   unsigned long long *minalive) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long mn = ~0ull;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = base + threadIdx.x;
    bool push = false;
    if (v < n && state[v] == 0) {
      const int32_t d = deg[v];
      if (d <= k) {
        push = true;
        state[v] = 2;
      } else if ((unsigned long long)d < mn) {
        mn = (unsigned long long)d;
      }
    }
    const uint64_t pm = __ballot(push);
    unsigned long long pos0 = 0;
    if (lane == 0 && pm) pos0 = atomicAdd(cnt, (unsigned long long)__popcll(pm));
    pos0 = __shfl(pos0, 0);
    if (push) front[pos0 + __popcll(pm & lt_mask)] = (int32_t)v;
  }
  if (mn != ~0ull) atomicMin(minalive, mn);
}

__global__ __launch_bounds__(256) void k_core_peel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ front, int64_t fn, int32_t k,
                                                   int32_t *deg, int32_t *state, int32_t *core, int32_t *next,
                                                   unsigned long long *ncnt) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < fn; i += nw) {
    const int32_t v = front[i];
    const int32_t beg = rp[v], end = rp[v + 1];
    for (int32_t j = beg + lane; j < end; j += 64) {
      const int32_t w = col[j];
      if (__atomic_load_n(&state[w], __ATOMIC_RELAXED) != 0) continue;
      const int32_t old = atomicSub(&deg[w], 1);
      if (old == k + 1) {  // w just reached degree k: it belongs to this level
        state[w] = 2;
        next[atomicAdd(ncnt, 1ull)] = w;
      }
    }
    if (lane == 0) {
      core[v] = k;
      state[v] = 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_weight_levels(int32_t mode, const int32_t *__restrict__ rp,
                                                       const uint64_t *__restrict__ edges,
                                                       const int32_t *__restrict__ core, int64_t m,
                                                       uint8_t *__restrict__ level,
                                                       unsigned long long *__restrict__ hist) {
  __shared__ unsigned long long sh[kWeightLevels];
  if (threadIdx.x < kWeightLevels) sh[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = edges[e];
    const int32_t u = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
    int64_t w;
    if (mode == 1) {
      w = (int64_t)(rp[u + 1] - rp[u]) + (int64_t)(rp[v + 1] - rp[v]) - 2;
    } else {
      const int32_t cu = core[u], cv = core[v];
      w = cu < cv ? cu : cv;
    }
    int l = 0;
    if (w >= 2) l = 63 - __clzll((unsigned long long)w);
    if (l > kWeightLevels - 1) l = kWeightLevels - 1;
    level[e] = (uint8_t)l;
    atomicAdd(&sh[l], 1ull);
  }
  __syncthreads();
  if (threadIdx.x < kWeightLevels && sh[threadIdx.x]) atomicAdd(hist + threadIdx.x, sh[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_select_hist(uint64_t seed, int64_t m, int32_t shift, uint64_t pre_hi,
                                                     uint64_t pre_lo, unsigned long long *hist) {
  __shared__ unsigned long long sh[256];
  sh[threadIdx.x] = 0;
  __syncthreads();
  const int top = shift + 8;  // bits [top, 128) must match the prefix
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t hi = philox_bits(seed, (uint64_t)e), lo = (uint64_t)e;
    bool match;
    if (top >= 128) {
      match = true;
    } else if (top >= 64) {
      match = (hi >> (top - 64)) == pre_hi;
    } else {
      match = hi == pre_hi && (top == 0 || (lo >> top) == pre_lo);
    }
    if (!match) continue;
    const uint32_t dig = shift >= 64 ? (uint32_t)((hi >> (shift - 64)) & 0xFFu) : (uint32_t)((lo >> shift) & 0xFFu);
    atomicAdd(&sh[dig], 1ull);
  }
  __syncthreads();
  if (sh[threadIdx.x]) atomicAdd(hist + threadIdx.x, sh[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Ordering of the split class by table-side endpoint (counting sort)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int sort_key(const SlotDesc &S, int32_t b) {
  if (S.hc <= 0) return kSortKeys - 1;
  const int32_t r = S.crank[b];  // < kMaxRanked
  return r >= 0 ? r : kSortKeys - 1;
}

__global__ __launch_bounds__(256) void k_sort_hist(const SlotDesc *__restrict__ slots,
                                                   const int32_t *__restrict__ bslot, const int32_t *__restrict__ bb,
                                                   const unsigned long long *__restrict__ ncount, int64_t *hist) {
  const int64_t n = (int64_t)*ncount;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long *)&hist[sort_key(slots[bslot[e]], bb[e])], 1ull);
}

__global__ __launch_bounds__(256) void k_sort_scatter(const SlotDesc *__restrict__ slots,
                                                      const int32_t *__restrict__ bslot,
                                                      const int32_t *__restrict__ ba, const int32_t *__restrict__ bb,
                                                      const unsigned long long *__restrict__ ncount, int64_t *off,
                                                      int32_t *slot2, int32_t *a2, int32_t *b2) {
  const int64_t n = (int64_t)*ncount;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t sl = bslot[e], b = bb[e];
    const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&off[sort_key(slots[sl], b)], 1ull);
    slot2[pos] = sl;
    a2[pos] = ba[e];
    b2[pos] = b;
  }
}

__global__ void k_zero_u64(unsigned long long *p, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// a one-job sequence's start: the counters and accumulators cleared and the
// job's range and slot descriptors, passed by value, stored where the
// kernels read them (one launch in place of a copy and a clear)
__global__ void k_seq_init(unsigned long long *p, int64_t len, RangeDesc *rdst, SlotDesc *sdst, RangeDesc r,
                           SlotDesc sd) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *rdst = r;
    *sdst = sd;
  }
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

hipError_t launch_graph_validate(const int32_t *row_ptr, const int32_t *col, int64_t n, int *err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_validate, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, n, err);
  return hipGetLastError();
}

hipError_t launch_graph_upper(const int32_t *row_ptr, const int32_t *col, int64_t n, int32_t *up_start,
                              int64_t *cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_upper, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, row_ptr, col, n, up_start, cnt);
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

hipError_t launch_scan_dev(const int64_t *in, int64_t *out, const unsigned long long *len, int64_t cap, int64_t *tmp,
                           unsigned long long *total, hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  const int grid = grid_for(cap, kScanBlock, 2048);
  hipLaunchKernelGGL(k_scan_dev_blocks, dim3(grid), dim3(256), 0, s, in, out, len, tmp);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_scan_dev_sums, dim3(1), dim3(256), 0, s, tmp, len, total);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_scan_dev_add, dim3(grid), dim3(256), 0, s, out, len, (const int64_t *)tmp);
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
  hipLaunchKernelGGL(k_graph_edges, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, up_start, eid_base,
                     n, edges);
  return hipGetLastError();
}

hipError_t launch_graph_vol2(const int32_t *row_ptr, const int32_t *col, int64_t n, int64_t *vol2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_vol2, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, n, vol2);
  return hipGetLastError();
}

hipError_t launch_graph_work(const int32_t *row_ptr, const uint64_t *edges, const int64_t *vol2, int64_t m,
                             unsigned long long *blocks, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_work, dim3(grid_for((m + kWorkBlock - 1) / kWorkBlock, 4, 8192)), dim3(256), 0, s,
                     row_ptr, edges, vol2, m, blocks);
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

hipError_t launch_codeg_count(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n,
                              int64_t *cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codeg_count, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, crank, n, cnt);
  return hipGetLastError();
}

hipError_t launch_codeg_fill(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n,
                             const int64_t *off, const int64_t *cnt, int32_t *list, int32_t *nlo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codeg_fill, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, col, crank, n, off, cnt,
                     list, nlo);
  return hipGetLastError();
}

hipError_t launch_codeg_rows(const int32_t *row_ptr, const int32_t *col, const int32_t *ranked, const int64_t *off,
                             const int64_t *cnt, const int32_t *list, const int32_t *nlo, int64_t hc, uint16_t *tab,
                             hipStream_t s) {
  if (hc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codeg_rows, dim3((unsigned)hc), dim3(kRowNT), 0, s, row_ptr, col, ranked, off, cnt, list, nlo,
                     hc, tab);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t len, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(len, 256, 4096)), dim3(256), 0, s, p, len);
  return hipGetLastError();
}

hipError_t launch_seq_init(unsigned long long *p, int64_t len, RangeDesc *rdst, SlotDesc *sdst, const RangeDesc &r,
                           const SlotDesc &sd, hipStream_t s) {
  hipLaunchKernelGGL(k_seq_init, dim3(grid_for(len, 256, 4096)), dim3(256), 0, s, p, len, rdst, sdst, r, sd);
  return hipGetLastError();
}

hipError_t launch_sample_bin(const SlotDesc *slots, const RangeDesc *ranges, int32_t nranges, int64_t total,
                             Bins bins, KernelCfg cfg, hipStream_t s) {
  if (total <= 0 || nranges <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_bin, dim3(grid_for(total, 256 * kSamplePer, cfg.grid_sample)), dim3(256), 0, s, slots, ranges,
                     nranges, total, bins, cfg);
  return hipGetLastError();
}

template <int NT, int CAP>
static hipError_t launch_lds(const SlotDesc *slots, Bins bins, int cls, int64_t bound, int grid_cap,
                             int32_t probe_ratio, hipStream_t s) {
  // the wavefront class claims runs of up to 64 edges and lets 16
  // workgroups per XCD take from the other queues; the workgroup class,
  // whose edges are heavy and fewer, claims single edges and lets every
  // workgroup take from every queue
  const int max_chunk = NT == kWave ? 64 : 1;
  const int stealers = NT == kWave ? kLdsStealers : (1 << 30);
  int grid = grid_for(bound, 1, grid_cap);
  if (grid >= kXcds) grid -= grid % kXcds;  // whole XCD segments
  hipLaunchKernelGGL((k_count_lds<NT, CAP>), dim3(grid), dim3(NT), 0, s, slots, bins.slot[cls], bins.a[cls],
                     bins.b[cls], bins.count + cls, bins.lds_xcd + kXcds * kLine * cls, bins.words + kXcds * kLine * cls,
                     probe_ratio, max_chunk, stealers);
  return hipGetLastError();
}

hipError_t launch_count_wave(const SlotDesc *slots, Bins bins, int64_t bound, KernelCfg cfg, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  const int d = cfg.wave_max_deg;
  if (d <= 64) return launch_lds<kWave, 64>(slots, bins, kClassWave, bound, cfg.grid_wave, cfg.probe_ratio, s);
  if (d <= 128) return launch_lds<kWave, 128>(slots, bins, kClassWave, bound, cfg.grid_wave, cfg.probe_ratio, s);
  if (d <= 256) return launch_lds<kWave, 256>(slots, bins, kClassWave, bound, cfg.grid_wave, cfg.probe_ratio, s);
  return launch_lds<kWave, 512>(slots, bins, kClassWave, bound, cfg.grid_wave, cfg.probe_ratio, s);
}

hipError_t launch_count_block(const SlotDesc *slots, Bins bins, int64_t bound, KernelCfg cfg, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  return launch_lds<256, kHubDeg>(slots, bins, kClassBlock, bound, cfg.grid_block, cfg.probe_ratio, s);
}

hipError_t launch_global_prep(const SlotDesc *slots, Bins bins, int64_t bound, int32_t chunk, int64_t *items,
                              int64_t *tcap, void *gacc, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_global_prep, dim3(grid_for(bound, 256, 8192)), dim3(256), 0, s, slots,
                     bins.slot[kClassGlobal], bins.a[kClassGlobal], bins.b[kClassGlobal], bins.count + kClassGlobal,
                     chunk, items, tcap, (GEdge *)gacc);
  return hipGetLastError();
}

hipError_t launch_global_scans(Bins bins, const int64_t *items, int64_t *item_pref, const int64_t *tcap,
                               int64_t *tbase, int64_t *tmp, hipStream_t s) {
  hipError_t e = launch_scan_dev(items, item_pref, bins.count + kClassGlobal, bins.cap, tmp, bins.gtot, s);
  if (e != hipSuccess) return e;
  return launch_scan_dev(tcap, tbase, bins.count + kClassGlobal, bins.cap, tmp, bins.gtot + 1, s);
}

hipError_t launch_item_fill(Bins bins, const int64_t *item_pref, const int64_t *items, const int64_t *tbase,
                            int64_t bound, int32_t *item_edge, void *gacc, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_fill, dim3(grid_for(bound, 256, 8192)), dim3(256), 0, s, bins, item_pref, items, tbase,
                     item_edge, (GEdge *)gacc);
  return hipGetLastError();
}

hipError_t launch_global_finish(const SlotDesc *slots, Bins bins, int64_t bound, const int64_t *item_cnt,
                                const void *gacc, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_global_finish, dim3(grid_for(bound, 4 * kWave, 1024)), dim3(256), 0, s, slots, bins,
                     (const GEdge *)gacc, item_cnt);
  return hipGetLastError();
}

hipError_t launch_global_classify(const SlotDesc *slots, Bins bins, const int64_t *item_pref,
                                  const int64_t *item_cnt, const int32_t *item_edge, const int64_t *tbase,
                                  int32_t *tlist, unsigned long long *tmask, void *gacc, KernelCfg cfg,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_global_classify, dim3(cfg.grid_global * (kGlobalNT / kPrepNT)), dim3(kPrepNT), 0, s, slots,
                     bins, item_pref, item_cnt, item_edge, tlist, tmask, (GEdge *)gacc, cfg.global_chunk,
                     (cfg.flags & kOptXcdLocal) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_sort_global(const SlotDesc *slots, Bins bins, int64_t bound, int32_t *slot2, int32_t *a2,
                              int32_t *b2, int64_t *hist, int64_t *off, int64_t *tmp, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  hipError_t e = launch_zero_u64((unsigned long long *)hist, kSortKeys, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_hist, dim3(grid_for(bound, 256, 4096)), dim3(256), 0, s, slots, bins.slot[kClassGlobal],
                     bins.b[kClassGlobal], bins.count + kClassGlobal, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan_i64(hist, off, kSortKeys, tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_scatter, dim3(grid_for(bound, 256, 4096)), dim3(256), 0, s, slots,
                     bins.slot[kClassGlobal], bins.a[kClassGlobal], bins.b[kClassGlobal], bins.count + kClassGlobal,
                     off, slot2, a2, b2);
  return hipGetLastError();
}

hipError_t launch_global_tbits(const SlotDesc *slots, Bins bins, int64_t bound, const int64_t *tbase,
                               const int32_t *tlist, unsigned long long *tbw, int16_t *tbi, void *gacc, hipStream_t s) {
  if (bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_global_tbits, dim3(grid_for(bound, 1, 8192)), dim3(kPrepNT), 0, s, slots,
                     bins.slot[kClassGlobal], bins, tbase, tlist, (GEdge *)gacc, tbw, tbi);
  return hipGetLastError();
}

hipError_t launch_count_global(const SlotDesc *slots, Bins bins, const int64_t *item_pref,
                               const int64_t *item_cnt, const int32_t *item_edge, const int32_t *tlist, const unsigned long long *tbw, const int16_t *tbi,
                               const unsigned long long *tmask, void *gacc, KernelCfg cfg, hipStream_t s) {
  hipLaunchKernelGGL(k_count_global, dim3(cfg.grid_global), dim3(kGlobalNT), 0, s, slots, bins, item_pref,
                     item_cnt, item_edge, tlist, tbw, tbi, tmask, (GEdge *)gacc, bins.cursor + kClassGlobal,
                     bins.xcd_cursor, bins.words + kXcds * kLine * kClassGlobal, cfg.probe_ratio, cfg.global_chunk, cfg.flags);
  return hipGetLastError();
}

size_t gedge_bytes() { return sizeof(GEdge); }

// ---------------------------------------------------------------------------
// Workspace of the allocation-free estimate: a fixed array in device memory
// (each GPU that loads the library holds its own copy until the process
// ends).  In host code its name is not a device address; the address comes
// from hipGetSymbolAddress on each device, once, and only that address is
// handed to kernels and copies.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_init_mu;
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_use_mu[kMaxDevices];
}  // namespace

hipError_t scratch_address(int device, void **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_init_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

std::mutex &scratch_lock(int device) { return g_scratch_use_mu[device]; }

hipError_t launch_vinfo(const int32_t *row_ptr, const int32_t *crank, const int32_t *hrow, const int32_t *rcol,
                        int64_t n, int4 *vinfo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vinfo, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, row_ptr, crank, hrow, rcol, n, vinfo);
  return hipGetLastError();
}

hipError_t launch_arc_rank(const int32_t *col, const int4 *vinfo, int64_t nnz, uint32_t *arh, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_arc_rank, dim3(grid_for(nnz, 256, 16384)), dim3(256), 0, s, col, vinfo, nnz, arh);
  return hipGetLastError();
}

int64_t rows_tile_entries(int) { return kTileCols; }

hipError_t launch_col_count(const int32_t *row_ptr, const uint32_t *arh, int64_t n, int64_t *cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_count, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, arh, n, cnt);
  return hipGetLastError();
}

hipError_t launch_col_fill(const int32_t *row_ptr, const uint32_t *arh, int64_t n, const int64_t *off, int32_t *clist,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_fill, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, row_ptr, arh, n, off, clist);
  return hipGetLastError();
}

hipError_t launch_rows_fill(const int32_t *row_ptr, const int32_t *col, const int64_t *coff, const int64_t *ccnt,
                            const int32_t *clist, const int32_t *hubs, int64_t nh, int64_t ncol, int64_t stride,
                            int width, uint8_t *rows, int64_t n, int32_t *toff, int64_t toff_len, hipStream_t s) {
  const int64_t ntiles = (ncol + kTileCols - 1) / kTileCols;
  if (nh <= 0 || ntiles <= 0) return hipSuccess;
  if (n <= 0 || toff_len < 2 * n) return hipErrorInvalidValue;
  // tiles per pass: as many as the segment-end buffer holds
  const int64_t nb_max = toff_len / n - 1;
  for (int64_t t0 = 0; t0 < ntiles; t0 += nb_max) {
    const int64_t nb = ntiles - t0 < nb_max ? ntiles - t0 : nb_max;
    hipLaunchKernelGGL(k_rows_offsets, dim3(grid_for(n * (nb + 1), 256, 65536)), dim3(256), 0, s, coff, ccnt, clist,
                       n, t0, nb, toff);
    hipLaunchKernelGGL(k_rows_fill, dim3(grid_for(nh * nb, 1, 1 << 20)), dim3(kTileNT), 0, s, row_ptr, col, clist,
                       hubs, nh, toff, t0, nb, ncol, stride, width, rows);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


hipError_t launch_codeg_bits(const int32_t *row_ptr, const int32_t *col, const int32_t *crank, int64_t n, int64_t hcw,
                             unsigned long long *bits, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codeg_bits, dim3(grid_for(n, 4, 16384)), dim3(256), 0, s, row_ptr, col, crank, n, hcw, bits);
  return hipGetLastError();
}


hipError_t launch_core_init(const int32_t *row_ptr, int64_t n, int32_t *deg, int32_t *state, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_core_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, row_ptr, n, deg, state);
  return hipGetLastError();
}

hipError_t launch_core_scan(int64_t n, int32_t k, int32_t *deg, int32_t *state, int32_t *front,
                            unsigned long long *cnt, unsigned long long *minalive, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_core_scan, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, k, deg, state, front, cnt,
                     minalive);
  return hipGetLastError();
}

hipError_t launch_core_peel(const int32_t *row_ptr, const int32_t *col, const int32_t *front, int64_t fn, int32_t k,
                            int32_t *deg, int32_t *state, int32_t *core, int32_t *next, unsigned long long *ncnt,
                            hipStream_t s) {
  if (fn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_core_peel, dim3(grid_for(fn, 4, 16384)), dim3(256), 0, s, row_ptr, col, front, fn, k, deg,
                     state, core, next, ncnt);
  return hipGetLastError();
}

hipError_t launch_weight_levels(int32_t mode, const int32_t *row_ptr, const uint64_t *edges, const int32_t *core,
                                int64_t m, uint8_t *level, unsigned long long *hist, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weight_levels, dim3(grid_for(m, 256, 4096)), dim3(256), 0, s, mode, row_ptr, edges, core, m,
                     level, hist);
  return hipGetLastError();
}

hipError_t launch_select_hist(uint64_t seed, int64_t m, int32_t shift, uint64_t pre_hi, uint64_t pre_lo,
                              unsigned long long *hist, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_hist, dim3(grid_for(m, 256, 4096)), dim3(256), 0, s, seed, m, shift, pre_hi, pre_lo,
                     hist);
  return hipGetLastError();
}


hipError_t launch_micro_arc_tri(const int32_t *row_ptr, const int32_t *col, const uint64_t *edges,
                                const int64_t *hoff, const uint32_t *htab, int64_t m, int32_t *t_arc, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_micro_arc_tri, dim3(grid_for(m, 256 / kMicroGroup, 16384)), dim3(256), 0, s, row_ptr, col,
                     edges, hoff, htab, m, t_arc);
  return hipGetLastError();
}

hipError_t launch_micro_vertex_tri(const int32_t *row_ptr, const int32_t *t_arc, int64_t n, int64_t *tri,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_micro_vertex_tri, dim3(grid_for(n, 4, 16384)), dim3(256), 0, s, row_ptr, t_arc, n, tri);
  return hipGetLastError();
}

hipError_t launch_micro_mark(long long *out, int64_t rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_micro_mark, dim3(grid_for(rows, 256, 8192)), dim3(256), 0, s, out, rows);
  return hipGetLastError();
}

hipError_t launch_micro_rows(const int32_t *row_ptr, const int32_t *col, const uint64_t *edges, const int64_t *vol2,
                             const int64_t *hoff, const uint32_t *htab, const int32_t *t_slot, const int4 *vinfo,
                             const int32_t *t_arc, const int64_t *tri, int64_t n, int64_t m, int64_t e0, int64_t e1,
                             long long *out, unsigned long long *colmax, int *err, int grid, hipStream_t s) {
  if (e1 <= e0) return hipSuccess;
  const int need = grid_for(e1 - e0, 256 / kMicroGroup, 1 << 20);
  const int g = need < grid ? need : grid;
  hipLaunchKernelGGL(k_micro_rows, dim3(g), dim3(256), 0, s, row_ptr, col, edges, vol2, hoff, htab, t_slot, vinfo,
                     t_arc, tri, n, m, e0, e1, out, colmax, err);
  return hipGetLastError();
}

hipError_t launch_micro_slot_tri(const int32_t *row_ptr, const int32_t *col, int64_t n, const int64_t *hoff,
                                 const uint32_t *htab, const int32_t *t_arc, int32_t *t_slot, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_micro_slot_tri, dim3(grid_for(n, 1, 65536)), dim3(256), 0, s, row_ptr, col, n, hoff, htab,
                     t_arc, t_slot);
  return hipGetLastError();
}


}  // namespace lge
