// Host-only arithmetic of the runtime (declared in lge_hostmath.h).
#include "lge_hostmath.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace lge {

u128 u128_of(const unsigned long long *p) { return ((u128)p[1] << 64) | (u128)p[0]; }

lge_u128 to_abi(u128 x) {
  lge_u128 r;
  r.lo = (uint64_t)x;
  r.hi = (uint64_t)(x >> 64);
  return r;
}

i128 binom(int64_t n, int k) {
  if (n < k) return 0;
  i128 r = 1;
  for (int i = 0; i < k; ++i) r = r * (i128)(n - i) / (i128)(i + 1);
  return r;
}

// correctly rounded int128 -> double (round to nearest even)
double to_double(i128 x) {
  const bool neg = x < 0;
  u128 a = neg ? (u128)0 - (u128)x : (u128)x;
  int bits = 0;
  for (u128 t = a; t; t >>= 1) ++bits;
  if (bits <= 53) {
    const double d = (double)(uint64_t)a;
    return neg ? -d : d;
  }
  const int sh = bits - 53;
  u128 mant = a >> sh;
  const u128 rem = a - (mant << sh);
  const u128 half = (u128)1 << (sh - 1);
  if (rem > half || (rem == half && (mant & 1))) ++mant;
  const double d = ldexp((double)(uint64_t)mant, sh);
  return neg ? -d : d;
}

void sums_from_acc(const unsigned long long *acc, ExactSums *s) {
  memset(s, 0, sizeof(*s));
  s->count = (uint64_t)u128_of(acc + 2 * kAccIdxCount);
  static const int cidx[kNumC] = {3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
  i128 *C = s->C;
  for (int k = 0; k < kNumC; ++k) C[cidx[k]] = (i128)u128_of(acc + 2 * k);
  for (int k = 0; k < kNumQ; ++k) s->Q[3 + k] = u128_of(acc + 2 * (kNumC + k));
  // Z_i = sum of 12 Y_i(e); the map from the C sums is linear
  i128 *Z = s->Z;
  const i128 d87 = C[8] - C[7];
  const i128 z9_3 = 2 * C[9] - 8 * d87;
  Z[3] = 4 * C[3];
  Z[4] = 6 * C[4];
  Z[5] = 12 * C[5];
  Z[6] = -(Z[3] + Z[4] + Z[5]);
  Z[7] = 2 * C[7];
  Z[8] = 12 * d87;
  Z[9] = 3 * z9_3;
  Z[10] = 3 * C[10];
  Z[11] = 4 * C[11] - z9_3;
  Z[12] = 12 * (C[12] - C[10]);
  Z[13] = 4 * C[13] - z9_3;
  Z[14] = 6 * C[14] - Z[12];
  Z[15] = 6 * C[15] - 3 * Z[7] - 2 * Z[8] - Z[9] - 2 * Z[10] - Z[12];
  Z[16] = 12 * C[16] - 2 * Z[15];
  Z[17] = 0;
  for (int i = 7; i <= 16; ++i) Z[17] -= Z[i];
}

void sums_add(ExactSums *a, const ExactSums &b) {
  for (int i = 0; i < 18; ++i) {
    a->C[i] += b.C[i];
    a->Z[i] += b.Z[i];
    a->Q[i] += b.Q[i];
  }
  a->count += b.count;
}

// Integer fields of a result from exact sums; K receives the constants
// K_6 = C(n,3), K_17 = C(n,4), E the exact counts valid when every edge is in
// the sample.
void fill_exact(int64_t n, int64_t m, double p, uint64_t seed, const ExactSums &t, lge_result *out,
                       i128 K[18], i128 E[18]) {
  memset(out, 0, sizeof(*out));
  out->n = n;
  out->m = m;
  out->p = p;
  out->seed = seed;
  out->sampled_edges = t.count;
  for (int i = 0; i < 18; ++i) K[i] = E[i] = 0;
  K[6] = binom(n, 3);
  K[17] = binom(n, 4);
  E[1] = m;
  E[2] = binom(n, 2) - m;
  for (int i = 3; i <= 17; ++i) E[i] = K[i] + t.Z[i] / 12;
  for (int i = 0; i < 18; ++i) {
    out->csum[i] = to_abi((u128)t.C[i]);
    out->z[i] = to_abi((u128)t.Z[i]);
    out->q[i] = to_abi(t.Q[i]);
    out->exact[i] = to_abi((u128)E[i]);
  }
}

void set_xv(lge_result *out, int i, double x, double v) {
  const double h = 1.96 * sqrt(v);
  out->estimate[i] = x;
  out->variance[i] = v;
  out->lower95[i] = x - h;
  out->upper95[i] = x + h;
}

U256 mul_u128(u128 a, u128 b) {
  const u128 a0 = (uint64_t)a, a1 = a >> 64, b0 = (uint64_t)b, b1 = b >> 64;
  const u128 p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
  const u128 mid = (p00 >> 64) + (u128)(uint64_t)p01 + (u128)(uint64_t)p10;
  U256 r;
  r.lo = (mid << 64) | (u128)(uint64_t)p00;
  r.hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
  return r;
}

U256 sub_u256(U256 a, U256 b) {
  U256 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1 : 0);
  return r;
}

int bitlen_u128(u128 x) {
  int b = 0;
  for (; x; x >>= 1) ++b;
  return b;
}

// correctly rounded (to nearest, ties to even)
double u256_to_double(U256 a) {
  const int bits = a.hi ? 128 + bitlen_u128(a.hi) : bitlen_u128(a.lo);
  if (bits <= 53) return (double)(uint64_t)a.lo;
  const int sh = bits - 53;  // 1 .. 203
  u128 mant;
  bool gt_half, eq_half;
  if (sh < 128) {
    mant = (a.hi << (128 - sh)) | (a.lo >> sh);
    const u128 rem = a.lo & ((((u128)1) << sh) - 1);
    const u128 h = (u128)1 << (sh - 1);
    gt_half = rem > h;
    eq_half = rem == h;
  } else if (sh == 128) {
    mant = a.hi;
    const u128 h = (u128)1 << 127;
    gt_half = a.lo > h;
    eq_half = a.lo == h;
  } else {
    mant = a.hi >> (sh - 128);
    const u128 rem_hi = a.hi & ((((u128)1) << (sh - 128)) - 1);
    const u128 h_hi = (u128)1 << (sh - 129);
    gt_half = rem_hi > h_hi || (rem_hi == h_hi && a.lo != 0);
    eq_half = rem_hi == h_hi && a.lo == 0;
  }
  if (gt_half || (eq_half && (mant & 1))) ++mant;
  return ldexp((double)(uint64_t)mant, sh);
}

// Every per-edge numerator 12*Y_i(e) must fit in int64 and every sum of
// squares in 128 bits: |12 Y| <= 16 * max count term, the largest term being
// C(n,2), 2*dmax*n, 4*dmax^2 or m.
bool sizes_in_range(int64_t n, int64_t m, int64_t dmax) {
  if (n >= kMaxVertices) return false;
  long double cmax = (long double)n * (long double)n / 2.0L;
  cmax = std::max(cmax, 2.0L * dmax * (long double)n);
  cmax = std::max(cmax, 4.0L * dmax * (long double)dmax);
  cmax = std::max(cmax, (long double)m);
  const long double zmax = 16.0L * cmax;
  if (zmax >= ldexpl(1.0L, 62)) return false;
  if ((long double)m * zmax * zmax >= ldexpl(1.0L, 127)) return false;
  return true;
}

}  // namespace lge

using namespace lge;

void lge_finalize(int64_t n, int64_t m, double p, uint64_t seed, const unsigned long long *acc,
                  lge_result *out) {
  ExactSums t;
  sums_from_acc(acc, &t);
  i128 K[18], E[18];
  fill_exact(n, m, p, seed, t, out, K, E);
  const double sigma = 1.0 / p;
  const double vfac = (1.0 - p) / (p * p);
  for (int i = 1; i <= 17; ++i) {
    if (i <= 2 || p == 1.0)
      set_xv(out, i, to_double(E[i]), 0.0);
    else
      set_xv(out, i, to_double(K[i]) + (to_double(t.Z[i]) * sigma) / 12.0,
             (to_double((i128)t.Q[i]) * vfac) / 144.0);
  }
}

extern "C" int lge_validate_csr_host(int64_t n, const int32_t *row_ptr, const int32_t *col) {
  if (n < 0 || !row_ptr) return LGE_EINVAL;
  if (row_ptr[0] != 0) return LGE_EGRAPH;
  for (int64_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return LGE_EGRAPH;
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && !col) return LGE_EINVAL;
  if (nnz % 2) return LGE_EGRAPH;
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<int> bad{0};
  auto work = [&](unsigned id) {
    for (int64_t u = id; u < n && !bad.load(std::memory_order_relaxed); u += nt) {
      for (int32_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
        const int32_t v = col[j];
        if (v < 0 || v >= n || v == u || (j > row_ptr[u] && col[j - 1] >= v)) {
          bad = 1;
          return;
        }
        if (!std::binary_search(col + row_ptr[v], col + row_ptr[v + 1], (int32_t)u)) {
          bad = 1;
          return;
        }
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned i = 1; i < nt; ++i) th.emplace_back(work, i);
  work(0);
  for (auto &t : th) t.join();
  return bad ? LGE_EGRAPH : LGE_OK;
}
