// Host-only arithmetic of the runtime: CSR validation, the size bounds of
// exact sums, and the finalisation of exact 128-bit sums into FP64 estimates,
// variances and 95% bounds (Sec. 2.4: sigma = 1/p; the variance estimator
// with weight (1 - p) / p^2).  No HIP: this part also builds with a plain C++
// compiler, which the tests use for an address / undefined-behaviour
// sanitizer build.
#pragma once

#include <stdint.h>

#include "../../include/lge.h"
#include "lge_layout.h"

typedef __int128 i128;
typedef unsigned __int128 u128;

namespace lge {

// The exact sums of one accumulator slot: C (unrestricted counts), Z (sums of
// 12 Y_i(e), linear in C), Q (sums of (12 Y_i(e))^2) and the edge count.
struct ExactSums {
  i128 C[18];
  i128 Z[18];
  u128 Q[18];
  uint64_t count;
};

u128 u128_of(const unsigned long long *p);
lge_u128 to_abi(u128 x);
// C(n, k) for k <= 4 (exact)
i128 binom(int64_t n, int k);
// correctly rounded int128 -> double (to nearest, ties to even)
double to_double(i128 x);
// acc: kAccSlots x {lo, hi} as the kernels produce them
void sums_from_acc(const unsigned long long *acc, ExactSums *s);
void sums_add(ExactSums *a, const ExactSums &b);
// integer fields of a result; K receives K_6 = C(n,3), K_17 = C(n,4), E the
// exact counts valid when every edge is in the sample
void fill_exact(int64_t n, int64_t m, double p, uint64_t seed, const ExactSums &t, lge_result *out,
                i128 K[18], i128 E[18]);
void set_xv(lge_result *out, int i, double x, double v);

// 256-bit helpers for the fixed-size variance numerator K Q - Z^2
struct U256 {
  u128 hi, lo;
};
U256 mul_u128(u128 a, u128 b);
U256 sub_u256(U256 a, U256 b);
// correctly rounded (to nearest, ties to even)
double u256_to_double(U256 a);

// do the per-edge numerators of a graph with n vertices, m edges and
// maximum degree dmax fit int64, and their sums of squares 128 bits?
bool sizes_in_range(int64_t n, int64_t m, int64_t dmax);

}  // namespace lge

// Exact integers -> lge_result (C, Z, Q, exact counts, FP64 estimates,
// variances, bounds) from one slot's accumulators.
void lge_finalize(int64_t n, int64_t m, double p, uint64_t seed, const unsigned long long *acc, lge_result *out);
