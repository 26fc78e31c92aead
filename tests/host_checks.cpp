// Host-only checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by tests/test_host_sanitizers.py with g++, no GPU): the runtime's
// CSR validation, its int128 / 256-bit -> double conversions and its
// finalisation of exact sums, each against the oracle or against values
// fixed by the arithmetic, and the oracle's own estimator on small graphs.
// Exit status 0 when every check holds; sanitizer reports abort the run.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../paper_1701_01772_amd/csrc/lge_hostmath.h"

// The oracle's C interface (oracle/lge_oracle.c).
extern "C" {
typedef struct {
  uint64_t lo, hi;
} oracle_u128;
typedef struct {
  int64_t n, m;
  double p;
  uint64_t seed;
  uint64_t sampled;
  oracle_u128 csum[18], zsum[18], qsum[18], exact[18];
  double estimate[18], variance[18], lower95[18], upper95[18];
} oracle_result;
int oracle_estimate(int64_t n, const int32_t *row_ptr, const int32_t *col, double p, uint64_t seed,
                    const uint8_t *mask, oracle_result *res);
double oracle_i128_to_double(uint64_t lo, uint64_t hi);
}

static int failures = 0;
#define CHECK(cond, ...)                                 \
  do {                                                   \
    if (!(cond)) {                                       \
      ++failures;                                        \
      fprintf(stderr, "check failed (%s): ", #cond);     \
      fprintf(stderr, __VA_ARGS__);                      \
      fprintf(stderr, "\n");                             \
    }                                                    \
  } while (0)

struct Csr {
  int64_t n = 0;
  std::vector<int32_t> rp, col;
};

// simple undirected graph with sorted rows from an edge probability
static Csr random_graph(int64_t n, double q, std::mt19937_64 &rng) {
  std::vector<std::vector<int32_t>> adj((size_t)n);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  for (int32_t u = 0; u < n; ++u)
    for (int32_t v = u + 1; v < n; ++v)
      if (U(rng) < q) {
        adj[(size_t)u].push_back(v);
        adj[(size_t)v].push_back(u);
      }
  Csr g;
  g.n = n;
  g.rp.push_back(0);
  for (auto &row : adj) {
    std::sort(row.begin(), row.end());
    g.col.insert(g.col.end(), row.begin(), row.end());
    g.rp.push_back((int32_t)g.col.size());
  }
  return g;
}

static int validate(const Csr &g) { return lge_validate_csr_host(g.n, g.rp.data(), g.col.data()); }

static Csr make(int64_t n, std::vector<int32_t> rp, std::vector<int32_t> col) {
  Csr g;
  g.n = n;
  g.rp = rp;
  g.col = col;
  return g;
}

static void check_validation(std::mt19937_64 &rng) {
  for (int k = 0; k < 20; ++k) {
    Csr g = random_graph(5 + k * 7, 0.2, rng);
    CHECK(validate(g) == LGE_OK, "valid graph %d rejected", k);
    if (g.col.size() < 4) continue;
    Csr bad = g;  // out of range
    bad.col[bad.col.size() - 1] = (int32_t)g.n + 3;
    CHECK(validate(bad) == LGE_EGRAPH, "out-of-range vertex accepted");
    bad = g;  // unsorted row
    for (int64_t u = 0; u < g.n; ++u)
      if (g.rp[(size_t)u + 1] - g.rp[(size_t)u] >= 2) {
        std::swap(bad.col[(size_t)g.rp[(size_t)u]], bad.col[(size_t)g.rp[(size_t)u] + 1]);
        CHECK(validate(bad) == LGE_EGRAPH, "unsorted row accepted");
        break;
      }
  }
  // one planted defect each, the rest of the graph well formed
  CHECK(validate(make(2, {0, 2, 4}, {0, 1, 0, 1})) == LGE_EGRAPH, "self loops accepted");
  CHECK(validate(make(3, {0, 1, 2, 2}, {1, 2})) == LGE_EGRAPH, "asymmetric graph accepted");
  CHECK(validate(make(2, {0, 2, 4}, {1, 1, 0, 0})) == LGE_EGRAPH, "duplicate entries accepted");
  CHECK(validate(make(3, {0, 2, 1, 4}, {1, 2, 0, 0})) == LGE_EGRAPH, "decreasing row pointer accepted");
  CHECK(validate(make(2, {1, 2, 2}, {1, 0})) == LGE_EGRAPH, "row_ptr[0] != 0 accepted");
  CHECK(validate(make(2, {0, 1, 1}, {1})) == LGE_EGRAPH, "odd entry count accepted");
  CHECK(validate(make(3, {0, 2, 4, 6}, {1, 2, 0, 2, 0, 1})) == LGE_OK, "triangle rejected");
  std::vector<int32_t> rp0 = {0};
  CHECK(lge_validate_csr_host(0, rp0.data(), nullptr) == LGE_OK, "empty graph rejected");
  CHECK(lge_validate_csr_host(-1, rp0.data(), nullptr) == LGE_EINVAL, "negative n accepted");
  CHECK(lge_validate_csr_host(3, nullptr, nullptr) == LGE_EINVAL, "null row_ptr accepted");
  std::vector<int32_t> rp2 = {0, 1, 2};
  CHECK(lge_validate_csr_host(2, rp2.data(), nullptr) == LGE_EINVAL, "null col accepted");
}

// x << s as 256 bits, x < 2^64, 0 <= s <= 192
static lge::U256 shl(u128 x, int s) {
  lge::U256 r{0, 0};
  if (s < 128) {
    r.lo = x << s;
    r.hi = s > 64 ? x >> (128 - s) : 0;
  } else {
    r.hi = x << (s - 128);
  }
  return r;
}

static lge::U256 add256(lge::U256 a, lge::U256 b) {
  lge::U256 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

static double i128_ref(i128 x) {  // the oracle's conversion
  const u128 u = (u128)x;
  return oracle_i128_to_double((uint64_t)u, (uint64_t)(u >> 64));
}

static void check_conversions(std::mt19937_64 &rng) {
  std::vector<i128> xs = {0, 1, -1, ((i128)1 << 53) + 1, ((i128)1 << 54) + 2, ((i128)1 << 54) + 6,
                          ((i128)1 << 100) + ((i128)1 << 47), ((i128)1 << 100) + ((i128)3 << 47),
                          (i128)(((u128)1 << 127) - 1), -(i128)(((u128)1 << 127) - 1)};
  for (int k = 0; k < 20000; ++k) {
    const u128 r = ((u128)rng() << 64) | (u128)rng();
    const int keep = 1 + (int)(rng() % 127);
    i128 x = (i128)(r >> (128 - keep));
    if (rng() & 1) x = -x;
    xs.push_back(x);
  }
  for (i128 x : xs) {
    const double a = lge::to_double(x), b = i128_ref(x);
    CHECK(memcmp(&a, &b, sizeof(a)) == 0, "to_double differs from the oracle: %.17g vs %.17g", a, b);
  }
  // 256-bit products: exact below 2^53, the int128 conversion for products
  // that fit 127 bits, and ties at every shift across the 128-bit boundary
  for (int k = 0; k < 20000; ++k) {
    const u128 a = (u128)(rng() >> (rng() % 64)), b = (u128)(rng() >> (rng() % 64));
    const lge::U256 p = lge::mul_u128(a, b);
    const u128 prod = a * b;  // fits: both below 2^64
    CHECK(p.hi == 0 && p.lo == prod, "mul_u128 of 64-bit operands");
    if (prod < ((u128)1 << 127)) {
      const double x = lge::u256_to_double(p), y = lge::to_double((i128)prod);
      CHECK(memcmp(&x, &y, sizeof(x)) == 0, "u256_to_double differs from to_double");
    }
  }
  for (int sh = 1; sh <= 200; ++sh) {
    // a 53-bit mantissa (odd, then even) followed by exactly half an ulp:
    // rounds to the even neighbour
    for (uint64_t mant : {(1ull << 52) | 1ull, (1ull << 52) | 2ull}) {
      const lge::U256 t = add256(shl(mant, sh), shl(1, sh - 1));
      const double got = lge::u256_to_double(t);
      const uint64_t want_m = (mant & 1) ? mant + 1 : mant;
      const double want = ldexp((double)want_m, sh);
      CHECK(got == want, "u256 tie at shift %d: %.17g vs %.17g", sh, got, want);
      // one unit above half rounds up whatever the parity
      const lge::U256 up = add256(t, shl(1, 0));
      CHECK(lge::u256_to_double(up) == ldexp((double)(mant + 1), sh), "u256 above half at %d", sh);
    }
  }
  CHECK(lge::binom(1000000, 4) == (i128)41666416667124999LL * 1000000 + 750000, "C(10^6, 4)");
  CHECK(lge::binom(3, 4) == 0 && lge::binom(4, 4) == 1 && lge::binom(2000, 2) == 1999000, "small binomials");
}

static void check_finalize(std::mt19937_64 &rng) {
  for (int k = 0; k < 12; ++k) {
    Csr g = random_graph(30 + 9 * k, 0.08 + 0.02 * (k % 5), rng);
    const double p = (k % 3 == 0) ? 1.0 : (k % 3 == 1 ? 0.5 : 0.13);
    oracle_result o;
    const int rc = oracle_estimate(g.n, g.rp.data(), g.col.data(), p, 77 + k, nullptr, &o);
    CHECK(rc == 0, "oracle_estimate returned %d", rc);
    // the kernels' accumulator layout: C3..C16 (without C6), Q3..Q17, count
    std::vector<unsigned long long> acc(2 * lge::kAccSlots, 0ull);
    static const int cidx[lge::kNumC] = {3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
    for (int i = 0; i < lge::kNumC; ++i) {
      acc[2 * i] = o.csum[cidx[i]].lo;
      acc[2 * i + 1] = o.csum[cidx[i]].hi;
    }
    for (int i = 0; i < lge::kNumQ; ++i) {
      acc[2 * (lge::kNumC + i)] = o.qsum[3 + i].lo;
      acc[2 * (lge::kNumC + i) + 1] = o.qsum[3 + i].hi;
    }
    acc[2 * lge::kAccIdxCount] = o.sampled;
    lge_result r;
    lge_finalize(g.n, (int64_t)g.col.size() / 2, p, 77 + k, acc.data(), &r);
    CHECK(r.sampled_edges == o.sampled, "sampled");
    for (int i = 3; i <= 17; ++i) {
      CHECK(r.z[i].lo == o.zsum[i].lo && r.z[i].hi == o.zsum[i].hi, "Z%d", i);
      CHECK(r.q[i].lo == o.qsum[i].lo && r.q[i].hi == o.qsum[i].hi, "Q%d", i);
      if (p == 1.0) CHECK(r.exact[i].lo == o.exact[i].lo && r.exact[i].hi == o.exact[i].hi, "exact %d", i);
    }
    for (int i = 1; i <= 17; ++i) {
      const double pairs[4][2] = {{r.estimate[i], o.estimate[i]}, {r.variance[i], o.variance[i]},
                                  {r.lower95[i], o.lower95[i]}, {r.upper95[i], o.upper95[i]}};
      for (auto &pr : pairs) {
        const double a = pr[0], b = pr[1];
        CHECK(a == b || fabs(a - b) <= 1e-12 * fmax(fabs(a), fabs(b)), "G%d: %.17g vs %.17g", i, a, b);
      }
    }
  }
}

static void check_sizes() {
  // the squared per-edge numerators, at most 16 C(n,2) each, summed over m
  // edges must stay below 2^127
  CHECK(lge::sizes_in_range(1000, 10000, 100), "small graph out of range");
  CHECK(lge::sizes_in_range(1000000, 10000000, 10000), "10^6 vertices out of range");
  CHECK(lge::sizes_in_range(4194304, 64156389, 163213), "R-MAT scale 22 out of range");
  CHECK(!lge::sizes_in_range(100000000, 1000000000, 100000), "10^8 vertices and 10^9 edges accepted");
  CHECK(!lge::sizes_in_range(lge::kMaxVertices, 10, 2), "kMaxVertices accepted");
  // a batch of 16,384 members of up to 5,000 vertices: each member is in
  // range, their disjoint union is not (the batch path checks members only)
  CHECK(lge::sizes_in_range(5000, 50000, 4999), "batch member out of range");
  CHECK(!lge::sizes_in_range(17000000, 100000000, 5000), "16,384-member union in range");
}

int main() {
  std::mt19937_64 rng(20240611);
  check_validation(rng);
  check_conversions(rng);
  check_finalize(rng);
  check_sizes();
  if (failures) {
    fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}
