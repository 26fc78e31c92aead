/*
 * ORACLE (test infrastructure only).  A plain, slow, single-thread CPU
 * implementation of the edge-centric graphlet estimator of "Estimation of
 * Graphlet Statistics" (Rossi, Zhou, Ahmed).  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code with the GPU library.
 *
 * What it computes, in the paper's order:
 *   - edge sampling (Alg. 1 with a Bernoulli(p) design, Sec. 2.4): edge e is
 *     in J iff its Philox4x32-10 uniform is below p;
 *   - per sampled edge e=(v,u), LocalizedGraphletEst (Alg. 2): mark Gamma(v)
 *     with lambda1, classify Gamma(u) into T_e (lambda3) and S_u (lambda2);
 *     Clique (Alg. 3) over T_e, Cycle (Alg. 4) over S_u (reading: it counts
 *     neighbours still marked lambda1, i.e. S_v);
 *   - the unrestricted counts (eqs. non-induced-conn-n1..n4 and
 *     non-induced-disconn-n1..n4, with the disconnected labels read as the
 *     X equations use them);
 *   - the estimates X_3..X_17 (eqs. graphlet-X-start .. graphlet-X-end with
 *     the weight vector eq. graphlet-W, entries 13..16 read as 1/3, 1/2,
 *     1/2, 1), the unbiased variance estimate (Sec. 2.4) and the 95% bounds
 *     (eq. bounds-95).
 *
 * All counts are exact integers (128-bit where sums can exceed 64 bits);
 * floating point appears only in the sampling compare and the final
 * scaling.  Functions that have no independent pin say so below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 S-box with multipliers
 * 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.
 * ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Bernoulli(p) draw for canonical edge id eid: key = (seed lo, seed hi),
 * counter = (eid lo, eid hi, 0, 0); the uniform is the top 53 bits of
 * (x1:x0) scaled by 2^-53; the edge is sampled iff uniform < p. */
int oracle_edge_sampled(uint64_t seed, uint64_t eid, double p) {
  uint32_t ctr[4] = {(uint32_t)eid, (uint32_t)(eid >> 32), 0u, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  uint64_t bits = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
  double u = (double)(bits >> 11) * 0x1.0p-53;
  return u < p;
}

/* ---------------------------------------------------------------------------
 * Per-edge local quantities (Alg. 2, 3, 4).
 * out[0..6] = |T_e|, |S_u|, |S_v|, n - |Gamma(u) u Gamma(v)|, Clique, Cycle,
 *             m - |Gamma(u)\{v}| - |Gamma(v)\{u}| - 1
 * psi is a caller-owned mark table of n int64 (never cleared: the marks are
 * unique per call through *stamp, as the paper does to avoid resets).
 * ------------------------------------------------------------------------ */
typedef struct {
  int64_t t, su, sv, r, clique, cycle, f;
} oracle_local;

static void local_counts(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, int32_t v,
                         int32_t u, int64_t *psi, int64_t *stamp, int32_t *tlist, int32_t *slist,
                         oracle_local *o) {
  const int64_t lam1 = *stamp + 1, lam2 = *stamp + 2, lam3 = *stamp + 3;
  *stamp += 4;
  /* mark Gamma(v) \ {u} with lambda1 */
  for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
    int32_t w = col[j];
    if (w != u) psi[w] = lam1;
  }
  /* classify Gamma(u) \ {v}: lambda1 -> triangle (re-mark lambda3), else wedge (lambda2) */
  int64_t nt = 0, ns = 0;
  for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
    int32_t w = col[j];
    if (w == v) continue;
    if (psi[w] == lam1) {
      tlist[nt++] = w;
      psi[w] = lam3;
    } else {
      slist[ns++] = w;
      psi[w] = lam2;
    }
  }
  int64_t du = row_ptr[u + 1] - row_ptr[u];
  int64_t dv = row_ptr[v + 1] - row_ptr[v];
  o->t = nt;
  o->su = ns;
  /* S_v = Gamma(v) \ {u} \ T_e : the vertices still marked lambda1 */
  int64_t sv = 0;
  for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j)
    if (psi[col[j]] == lam1) ++sv;
  o->sv = sv;
  /* |Gamma(u) u Gamma(v)|: Gamma(v) plus the members of Gamma(u) not in Gamma(v);
   * v itself is in Gamma(u) and not in Gamma(v), the S_u members likewise. */
  int64_t uni = dv + 1 + ns;
  o->r = n - uni;
  /* Clique (Alg. 3): for w in T_e count neighbours marked lambda3, then reset
   * psi(w); sequential order makes each edge inside T_e count once. */
  int64_t clique = 0;
  for (int64_t i = 0; i < nt; ++i) {
    int32_t w = tlist[i];
    for (int64_t j = row_ptr[w]; j < row_ptr[w + 1]; ++j)
      if (psi[col[j]] == lam3) ++clique;
    psi[w] = 0;
  }
  /* Cycle (Alg. 4): for w in S_u count neighbours in S_v (marked lambda1). */
  int64_t cycle = 0;
  for (int64_t i = 0; i < ns; ++i) {
    int32_t w = slist[i];
    for (int64_t j = row_ptr[w]; j < row_ptr[w + 1]; ++j)
      if (psi[col[j]] == lam1) ++cycle;
    psi[w] = 0;
  }
  o->clique = clique;
  o->cycle = cycle;
  o->f = m - (du - 1) - (dv - 1) - 1;
}

/* ---------------------------------------------------------------------------
 * Unrestricted counts of one edge, indexed by graphlet number (c[3..16],
 * c[6] unused), from the local quantities:
 *   C3 += |T|, C4 += |S_u|+|S_v|, C5 += r               (Alg. 2)
 *   C7 += Clique, C10 += Cycle                           (Alg. 3, 4)
 *   C8 += C(|T|,2), C9 += |T|(|S_u|+|S_v|),
 *   C11 += C(|S_u|,2)+C(|S_v|,2), C12 += |S_u||S_v|       (non-induced-conn)
 *   C13 += |T| r, C14 += (|S_u|+|S_v|) r, C15 += f, C16 += C(r,2)
 *        (non-induced-disconn, labels as used by X13..X16)
 * where r = n - |Gamma(u) u Gamma(v)| and f = m - (d_u-1) - (d_v-1) - 1.
 * ------------------------------------------------------------------------ */
static void unrestricted(const oracle_local *o, i128 c[17]) {
  for (int i = 0; i < 17; ++i) c[i] = 0;
  i128 t = o->t, su = o->su, sv = o->sv, r = o->r;
  c[3] = t;
  c[4] = su + sv;
  c[5] = r;
  c[7] = o->clique;
  c[8] = t * (t - 1) / 2;
  c[9] = t * (su + sv);
  c[10] = o->cycle;
  c[11] = su * (su - 1) / 2 + sv * (sv - 1) / 2;
  c[12] = su * sv;
  c[13] = t * r;
  c[14] = (su + sv) * r;
  c[15] = o->f;
  c[16] = r * (r - 1) / 2;
}

/* ---------------------------------------------------------------------------
 * The estimate equations with sigma = 1 and the binomial constants removed,
 * scaled by 12 so every term is an integer: z[i] = 12 * Y_i for the counts
 * c.  Applied to one edge's counts this is the per-edge contribution; applied
 * to the sums it is the sum of contributions (the map is linear).
 *   X3 = W3 C3, X4 = W4 C4, X5 = W5 C5, X6 = W6 [C(n,3) - X3 - X4 - X5]
 *   X7 = W7 C7, X8 = W8 (C8 - C7), X9 = W9 (C9 - 4 X8), X10 = W10 C10,
 *   X11 = W11 (C11 - X9), X12 = W12 (C12 - C10)
 *   X13 = W13 (C13 - X9), X14 = W14 (C14 - 2 X12),
 *   X15 = W15 (C15 - 6X7 - 4X8 - 2X9 - 4X10 - 2X12), X16 = W16 (C16 - 2 X15),
 *   X17 = W17 [C(n,4) - sum_{7..16} X_i]
 * with W = (1,1,1/3,1/2,1,1,1/6,1,1/2,1/4,1/3,1,1/3,1/2,1/2,1,1).
 * Returns 0, or -1 if a division is not exact (it always is for counts that
 * come from a graph).
 * ------------------------------------------------------------------------ */
static int div_exact(i128 num, i128 den, i128 *q) {
  if (num % den != 0) return -1;
  *q = num / den;
  return 0;
}

static int estimate_numerators(const i128 c[17], i128 z[18]) {
  for (int i = 0; i < 18; ++i) z[i] = 0;
  int bad = 0;
  /* z = 12 X, W_i = 1/w_i written as a division by w_i */
  bad |= div_exact(12 * c[3], 3, &z[3]);
  bad |= div_exact(12 * c[4], 2, &z[4]);
  z[5] = 12 * c[5];
  z[6] = -(z[3] + z[4] + z[5]);
  bad |= div_exact(12 * c[7], 6, &z[7]);
  z[8] = 12 * (c[8] - c[7]);
  bad |= div_exact(12 * c[9] - 4 * z[8], 2, &z[9]);
  bad |= div_exact(12 * c[10], 4, &z[10]);
  bad |= div_exact(12 * c[11] - z[9], 3, &z[11]);
  z[12] = 12 * (c[12] - c[10]);
  bad |= div_exact(12 * c[13] - z[9], 3, &z[13]);
  bad |= div_exact(12 * c[14] - 2 * z[12], 2, &z[14]);
  bad |= div_exact(12 * c[15] - 6 * z[7] - 4 * z[8] - 2 * z[9] - 4 * z[10] - 2 * z[12], 2, &z[15]);
  z[16] = 12 * c[16] - 2 * z[15];
  i128 s = 0;
  for (int i = 7; i <= 16; ++i) s += z[i];
  z[17] = -s;
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Result of one estimate.  Indices follow the graphlet numbers G1..G17
 * (slot 0 unused).  128-bit values are stored as (lo, hi) 64-bit limbs.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint64_t lo, hi;
} oracle_u128;

typedef struct {
  int64_t n, m;
  double p;
  uint64_t seed;
  uint64_t sampled;
  oracle_u128 csum[18];  /* C_i = sum over J of the unrestricted counts */
  oracle_u128 zsum[18];  /* Z_i = sum over J of 12 Y_i(e) (signed) */
  oracle_u128 qsum[18];  /* Q_i = sum over J of (12 Y_i(e))^2 */
  oracle_u128 exact[18]; /* exact counts, valid when every edge is sampled */
  double estimate[18], variance[18], lower95[18], upper95[18];
} oracle_result;

static oracle_u128 pack(u128 x) {
  oracle_u128 r;
  r.lo = (uint64_t)x;
  r.hi = (uint64_t)(x >> 64);
  return r;
}

static i128 choose(i128 n, int k) {
  if (n < k) return 0;
  i128 r = 1;
  for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
  return r;
}

/* int128 -> double, round to nearest even (written out: the two limbs are
 * converted separately only when that is exact). */
static double i128_to_double(i128 x) {
  int neg = x < 0;
  u128 a = neg ? (u128)(-(x + 1)) + 1 : (u128)x;
  double d;
  if ((a >> 53) == 0) {
    d = (double)(uint64_t)a;
  } else {
    int bits = 0; /* significant bits of a, 54..128 here */
    for (u128 t = a; t != 0; t >>= 1) ++bits;
    int shift = bits - 53;
    u128 mant = a >> shift;
    u128 rem = a & (((u128)1 << shift) - 1);
    u128 half = (u128)1 << (shift - 1);
    if (rem > half || (rem == half && (mant & 1))) ++mant;
    d = ldexp((double)(uint64_t)mant, shift);
  }
  return neg ? -d : d;
}

/*
 * Finalisation (shared by the Philox and the explicit-mask entry points).
 * sigma = 1/p (Bernoulli design, Sec. 2.4); X_i = K_i + (Z_i * sigma) / 12
 * with K_6 = C(n,3), K_17 = C(n,4), else 0; when p == 1 the exact integer is
 * converted once instead.  The unbiased variance estimate of a Horvitz-
 * Thompson sum under Bernoulli(p) sampling is (1-p)/p^2 * sum_J Y_i(e)^2,
 * i.e. Q_i (1-p)/p^2 / 144; bounds X -/+ 1.96 sqrt(V) (eq. bounds-95).
 */
static int finalize(int64_t n, int64_t m, double p, const i128 csum[17], const u128 q[18],
                    oracle_result *res) {
  i128 z[18];
  if (estimate_numerators(csum, z) != 0) return -2;
  i128 nn = n;
  i128 K[18] = {0};
  K[6] = choose(nn, 3);
  K[17] = choose(nn, 4);
  for (int i = 0; i < 17; ++i) res->csum[i] = pack((u128)csum[i]);
  res->csum[17] = pack(0);
  for (int i = 0; i < 18; ++i) {
    res->zsum[i] = pack((u128)z[i]);
    res->qsum[i] = pack(q[i]);
  }
  /* exact counts (meaningful when J = E) */
  i128 ex[18] = {0};
  ex[1] = m;
  ex[2] = choose(nn, 2) - m;
  for (int i = 3; i <= 17; ++i) ex[i] = K[i] + z[i] / 12;
  for (int i = 0; i < 18; ++i) res->exact[i] = pack((u128)ex[i]);
  double sigma = 1.0 / p;
  double vfac = (1.0 - p) / (p * p);
  for (int i = 0; i < 18; ++i) {
    res->estimate[i] = res->variance[i] = res->lower95[i] = res->upper95[i] = 0.0;
  }
  for (int i = 1; i <= 17; ++i) {
    double x, v;
    if (i <= 2) {
      x = i128_to_double(ex[i]);
      v = 0.0;
    } else if (p == 1.0) {
      x = i128_to_double(ex[i]);
      v = 0.0;
    } else {
      x = i128_to_double(K[i]) + (i128_to_double(z[i]) * sigma) / 12.0;
      v = (i128_to_double((i128)q[i]) * vfac) / 144.0;
    }
    res->estimate[i] = x;
    res->variance[i] = v;
    double h = 1.96 * sqrt(v);
    res->lower95[i] = x - h;
    res->upper95[i] = x + h;
  }
  return 0;
}

/*
 * Estimate over the edges selected either by Philox(seed) < p (mask == NULL)
 * or by mask[eid] != 0 (explicit sample, used to enumerate sample outcomes;
 * p is then only the design probability used for scaling).  Canonical edge
 * id: rank of (u, v), u < v, in row-major order of the sorted CSR.
 * Returns 0, -1 on allocation failure, -2 on an inexact division.
 */
int oracle_estimate(int64_t n, const int32_t *row_ptr, const int32_t *col, double p, uint64_t seed,
                    const uint8_t *mask, oracle_result *res) {
  memset(res, 0, sizeof(*res));
  int64_t m = (int64_t)row_ptr[n] / 2;
  res->n = n;
  res->m = m;
  res->p = p;
  res->seed = seed;
  int64_t *psi = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  int64_t maxd = 1;
  for (int64_t x = 0; x < n; ++x)
    if (row_ptr[x + 1] - row_ptr[x] > maxd) maxd = row_ptr[x + 1] - row_ptr[x];
  int32_t *tlist = (int32_t *)malloc((size_t)maxd * sizeof(int32_t));
  int32_t *slist = (int32_t *)malloc((size_t)maxd * sizeof(int32_t));
  if (!psi || !tlist || !slist) {
    free(psi);
    free(tlist);
    free(slist);
    return -1;
  }
  int64_t stamp = 0;
  i128 csum[17] = {0};
  u128 q[18] = {0};
  uint64_t eid = 0, sampled = 0;
  int rc = 0;
  for (int32_t a = 0; a < n && rc == 0; ++a) {
    for (int64_t j = row_ptr[a]; j < row_ptr[a + 1]; ++j) {
      int32_t b = col[j];
      if (b <= a) continue;
      uint64_t e = eid++;
      int take = mask ? (mask[e] != 0) : oracle_edge_sampled(seed, e, p);
      if (!take) continue;
      ++sampled;
      /* the scan side u is the endpoint of smaller degree (Sec. 2.5) */
      int64_t da = row_ptr[a + 1] - row_ptr[a], db = row_ptr[b + 1] - row_ptr[b];
      int32_t u = da <= db ? a : b, v = da <= db ? b : a;
      oracle_local o;
      local_counts(n, m, row_ptr, col, v, u, psi, &stamp, tlist, slist, &o);
      i128 c[17], z[18];
      unrestricted(&o, c);
      if (estimate_numerators(c, z) != 0) {
        rc = -2;
        break;
      }
      for (int i = 0; i < 17; ++i) csum[i] += c[i];
      for (int i = 3; i <= 17; ++i) {
        i128 zi = z[i];
        u128 az = (u128)(zi < 0 ? -zi : zi);
        q[i] += az * az;
      }
    }
  }
  free(psi);
  free(tlist);
  free(slist);
  res->sampled = sampled;
  if (rc != 0) return rc;
  return finalize(n, m, p, csum, q, res);
}

/* The finalisation above applied to sums the caller already holds: csum[0..16]
 * (C_i by graphlet number, two's complement limbs) and q[0..17] (Q_i), e.g.
 * the exact totals of several oracle_estimate calls over disjoint masks.
 * Returns 0 or -2 on an inexact division. */
int oracle_finalize_sums(int64_t n, int64_t m, double p, uint64_t seed, uint64_t sampled,
                         const oracle_u128 csum_in[17], const oracle_u128 q_in[18], oracle_result *res) {
  memset(res, 0, sizeof(*res));
  res->n = n;
  res->m = m;
  res->p = p;
  res->seed = seed;
  res->sampled = sampled;
  i128 csum[17];
  u128 q[18];
  for (int i = 0; i < 17; ++i) csum[i] = (i128)(((u128)csum_in[i].hi << 64) | (u128)csum_in[i].lo);
  for (int i = 0; i < 18; ++i) q[i] = ((u128)q_in[i].hi << 64) | (u128)q_in[i].lo;
  return finalize(n, m, p, csum, q, res);
}

/* The int128 -> double conversion used by the finalisation, exposed so that
 * its rounding (to nearest, ties to even, above 2^53) can be pinned. */
double oracle_i128_to_double(uint64_t lo, uint64_t hi) {
  return i128_to_double((i128)(((u128)hi << 64) | (u128)lo));
}

/* Per-edge local quantities for edge (u, v) (micro view, Alg. 2-4);
 * out[0..6] = t, s_u, s_v, r, clique, cycle, f with u the scan side as given. */
int oracle_edge_local(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t u, int32_t v,
                      int64_t out[7]) {
  int64_t m = (int64_t)row_ptr[n] / 2;
  int64_t *psi = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  int64_t du = row_ptr[u + 1] - row_ptr[u];
  int32_t *tlist = (int32_t *)malloc((size_t)(du > 0 ? du : 1) * sizeof(int32_t));
  int32_t *slist = (int32_t *)malloc((size_t)(du > 0 ? du : 1) * sizeof(int32_t));
  if (!psi || !tlist || !slist) {
    free(psi);
    free(tlist);
    free(slist);
    return -1;
  }
  int64_t stamp = 0;
  oracle_local o;
  local_counts(n, m, row_ptr, col, v, u, psi, &stamp, tlist, slist, &o);
  out[0] = o.t;
  out[1] = o.su;
  out[2] = o.sv;
  out[3] = o.r;
  out[4] = o.clique;
  out[5] = o.cycle;
  out[6] = o.f;
  free(psi);
  free(tlist);
  free(slist);
  return 0;
}

/* Sampler over a range of canonical edge ids: mask[e - e0] = 1 iff edge e is
 * sampled; returns the number sampled (used to check full-size runs and to
 * build explicit masks for range estimates). */
uint64_t oracle_sample_mask(uint64_t seed, double p, uint64_t e0, uint64_t e1, uint8_t *mask) {
  uint64_t cnt = 0;
  for (uint64_t e = e0; e < e1; ++e) {
    int s = oracle_edge_sampled(seed, e, p);
    if (mask) mask[e - e0] = (uint8_t)s;
    cnt += (uint64_t)s;
  }
  return cnt;
}

/* ---------------------------------------------------------------------------
 * Micro-level graphlet statistics of single edges (Sec. 3, Alg. 7 with
 * p_e = 1, every neighbour examined once).  y[i-1] is the number of induced
 * k-vertex subgraphs of type G_i whose vertex set holds both ends of e
 * (k = 2, 3, 4): G1 = 1 (e itself), and G2, G6, G17 (no edges) are 0.
 *
 * Plainly: mark u, v, T_e, S_u, S_v, then walk Gamma(w) of every w in
 * T_e u S_u u S_v and tally where each neighbour r falls (T_e, S_u, S_v, or
 * R = the vertices adjacent to neither end).  With those tallies every
 * 4-vertex graphlet containing e is counted by the role e plays in it:
 *   G7  4-clique       : edges inside T_e
 *   G8  chordal cycle  : e the chord: C(t,2) - k4; e on the rim: edges T_e-S
 *   G9  tailed triangle: e the tail: edges inside S_u and inside S_v;
 *                        e next to the tail: t*s - edges T_e-S;
 *                        e opposite the tail: edges T_e-R
 *   G10 4-cycle        : edges S_u-S_v
 *   G11 3-star         : C(s_u,2) - e(S_u) + C(s_v,2) - e(S_v)
 *   G12 4-path         : e the middle: s_u s_v - e(S_u,S_v); e an end: edges S-R
 *   G13 triangle + 1   : t*r - edges T_e-R
 *   G14 2-star + 1     : s*r - edges S-R
 *   G15 2 edges        : edges inside R
 *   G16 1 edge         : C(r,2) - edges inside R
 * where edges inside R = (edges sharing no end with e) - (edges inside
 * T_e u S) - (edges T_e-R) - (edges S-R).
 * The rows are pinned to a brute-force enumeration of the subsets that hold
 * both ends of e, and their column sums to (edges of G_i) x (count of G_i).
 * ------------------------------------------------------------------------ */
enum { MK_T = 1, MK_SU = 2, MK_SV = 3, MK_END = 4 };

static void micro_edge(int64_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, int32_t u, int32_t v,
                       int64_t *tag, int64_t *stamp, int64_t y[17]) {
  const int64_t base = *stamp;
  *stamp += 8;
  /* tag values: base + MK_* (anything below base is "unmarked") */
  for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) tag[col[j]] = base + MK_SV;
  int64_t t = 0, su = 0, sv = 0;
  for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
    const int32_t w = col[j];
    if (w == v) continue;
    if (tag[w] == base + MK_SV) {
      tag[w] = base + MK_T;
      ++t;
    } else {
      tag[w] = base + MK_SU;
      ++su;
    }
  }
  tag[u] = base + MK_END;
  tag[v] = base + MK_END;
  sv = (row_ptr[v + 1] - row_ptr[v]) - 1 - t;
  const int64_t du = row_ptr[u + 1] - row_ptr[u], dv = row_ptr[v + 1] - row_ptr[v];
  /* tallies: [kind of w][kind of r] for kinds T, S_u, S_v, R */
  int64_t tally[4][5];
  memset(tally, 0, sizeof(tally));
  for (int side = 0; side < 2; ++side) {
    const int32_t x = side == 0 ? u : v;
    for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j) {
      const int32_t w = col[j];
      const int64_t tw = tag[w];
      if (tw == base + MK_END) continue;
      if (side == 1 && tw == base + MK_T) continue; /* T_e members are visited from u */
      const int kw = (int)(tw - base); /* MK_T, MK_SU or MK_SV */
      for (int64_t k = row_ptr[w]; k < row_ptr[w + 1]; ++k) {
        const int64_t tr = tag[col[k]];
        int kr;
        if (tr == base + MK_END) continue; /* links to u or v */
        if (tr >= base) kr = (int)(tr - base);
        else kr = 0; /* R */
        tally[kw][kr] += 1;
      }
    }
  }
  const int64_t r = n - (du + dv - t);
  const int64_t s = su + sv;
  const int64_t k4 = tally[MK_T][MK_T] / 2;
  const int64_t ts = tally[MK_T][MK_SU] + tally[MK_T][MK_SV];
  const int64_t tr_ = tally[MK_T][0];
  const int64_t esu = tally[MK_SU][MK_SU] / 2, esv = tally[MK_SV][MK_SV] / 2;
  const int64_t cyc = tally[MK_SU][MK_SV];
  const int64_t sr = tally[MK_SU][0] + tally[MK_SV][0];
  const int64_t f = m - du - dv + 1;
  const int64_t inside = k4 + ts + esu + esv + cyc; /* edges inside T_e u S */
  const int64_t er = f - inside - tr_ - sr;
  for (int i = 0; i < 17; ++i) y[i] = 0;
  y[0] = 1;
  y[2] = t;
  y[3] = s;
  y[4] = r;
  y[6] = k4;
  y[7] = t * (t - 1) / 2 - k4 + ts;
  y[8] = esu + esv + (t * s - ts) + tr_;
  y[9] = cyc;
  y[10] = su * (su - 1) / 2 - esu + sv * (sv - 1) / 2 - esv;
  y[11] = su * sv - cyc + sr;
  y[12] = t * r - tr_;
  y[13] = s * r - sr;
  y[14] = er;
  y[15] = r * (r - 1) / 2 - er;
}

/* Rows for the edges (us[k], vs[k]), k < count; out is count x 17. */
int oracle_micro(int64_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *us, const int32_t *vs,
                 int64_t count, int64_t *out) {
  const int64_t m = (int64_t)row_ptr[n] / 2;
  int64_t *tag = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  if (!tag) return -1;
  int64_t stamp = 8;
  for (int64_t k = 0; k < count; ++k) micro_edge(n, m, row_ptr, col, us[k], vs[k], tag, &stamp, out + 17 * k);
  free(tag);
  return 0;
}

/* The 64-bit Philox output (x1:x0) of every edge id in [e0, e1): the key
 * whose top 53 bits are the edge's uniform (fixed-size samples take the K
 * smallest keys). */
void oracle_philox_keys(uint64_t seed, uint64_t e0, uint64_t e1, uint64_t *out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (uint64_t e = e0; e < e1; ++e) {
    uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), 0u, 0u};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    out[e - e0] = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
  }
}
