/*
 * Seeded synthetic graph generators producing undirected simple graphs as
 * int32 CSR with strictly increasing adjacency lists.
 *
 * This file is input generation only: it draws random graphs with the
 * shapes of the workloads (Erdos-Renyi, Chung-Lu power law, R-MAT) and holds
 * none of the graphlet-counting arithmetic.  Both the CPU oracle and the GPU
 * path consume what it writes.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded through
 * splitmix64, so a (generator, parameters, seed) triple names one graph on
 * every machine.
 *
 * Every entry point writes row_ptr[n+1] and col[col_cap] supplied by the
 * caller and returns the number of CSR entries (2M), or a negative value:
 *   -1 bad argument, -2 out of memory, -3 col_cap too small, -4 more than
 *   2^31-1 CSR entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t s[4];
} gg_rng;

static uint64_t gg_splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static void gg_seed(gg_rng *r, uint64_t seed, uint64_t stream) {
  uint64_t x = seed ^ (stream * 0xd1b54a32d192ed03ULL);
  for (int i = 0; i < 4; ++i) r->s[i] = gg_splitmix64(&x);
}

static inline uint64_t gg_rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t gg_next(gg_rng *r) {
  uint64_t *s = r->s;
  uint64_t res = gg_rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = gg_rotl(s[3], 45);
  return res;
}

/* uniform in [0,1) with 53 random bits */
static inline double gg_u01(gg_rng *r) { return (double)(gg_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n) (Lemire's multiply-shift, with rejection) */
static inline uint64_t gg_below(gg_rng *r, uint64_t n) {
  unsigned __int128 m = (unsigned __int128)gg_next(r) * n;
  uint64_t lo = (uint64_t)m;
  if (lo < n) {
    uint64_t thr = (0 - n) % n;
    while (lo < thr) {
      m = (unsigned __int128)gg_next(r) * n;
      lo = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static void sort_i32(int32_t *v, int64_t len) {
  if (len < 24) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t x = v[i];
      int64_t j = i - 1;
      while (j >= 0 && v[j] > x) {
        v[j + 1] = v[j];
        --j;
      }
      v[j + 1] = x;
    }
  } else {
    qsort(v, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

/*
 * Build the CSR of the simple undirected graph spanned by npairs endpoint
 * pairs: self-loops are dropped, duplicates merged, both directions stored.
 */
static int64_t gg_pairs_to_csr(int64_t n, int64_t npairs, const int32_t *pa, const int32_t *pb,
                               int32_t *row_ptr, int32_t *col, int64_t col_cap) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
  int64_t total = 0;
  for (int64_t i = 0; i < npairs; ++i) {
    if (pa[i] == pb[i]) continue;
    cnt[pa[i] + 1]++;
    cnt[pb[i] + 1]++;
    total += 2;
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int32_t *tmp = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!tmp || !pos) {
    free(cnt);
    free(tmp);
    free(pos);
    return -2;
  }
  memcpy(pos, cnt, (size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < npairs; ++i) {
    int32_t a = pa[i], b = pb[i];
    if (a == b) continue;
    tmp[pos[a]++] = b;
    tmp[pos[b]++] = a;
  }
  free(pos);
  int64_t out = 0;
  row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t beg = cnt[v], end = cnt[v + 1];
    sort_i32(tmp + beg, end - beg);
    int64_t last = -1;
    for (int64_t j = beg; j < end; ++j) {
      if (tmp[j] == last) continue;
      last = tmp[j];
      if (out >= col_cap) {
        free(cnt);
        free(tmp);
        return -3;
      }
      col[out++] = tmp[j];
    }
    if (out > INT32_MAX) {
      free(cnt);
      free(tmp);
      return -4;
    }
    row_ptr[v + 1] = (int32_t)out;
  }
  free(cnt);
  free(tmp);
  return out;
}

/*
 * Erdos-Renyi G(n, q): every unordered pair independently present with
 * probability q.  Pairs are visited in lexicographic order by geometric
 * skips, which draws the same distribution as one Bernoulli per pair.
 */
int64_t gg_erdos_renyi(int64_t n, double q, uint64_t seed, int32_t *row_ptr, int32_t *col,
                       int64_t col_cap) {
  if (n < 0 || n > INT32_MAX || !(q >= 0.0 && q <= 1.0)) return -1;
  gg_rng r;
  gg_seed(&r, seed, 1);
  int64_t cap = col_cap / 2 + 1;
  int32_t *pa = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  int32_t *pb = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  if (!pa || !pb) {
    free(pa);
    free(pb);
    return -2;
  }
  int64_t np = 0;
  if (q > 0.0 && n > 1) {
    double lq = log1p(-q);
    int64_t i = 0, j = 0; /* current pair is (i, j) with j > i; start before (0,1) */
    for (;;) {
      int64_t skip;
      if (q >= 1.0) {
        skip = 0;
      } else {
        double u = 1.0 - gg_u01(&r); /* (0,1] */
        double g = floor(log(u) / lq);
        skip = g > 9.0e15 ? (int64_t)9.0e15 : (int64_t)g;
      }
      /* advance (i, j) by skip+1 pairs */
      int64_t adv = skip + 1;
      while (adv > 0) {
        int64_t room = n - 1 - j; /* pairs left in row i after j */
        if (adv <= room) {
          j += adv;
          adv = 0;
        } else {
          adv -= room;
          ++i;
          j = i;
          if (i >= n - 1) break;
        }
      }
      if (i >= n - 1) break;
      if (np >= cap) {
        free(pa);
        free(pb);
        return -3;
      }
      pa[np] = (int32_t)i;
      pb[np] = (int32_t)j;
      ++np;
    }
  }
  int64_t res = gg_pairs_to_csr(n, np, pa, pb, row_ptr, col, col_cap);
  free(pa);
  free(pb);
  return res;
}

/*
 * Chung-Lu power law: vertex weights w_i = min(c (i+1)^(-1/(gamma-1)), cap)
 * with the scale c solved by bisection so that the mean weight equals
 * avg_deg; round(n avg_deg / 2) edges are drawn with both endpoints
 * proportional to w (Vose alias table); loops dropped, duplicates merged.
 */
int64_t gg_chung_lu(int64_t n, double avg_deg, double gamma, double cap, uint64_t seed,
                    int32_t *row_ptr, int32_t *col, int64_t col_cap) {
  if (n < 1 || n > INT32_MAX || !(gamma > 1.0) || !(avg_deg > 0.0) || !(cap > 0.0)) return -1;
  double beta = 1.0 / (gamma - 1.0);
  double *w = (double *)malloc((size_t)n * sizeof(double));
  if (!w) return -2;
  double target = avg_deg;
  if (target > cap) target = cap;
  double lo = 0.0, hi = 1.0;
  for (;;) { /* grow hi until the mean reaches the target */
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double x = hi * pow((double)(i + 1), -beta);
      s += x < cap ? x : cap;
    }
    if (s / (double)n >= target || hi > 1e300) break;
    hi *= 2.0;
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi), s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double x = mid * pow((double)(i + 1), -beta);
      s += x < cap ? x : cap;
    }
    if (s / (double)n < target)
      lo = mid;
    else
      hi = mid;
    if (hi - lo <= 1e-12 * hi) break;
  }
  double tot = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double x = hi * pow((double)(i + 1), -beta);
    w[i] = x < cap ? x : cap;
    tot += w[i];
  }
  /* Vose alias table */
  double *prob = (double *)malloc((size_t)n * sizeof(double));
  int32_t *alias = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *small = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *large = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!prob || !alias || !small || !large) {
    free(w);
    free(prob);
    free(alias);
    free(small);
    free(large);
    return -2;
  }
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    prob[i] = w[i] * (double)n / tot;
    alias[i] = (int32_t)i;
    if (prob[i] < 1.0)
      small[ns++] = (int32_t)i;
    else
      large[nl++] = (int32_t)i;
  }
  while (ns > 0 && nl > 0) {
    int32_t s = small[--ns], l = large[--nl];
    alias[s] = l;
    prob[l] = prob[l] + prob[s] - 1.0;
    if (prob[l] < 1.0)
      small[ns++] = l;
    else
      large[nl++] = l;
  }
  while (nl > 0) prob[large[--nl]] = 1.0;
  while (ns > 0) prob[small[--ns]] = 1.0;
  free(small);
  free(large);
  free(w);

  int64_t draws = (int64_t)llround((double)n * avg_deg / 2.0);
  int32_t *pa = (int32_t *)malloc((size_t)(draws > 0 ? draws : 1) * sizeof(int32_t));
  int32_t *pb = (int32_t *)malloc((size_t)(draws > 0 ? draws : 1) * sizeof(int32_t));
  if (!pa || !pb) {
    free(prob);
    free(alias);
    free(pa);
    free(pb);
    return -2;
  }
  gg_rng r;
  gg_seed(&r, seed, 2);
  for (int64_t k = 0; k < draws; ++k) {
    for (int e = 0; e < 2; ++e) {
      int64_t i = (int64_t)gg_below(&r, (uint64_t)n);
      int32_t v = gg_u01(&r) < prob[i] ? (int32_t)i : alias[i];
      if (e == 0)
        pa[k] = v;
      else
        pb[k] = v;
    }
  }
  free(prob);
  free(alias);
  int64_t res = gg_pairs_to_csr(n, draws, pa, pb, row_ptr, col, col_cap);
  free(pa);
  free(pb);
  return res;
}

/*
 * R-MAT (Graph500 style, no per-level noise): n = 2^scale vertices,
 * edge_factor * n draws; each draw descends scale levels choosing quadrant
 * (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1) w.p. 1-a-b-c.  With
 * relabel != 0 a seeded random permutation of vertex ids is applied so that
 * vertex id carries no degree information.  Loops dropped, duplicates merged.
 */
int64_t gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, int relabel,
                uint64_t seed, int32_t *row_ptr, int32_t *col, int64_t col_cap) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
    return -1;
  int64_t n = (int64_t)1 << scale;
  int64_t draws = edge_factor * n;
  int32_t *pa = (int32_t *)malloc((size_t)draws * sizeof(int32_t));
  int32_t *pb = (int32_t *)malloc((size_t)draws * sizeof(int32_t));
  if (!pa || !pb) {
    free(pa);
    free(pb);
    return -2;
  }
  gg_rng r;
  gg_seed(&r, seed, 3);
  /* 32-bit thresholds: one 64-bit draw feeds two levels */
  uint64_t ta = (uint64_t)(a * 4294967296.0);
  uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
  uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
  for (int64_t k = 0; k < draws; ++k) {
    uint32_t row = 0, cl = 0;
    uint64_t bits = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      if ((lvl & 1) == 0) bits = gg_next(&r);
      uint64_t x = (lvl & 1) ? (bits >> 32) : (bits & 0xffffffffULL);
      uint32_t rb = x >= tb;
      uint32_t cb = (x >= ta && x < tb) || x >= tc;
      row |= rb << lvl;
      cl |= cb << lvl;
    }
    pa[k] = (int32_t)row;
    pb[k] = (int32_t)cl;
  }
  if (relabel) {
    int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!perm) {
      free(pa);
      free(pb);
      return -2;
    }
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    gg_rng rp;
    gg_seed(&rp, seed, 4);
    for (int64_t i = n - 1; i > 0; --i) {
      int64_t j = (int64_t)gg_below(&rp, (uint64_t)(i + 1));
      int32_t t = perm[i];
      perm[i] = perm[j];
      perm[j] = t;
    }
    for (int64_t k = 0; k < draws; ++k) {
      pa[k] = perm[pa[k]];
      pb[k] = perm[pb[k]];
    }
    free(perm);
  }
  int64_t res = gg_pairs_to_csr(n, draws, pa, pb, row_ptr, col, col_cap);
  free(pa);
  free(pb);
  return res;
}

/* CSR from caller-provided endpoint pairs (used for hand-made test graphs). */
int64_t gg_from_pairs(int64_t n, int64_t npairs, const int32_t *pa, const int32_t *pb,
                      int32_t *row_ptr, int32_t *col, int64_t col_cap) {
  if (n < 0 || n > INT32_MAX) return -1;
  for (int64_t i = 0; i < npairs; ++i)
    if (pa[i] < 0 || pa[i] >= n || pb[i] < 0 || pb[i] >= n) return -1;
  return gg_pairs_to_csr(n, npairs, pa, pb, row_ptr, col, col_cap);
}
