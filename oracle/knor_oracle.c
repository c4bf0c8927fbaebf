/*
 * knor_oracle.c -- plain, slow, obviously correct FP64 Lloyd's k-means and
 * its MTI-pruned variant.  TEST INFRASTRUCTURE ONLY: the GPU library never
 * links, calls or includes this file; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark use it.
 *
 * Compile with -O2 -ffp-contract=off (no fused multiply-add, no fast-math) so
 * every operation below is one correctly rounded IEEE-754 binary64 operation.
 * OpenMP (if enabled) splits loops over independent points or clusters only;
 * every result is independent of the thread count.
 *
 * Paper: Mhembere et al., "knor: A NUMA-Optimized In-Memory, Distributed and
 * Semi-External-Memory k-means Library" (HPDC'17), arXiv 1606.08905.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - distance: squared Euclidean D(x,c) = sum_i (x_i - c_i)^2 accumulated in
 *    index order from +0.0 (Section "Nomenclature", metric d = sqrt(D)); the
 *    argmin is taken over D.
 *  - assignment: scan centroids in ascending index and replace only on a
 *    strict "<" (Algorithm 1, the nearest-centroid loop), so the lowest index
 *    wins a tie.
 *  - update: the centroid is the mean of its members (Section "Parallel
 *    Lloyd's Algorithm", Phase II).  Summation order: members in increasing
 *    point index, leaves of LEAF=64 consecutive members summed left to right
 *    starting from the first member's value, leaf sums combined by the
 *    pairwise tree Pair(s[0:m]) = Pair(s[0:h]) + Pair(s[h:m]), h the largest
 *    power of two below m; then one correctly rounded division by the count.
 *    An empty cluster keeps its previous centroid.  A second reading,
 *    oracle_update_exact, rounds the exact mean once (ties to even), which
 *    makes the centroid independent of any summation order.
 *  - loop: stop when #changed labels <= tol * n, or after max_iters.
 *  - MTI (Section "Minimal Triangle Inequality (MTI) Pruning"): one upper
 *    bound u per point, drift f(c) = d(c^t, c^{t-1}), centroid-pair distances
 *    CC, s(c) = 1/2 min_{j != c} CC(c, j) (Elkan's Lemma 1 factor 1/2), with
 *    strict tests and a relative margin ETA so that every pruned comparison
 *    is decided by a gap far above FP64 rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LEAF 64
#define ETA 1e-12

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_MEM = 2 };

/* ------------------------------------------------------------------------ */
/* distance (Section "Nomenclature")                                         */
/* ------------------------------------------------------------------------ */

double oracle_dist2(const double* x, const double* c, int d) {
  double acc = 0.0;
  for (int i = 0; i < d; ++i) {
    double t = x[i] - c[i];
    double t2 = t * t;
    acc = acc + t2;
  }
  return acc;
}

/* ------------------------------------------------------------------------ */
/* assignment (Algorithm 1, nearest-centroid loop)                          */
/* ------------------------------------------------------------------------ */

static int32_t nearest(const double* x, const double* C, int d, int k,
                       double* best_out) {
  double best = INFINITY;
  int32_t a = -1;
  for (int j = 0; j < k; ++j) {
    double D = oracle_dist2(x, C + (size_t)j * d, d);
    if (D < best) { best = D; a = j; }
  }
  *best_out = best;
  return a;
}

/* labels[p] = argmin_j D(x_p, c_j) (lowest index on ties); dist2[p] = that D
 * (dist2 may be NULL). */
int oracle_assign(const double* X, int64_t n, int d, const double* C, int k,
                  int32_t* labels, double* dist2) {
  if (!X || !C || !labels || n < 0 || d < 1 || k < 1) return OR_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n; ++p) {
    double b;
    labels[p] = nearest(X + (size_t)p * d, C, d, k, &b);
    if (dist2) dist2[p] = b;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* canonical sums                                                            */
/* ------------------------------------------------------------------------ */

/* Pair(s[0:m]) over m vectors of length d stored row-major in s; result in
 * out.  Recursive form of the definition. */
static void pair_tree(const double* s, int64_t m, int d, double* out) {
  if (m == 1) {
    memcpy(out, s, sizeof(double) * (size_t)d);
    return;
  }
  int64_t h = 1;
  while (h * 2 < m) h *= 2;              /* largest power of two < m */
  double* l = (double*)malloc(sizeof(double) * (size_t)d);
  double* r = (double*)malloc(sizeof(double) * (size_t)d);
  pair_tree(s, h, d, l);
  pair_tree(s + (size_t)h * d, m - h, d, r);
  for (int i = 0; i < d; ++i) out[i] = l[i] + r[i];
  free(l);
  free(r);
}

/* Canonical sum of the rows X[idx[0..cnt-1]] (idx increasing). */
static void canonical_row_sum(const double* X, int d, const int64_t* idx,
                              int64_t cnt, double* out) {
  int64_t nleaf = (cnt + LEAF - 1) / LEAF;
  double* leaves = (double*)malloc(sizeof(double) * (size_t)nleaf * d);
  for (int64_t L = 0; L < nleaf; ++L) {
    double* s = leaves + (size_t)L * d;
    int64_t m0 = L * LEAF, m1 = m0 + LEAF < cnt ? m0 + LEAF : cnt;
    const double* x0 = X + (size_t)idx[m0] * d;
    for (int i = 0; i < d; ++i) s[i] = x0[i];
    for (int64_t m = m0 + 1; m < m1; ++m) {
      const double* x = X + (size_t)idx[m] * d;
      for (int i = 0; i < d; ++i) s[i] = s[i] + x[i];
    }
  }
  pair_tree(leaves, nleaf, d, out);
  free(leaves);
}

/* Canonical sum of a scalar sequence v[0..n-1] (same leaf + tree rule). */
double oracle_canonical_sum(const double* v, int64_t n) {
  if (n <= 0) return 0.0;
  int64_t nleaf = (n + LEAF - 1) / LEAF;
  double* leaves = (double*)malloc(sizeof(double) * (size_t)nleaf);
#pragma omp parallel for schedule(static)
  for (int64_t L = 0; L < nleaf; ++L) {
    int64_t m0 = L * LEAF, m1 = m0 + LEAF < n ? m0 + LEAF : n;
    double s = v[m0];
    for (int64_t m = m0 + 1; m < m1; ++m) s = s + v[m];
    leaves[L] = s;
  }
  double out;
  pair_tree(leaves, nleaf, 1, &out);
  free(leaves);
  return out;
}

/* ------------------------------------------------------------------------ */
/* update (Phase II / Algorithm 1 merge)                                     */
/* ------------------------------------------------------------------------ */

/* C_out[j] = mean of the rows with labels == j, in the canonical order; an
 * empty cluster copies C_prev[j].  counts (may be NULL) gets |members|. */
int oracle_update(const double* X, int64_t n, int d, const int32_t* labels,
                  int k, const double* C_prev, double* C_out,
                  int64_t* counts) {
  if (!X || !labels || !C_prev || !C_out || n < 0 || d < 1 || k < 1)
    return OR_ERR_ARG;
  for (int64_t p = 0; p < n; ++p)
    if (labels[p] < 0 || labels[p] >= k) return OR_ERR_ARG;
  int64_t* cnt = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
  int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  if (!cnt || !members) { free(cnt); free(members); return OR_ERR_MEM; }
  for (int64_t p = 0; p < n; ++p) cnt[labels[p] + 1]++;
  for (int j = 0; j < k; ++j) cnt[j + 1] += cnt[j];          /* offsets */
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  for (int j = 0; j < k; ++j) fill[j] = cnt[j];
  for (int64_t p = 0; p < n; ++p) members[fill[labels[p]]++] = p;  /* stable */
  free(fill);
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < k; ++j) {
    int64_t nj = cnt[j + 1] - cnt[j];
    double* c = C_out + (size_t)j * d;
    if (nj == 0) {
      memcpy(c, C_prev + (size_t)j * d, sizeof(double) * (size_t)d);
    } else {
      canonical_row_sum(X, d, members + cnt[j], nj, c);
      double dn = (double)nj;
      for (int i = 0; i < d; ++i) c[i] = c[i] / dn;
    }
  }
  if (counts)
    for (int j = 0; j < k; ++j) counts[j] = cnt[j + 1] - cnt[j];
  free(cnt);
  free(members);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* update, second reading: the exactly rounded mean                          */
/* ------------------------------------------------------------------------ */

/* The centroid as the mean of its members with a single rounding: the
 * exact sum of the members' values divided by their count, rounded to the
 * nearest double (ties to even).  Unlike the canonical sum above it does not
 * depend on the order of the members.
 *
 * The exact sum is kept as two non-negative fixed-point integers (the sums
 * of the positive and of the negative terms) in units of 2^-1074, the
 * spacing of the smallest doubles: every finite double is an integer in
 * these units below 2^2098, and XW 64-bit words leave room for 2^63 terms. */
#define XW 34

typedef struct {
  uint64_t pos[XW], neg[XW];
} xacc;

/* w += m * 2^shift (m < 2^64) */
static void xw_add_shifted(uint64_t* w, uint64_t m, int64_t shift) {
  int64_t i = shift / 64;
  int off = (int)(shift % 64);
  uint64_t lo = m << off;
  uint64_t hi = off ? (m >> (64 - off)) : 0;
  uint64_t carry = 0;
  for (int64_t j = i; j < XW; ++j) {
    uint64_t add = (j == i) ? lo : (j == i + 1 ? hi : 0);
    uint64_t t = w[j] + add;
    uint64_t c1 = t < add;
    uint64_t t2 = t + carry;
    uint64_t c2 = t2 < carry;
    w[j] = t2;
    carry = c1 | c2;
    if (j > i && !carry && j >= i + 1) break;
  }
}

static void xacc_add(xacc* a, double v) {
  if (v == 0.0) return;
  int e;
  double f = frexp(fabs(v), &e);              /* |v| = f 2^e, f in [0.5, 1) */
  uint64_t m = (uint64_t)ldexp(f, 53);        /* |v| = m 2^(e-53), exactly  */
  int64_t shift = (int64_t)e - 53 + 1074;     /* in units of 2^-1074        */
  if (shift < 0) {                            /* subnormal: the low bits of */
    m >>= -shift;                             /* m are zero                 */
    shift = 0;
  }
  xw_add_shifted(v > 0 ? a->pos : a->neg, m, shift);
}

/* Bit b of a little-endian word array. */
static int xw_bit(const uint64_t* w, int64_t b) {
  return (int)((w[b / 64] >> (b % 64)) & 1u);
}

/* RN((pos - neg) * 2^-1074 / n), n >= 1. */
static double xacc_mean(const xacc* a, int64_t n) {
  uint64_t mag[XW];
  /* mag = |pos - neg|, sign from the comparison */
  int cmp = 0;
  for (int j = XW - 1; j >= 0 && cmp == 0; --j)
    cmp = a->pos[j] > a->neg[j] ? 1 : (a->pos[j] < a->neg[j] ? -1 : 0);
  if (cmp == 0) return 0.0;
  const uint64_t* big = cmp > 0 ? a->pos : a->neg;
  const uint64_t* small = cmp > 0 ? a->neg : a->pos;
  uint64_t borrow = 0;
  for (int j = 0; j < XW; ++j) {
    uint64_t t = big[j] - small[j];
    uint64_t b1 = big[j] < small[j];
    uint64_t t2 = t - borrow;
    uint64_t b2 = t < borrow;
    mag[j] = t2;
    borrow = b1 | b2;
  }
  /* q = floor(mag * 2^128 / n), units 2^-1202; rem != 0 marks a remainder */
  enum { QW = XW + 2 };
  uint64_t num[QW], q[QW];
  num[0] = 0;
  num[1] = 0;
  for (int j = 0; j < XW; ++j) num[j + 2] = mag[j];
  unsigned __int128 rem = 0;
  for (int j = QW - 1; j >= 0; --j) {
    unsigned __int128 cur = (rem << 64) | num[j];
    q[j] = (uint64_t)(cur / (uint64_t)n);
    rem = cur % (uint64_t)n;
  }
  int64_t top = -1;
  for (int64_t b = (int64_t)QW * 64 - 1; b >= 0; --b)
    if (xw_bit(q, b)) { top = b; break; }
  if (top < 0) return cmp > 0 ? 0.0 : -0.0;   /* below half of 2^-1202 ... */
  /* result ulp: 2^(top - 52) in q's units, at least 2^-1074 = 2^128 units */
  int64_t sh = top - 52 > 128 ? top - 52 : 128;
  uint64_t mant = 0;
  for (int64_t b = top; b >= sh; --b) mant = (mant << 1) | (uint64_t)xw_bit(q, b);
  int round = sh >= 1 ? xw_bit(q, sh - 1) : 0;
  int sticky = rem != 0;
  for (int64_t b = sh - 2; b >= 0 && !sticky; --b) sticky = xw_bit(q, b);
  if (round && (sticky || (mant & 1u))) mant += 1;
  double r = ldexp((double)mant, (int)(sh - 1202));
  return cmp > 0 ? r : -r;
}

/* C_out[j] = the exactly rounded mean of the rows with labels == j; an empty
 * cluster copies C_prev[j].  counts (may be NULL) gets |members|. */
int oracle_update_exact(const double* X, int64_t n, int d, const int32_t* labels,
                        int k, const double* C_prev, double* C_out,
                        int64_t* counts) {
  if (!X || !labels || !C_prev || !C_out || n < 0 || d < 1 || k < 1)
    return OR_ERR_ARG;
  for (int64_t p = 0; p < n; ++p)
    if (labels[p] < 0 || labels[p] >= k) return OR_ERR_ARG;
  int64_t* cnt = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  if (!cnt) return OR_ERR_MEM;
  for (int64_t p = 0; p < n; ++p) cnt[labels[p]]++;
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < k; ++j) {
    double* c = C_out + (size_t)j * d;
    if (cnt[j] == 0) {                       /* empty: keep the previous */
      for (int i = 0; i < d; ++i) c[i] = C_prev[(size_t)j * d + i];
      continue;
    }
    xacc* acc = (xacc*)calloc((size_t)d, sizeof(xacc));
    for (int64_t p = 0; p < n; ++p)
      if (labels[p] == j)
        for (int i = 0; i < d; ++i) xacc_add(&acc[i], X[(size_t)p * d + i]);
    for (int i = 0; i < d; ++i) c[i] = xacc_mean(&acc[i], cnt[j]);
    free(acc);
  }
  if (counts)
    for (int j = 0; j < k; ++j) counts[j] = cnt[j];
  free(cnt);
  return OR_OK;
}

/* The exactly rounded mean of v[0..n) (n >= 1). */
double oracle_exact_mean(const double* v, int64_t n) {
  xacc a;
  memset(&a, 0, sizeof a);
  for (int64_t i = 0; i < n; ++i) xacc_add(&a, v[i]);
  return xacc_mean(&a, n);
}

/* ------------------------------------------------------------------------ */
/* Lloyd's loop                                                              */
/* ------------------------------------------------------------------------ */

/* Per-iteration record.  Every pointer may be NULL; arrays hold max_iters
 * entries (label_hist: max_iters * n). */
typedef struct {
  int32_t iters;
  int32_t converged;
  int64_t* changed;       /* labels that differ from the previous iteration */
  double* objective;      /* J_t = canonical sum over points of D(x, c_a)   */
  int64_t* ndist;         /* point-centroid distances evaluated             */
  int64_t* pruned1;       /* points decided by Clause 1 (MTI only)          */
  int32_t* label_hist;    /* labels after the assignment of each iteration  */
  int32_t bound_violations; /* MTI only: times u < d(x, c_a) was observed   */
} oracle_trace;

static int fit_common(const double* X, int64_t n, int d, int k,
                      const double* C0, int max_iters, double tol, int mti,
                      int exact_mean, double* C_out, int32_t* labels_out,
                      oracle_trace* tr);

int oracle_fit(const double* X, int64_t n, int d, int k, const double* C0,
               int max_iters, double tol, double* C_out, int32_t* labels_out,
               oracle_trace* tr) {
  return fit_common(X, n, d, k, C0, max_iters, tol, 0, 0, C_out, labels_out, tr);
}

int oracle_mti_fit(const double* X, int64_t n, int d, int k, const double* C0,
                   int max_iters, double tol, double* C_out,
                   int32_t* labels_out, oracle_trace* tr) {
  return fit_common(X, n, d, k, C0, max_iters, tol, 1, 0, C_out, labels_out, tr);
}

/* Either loop with either update: exact_mean = 1 takes the exactly rounded
 * mean (oracle_update_exact) instead of the canonical sum. */
int oracle_fit_ex(const double* X, int64_t n, int d, int k, const double* C0,
                  int max_iters, double tol, int mti, int exact_mean,
                  double* C_out, int32_t* labels_out, oracle_trace* tr) {
  return fit_common(X, n, d, k, C0, max_iters, tol, mti ? 1 : 0,
                    exact_mean ? 1 : 0, C_out, labels_out, tr);
}

/* MTI assignment of one point for iteration t >= 1 (Clauses 1-3).
 * a, u: in/out label and upper bound (u >= d(x, c_a) on entry).
 * s: s(c) = 1/2 min_{j != c} CC(c, j).  CC: k x k centroid distances.
 * Returns the number of distances computed; *p1 = 1 if Clause 1 decided. */
static int64_t mti_point(const double* x, const double* C, int d, int k,
                         const double* CC, const double* s, int32_t* a_io,
                         double* u_io, double* Dbest_out, int* p1,
                         int* violation) {
  int32_t a0 = *a_io, a = a0;
  double u = *u_io;
  int64_t nd = 0;
  *p1 = 0;
  /* Clause 1: u <= s(a) with margin -> no distance at all. */
  if (u * (1.0 + ETA) < s[a0] * (1.0 - ETA)) {
    *p1 = 1;
    *Dbest_out = NAN;
    return 0;
  }
  int tight = 0;
  double Da = NAN;
  for (int j = 0; j < k; ++j) {
    if (j == a0) continue;
    /* Clause 2: u <= 1/2 d(c_a, c_j) -> skip c_j. */
    if (u * (1.0 + ETA) < 0.5 * CC[(size_t)a * k + j] * (1.0 - ETA)) continue;
    if (!tight) {
      /* Clause 3: U(u) fully tightens the bound, then re-test Clause 2. */
      Da = oracle_dist2(x, C + (size_t)a0 * d, d);
      ++nd;
      double ut = sqrt(Da);
      if (ut > u * (1.0 + ETA)) *violation = 1;
      u = ut;
      tight = 1;
      if (u * (1.0 + ETA) < 0.5 * CC[(size_t)a * k + j] * (1.0 - ETA)) continue;
    }
    double Dj = oracle_dist2(x, C + (size_t)j * d, d);
    ++nd;
    if (Dj < Da || (Dj == Da && j < a)) {
      a = j;
      Da = Dj;
      u = sqrt(Dj);
    }
  }
  if (!tight) {
    /* every other centroid was pruned by Clause 2 with the loose bound */
    *Dbest_out = NAN;
  } else {
    *Dbest_out = Da;
  }
  *a_io = a;
  *u_io = u;
  return nd;
}

static int fit_common(const double* X, int64_t n, int d, int k,
                      const double* C0, int max_iters, double tol, int mti,
                      int exact_mean, double* C_out, int32_t* labels_out,
                      oracle_trace* tr) {
  if (!X || !C0 || !C_out || !labels_out || n < 1 || d < 1 || k < 1 ||
      k > n || max_iters < 1 || !(tol >= 0.0 && tol < 1.0))
    return OR_ERR_ARG;
  size_t kd = (size_t)k * d;
  double* C = (double*)malloc(sizeof(double) * kd);
  double* Cn = (double*)malloc(sizeof(double) * kd);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* an = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  double* D = (double*)malloc(sizeof(double) * (size_t)n);
  double* u = mti ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
  double* CC = mti ? (double*)malloc(sizeof(double) * (size_t)k * k) : NULL;
  double* s = mti ? (double*)malloc(sizeof(double) * (size_t)k) : NULL;
  double* drift = mti ? (double*)malloc(sizeof(double) * (size_t)k) : NULL;
  if (!C || !Cn || !a || !an || !D || (mti && (!u || !CC || !s || !drift))) {
    free(C); free(Cn); free(a); free(an); free(D); free(u); free(CC); free(s);
    free(drift);
    return OR_ERR_MEM;
  }
  memcpy(C, C0, sizeof(double) * kd);
  int converged = 0, t;
  int violation = 0;
  const int want_obj = tr && tr->objective;
  for (t = 0; t < max_iters; ++t) {
    int64_t nd = 0, np1 = 0;
    if (!mti || t == 0) {
      oracle_assign(X, n, d, C, k, an, D);
      nd = (int64_t)n * k;
      if (mti)
        for (int64_t p = 0; p < n; ++p) u[p] = sqrt(D[p]);
    } else {
#pragma omp parallel for schedule(static) reduction(+ : nd, np1)
      for (int64_t p = 0; p < n; ++p) {
        int32_t ap = a[p];
        double up = u[p], Db;
        int p1, viol = 0;
        nd += mti_point(X + (size_t)p * d, C, d, k, CC, s, &ap, &up, &Db, &p1,
                        &viol);
        np1 += p1;
        if (viol) {
#pragma omp atomic write
          violation = 1;
        }
        an[p] = ap;
        u[p] = up;
        /* the traced objective needs D(x, c_a); recompute it where pruning
           skipped it (trace only, not counted as work of the method) */
        if (want_obj && isnan(Db))
          Db = oracle_dist2(X + (size_t)p * d, C + (size_t)ap * d, d);
        D[p] = Db;
      }
    }
    int64_t changed = 0;
    if (t == 0) {
      changed = n;
    } else {
      for (int64_t p = 0; p < n; ++p) changed += (an[p] != a[p]);
    }
    memcpy(a, an, sizeof(int32_t) * (size_t)n);
    if (tr) {
      if (tr->changed) tr->changed[t] = changed;
      if (tr->objective) tr->objective[t] = oracle_canonical_sum(D, n);
      if (tr->ndist) tr->ndist[t] = nd;
      if (tr->pruned1) tr->pruned1[t] = np1;
      if (tr->label_hist)
        memcpy(tr->label_hist + (size_t)t * n, a, sizeof(int32_t) * (size_t)n);
    }
    if (exact_mean)
      oracle_update_exact(X, n, d, a, k, C, Cn, NULL);
    else
      oracle_update(X, n, d, a, k, C, Cn, NULL);
    if (mti) {
      /* drift f(c) = d(c^{t+1}, c^t); centroid-pair distances; s(c). */
      for (int j = 0; j < k; ++j)
        drift[j] = sqrt(oracle_dist2(Cn + (size_t)j * d, C + (size_t)j * d, d));
#pragma omp parallel for schedule(static)
      for (int i = 0; i < k; ++i) {
        CC[(size_t)i * k + i] = 0.0;
        for (int j = 0; j < k; ++j)
          if (j != i)
            CC[(size_t)i * k + j] =
                sqrt(oracle_dist2(Cn + (size_t)i * d, Cn + (size_t)j * d, d));
      }
      for (int i = 0; i < k; ++i) {
        double m = INFINITY;
        for (int j = 0; j < k; ++j)
          if (j != i && CC[(size_t)i * k + j] < m) m = CC[(size_t)i * k + j];
        s[i] = 0.5 * m;
      }
      for (int64_t p = 0; p < n; ++p) u[p] = u[p] + drift[a[p]];
    }
    double* tmp = C; C = Cn; Cn = tmp;
    if ((double)changed <= tol * (double)n) { converged = 1; ++t; break; }
  }
  memcpy(C_out, C, sizeof(double) * kd);
  memcpy(labels_out, a, sizeof(int32_t) * (size_t)n);
  if (tr) {
    tr->iters = converged ? t : max_iters;
    tr->converged = converged;
    tr->bound_violations = violation;
  }
  free(C); free(Cn); free(a); free(an); free(D); free(u); free(CC); free(s);
  free(drift);
  return OR_OK;
}

/* Centroid-pair bounds for a given centroid set: s[j] = 1/2 min_{i != j}
 * d(c_i, c_j) (k >= 2; with k == 1, s = +inf). */
int oracle_cc_bounds(const double* C, int k, int d, double* s) {
  if (!C || !s || k < 1 || d < 1) return OR_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < k; ++i) {
    double m = INFINITY;
    for (int j = 0; j < k; ++j) {
      if (j == i) continue;
      double v = sqrt(oracle_dist2(C + (size_t)i * d, C + (size_t)j * d, d));
      if (v < m) m = v;
    }
    s[i] = 0.5 * m;
  }
  return OR_OK;
}

/* Objective for given labels: canonical sum over points of D(x_p, c_{l_p}). */
double oracle_objective(const double* X, int64_t n, int d, const double* C,
                        const int32_t* labels) {
  double* D = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n; ++p)
    D[p] = oracle_dist2(X + (size_t)p * d, C + (size_t)labels[p] * d, d);
  double s = oracle_canonical_sum(D, n);
  free(D);
  return s;
}

/* Thread count of the later parallel regions (no effect on any result: every
 * loop is statically scheduled over fixed point blocks or per cluster). */
void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
