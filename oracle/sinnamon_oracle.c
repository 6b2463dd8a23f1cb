/*
 * FP64 reference ("oracle") for the Sinnamon method of Bruch, Nardini, Ingber
 * and Liberty, "An Approximate Algorithm for Maximum Inner Product Search over
 * Streaming Sparse Vectors" (arXiv 2301.10622).
 *
 * THIS FILE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it. The GPU library never links,
 * includes or calls it, and it shares no code, header or table with that
 * library: its hash, sketch, scoring and selection are written here from the
 * paper alone.
 *
 * Everything is plain, slow and in the paper's order:
 *   - nz(x): the coordinates with a non-zero value (Alg. 1 and Alg. 5, first step).
 *   - h random mappings pi_o: [n] -> [m] (Alg. 5 requirements). The paper does not
 *     say which; here pi_o(j) = mix64(mix64(seed + o) XOR j) mod m with the
 *     SplitMix64 output function of Steele, Lea and Flood (OOPSLA 2014).
 *   - sketching (Alg. 5): u[k] is the largest and l[k] the smallest value among
 *     the coordinates that at least one mapping sends to bucket k. A bucket no
 *     coordinate maps to is written as 0 (the paper is silent; it is never read).
 *     Optionally stored in bfloat16 as the paper does, U rounded up, L down.
 *   - scoring (Alg. 6, T = infinity): the non-zero query coordinates sorted by
 *     |q_j| descending (ties: lower j first); for every document i on the
 *     inverted list of j add q_j * min_o U[pi_o(j)][i] if q_j > 0, else
 *     q_j * max_o L[pi_o(j)][i]. Untouched documents keep score 0.
 *   - exact scoring (Eq. 2 via Alg. 2): the same walk with the true value x_i[j].
 *   - ranking with k' = k (Alg. 7 reduces to Alg. 3): FindLargest with a binary
 *     heap. Ties at equal score are broken by the lower external id.
 *   - ranking with k' >= k (Alg. 7): FindLargest(k') over the estimates, the
 *     exact inner product of each of those k' vectors fetched from the vector
 *     storage, FindLargest(k) over the exact scores.
 *   - the small MLP of the learned threshold filter (not in the paper): dense
 *     layers in FP64 with ReLU, mean squared error, plain back-propagation.
 *
 * Arithmetic is FP64. Inputs are FP32, so every product q_j * x is exact and
 * only the running sums round.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Random mappings pi_o (Alg. 5 requirements)                                 */
/* ------------------------------------------------------------------------- */

uint64_t orc_mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint32_t orc_bucket(uint64_t seed, uint32_t o, uint32_t j, uint32_t m) {
  return (uint32_t)(orc_mix64(orc_mix64(seed + (uint64_t)o) ^ (uint64_t)j) % (uint64_t)m);
}

void orc_bucket_table(uint64_t seed, uint32_t h, uint32_t n, uint32_t m, uint32_t *out) {
  for (uint32_t o = 0; o < h; ++o)
    for (uint32_t j = 0; j < n; ++j) out[(size_t)o * n + j] = orc_bucket(seed, o, j, m);
}

/* ------------------------------------------------------------------------- */
/* Sketching (Alg. 5)                                                          */
/* ------------------------------------------------------------------------- */

/* Alg. 5 exactly as printed: for every bucket k, scan nz(x) for coordinates that
 * some mapping sends to k. O(m * nnz * h); used on small inputs to pin the
 * faster form below. filled[k] is 1 when the set for bucket k is non-empty. */
void orc_sketch_by_bucket(uint32_t nnz, const uint32_t *coords, const float *vals, uint32_t m,
                          uint32_t h, uint64_t seed, double *u, double *l, uint8_t *filled) {
  for (uint32_t k = 0; k < m; ++k) {
    int any = 0;
    double mx = 0.0, mn = 0.0;
    for (uint32_t t = 0; t < nnz; ++t) {
      if (vals[t] == 0.0f) continue; /* not in nz(x) */
      int hit = 0;
      for (uint32_t o = 0; o < h; ++o)
        if (orc_bucket(seed, o, coords[t], m) == k) hit = 1;
      if (!hit) continue;
      double x = (double)vals[t];
      if (!any || x > mx) mx = x;
      if (!any || x < mn) mn = x;
      any = 1;
    }
    u[k] = any ? mx : 0.0;
    l[k] = any ? mn : 0.0;
    if (filled) filled[k] = (uint8_t)any;
  }
}

/* The same sets, visited member by member: every (j, o) pair updates bucket
 * pi_o(j). The max/min over a set does not depend on the visiting order. */
void orc_sketch(uint32_t nnz, const uint32_t *coords, const float *vals, uint32_t m, uint32_t h,
                uint64_t seed, double *u, double *l, uint8_t *filled) {
  uint8_t *any = (uint8_t *)calloc(m, 1);
  for (uint32_t k = 0; k < m; ++k) u[k] = l[k] = 0.0;
  for (uint32_t t = 0; t < nnz; ++t) {
    if (vals[t] == 0.0f) continue;
    double x = (double)vals[t];
    for (uint32_t o = 0; o < h; ++o) {
      uint32_t k = orc_bucket(seed, o, coords[t], m);
      if (!any[k] || x > u[k]) u[k] = x;
      if (!any[k] || x < l[k]) l[k] = x;
      any[k] = 1;
    }
  }
  if (filled) memcpy(filled, any, m);
  free(any);
}

/* bfloat16 keeps the top 16 bits of an IEEE binary32 value (sign, 8 exponent
 * bits, 7 fraction bits). The paper stores its sketches in bfloat16 (Section
 * 4.1). To keep every stored bound a bound, the upper half U is rounded toward
 * +infinity and the lower half L toward -infinity: dropping the low 16 bits
 * moves a value toward zero, so a positive value rounded up (a negative one
 * rounded down) takes the next bfloat16 away from zero instead. */
static float orc_bits_to_float(uint32_t b) {
  float f;
  memcpy(&f, &b, 4);
  return f;
}

double orc_bf16_up(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  if ((b & 0xFFFFu) == 0) return (double)x;            /* already a bfloat16 */
  uint32_t t = b & 0xFFFF0000u;                         /* toward zero */
  if (x > 0.0f) t += 0x10000u;                          /* away from zero = up */
  return (double)orc_bits_to_float(t);
}

double orc_bf16_down(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  if ((b & 0xFFFFu) == 0) return (double)x;
  uint32_t t = b & 0xFFFF0000u;
  if (x < 0.0f) t += 0x10000u;                          /* away from zero = down */
  return (double)orc_bits_to_float(t);
}

/* Decoding used by Alg. 6: least upper bound and greatest lower bound of x[j]. */
double orc_decode_upper(const double *u, uint32_t j, uint32_t m, uint32_t h, uint64_t seed) {
  double v = u[orc_bucket(seed, 0, j, m)];
  for (uint32_t o = 1; o < h; ++o) {
    double w = u[orc_bucket(seed, o, j, m)];
    if (w < v) v = w;
  }
  return v;
}

double orc_decode_lower(const double *l, uint32_t j, uint32_t m, uint32_t h, uint64_t seed) {
  double v = l[orc_bucket(seed, 0, j, m)];
  for (uint32_t o = 1; o < h; ++o) {
    double w = l[orc_bucket(seed, o, j, m)];
    if (w > v) v = w;
  }
  return v;
}

/* Both decodes of every coordinate of one document, from its own sketch. */
void orc_decode_doc(uint32_t nnz, const uint32_t *coords, const float *vals, uint32_t m, uint32_t h,
                    uint64_t seed, double *upper, double *lower) {
  double *u = (double *)malloc(sizeof(double) * m), *l = (double *)malloc(sizeof(double) * m);
  orc_sketch(nnz, coords, vals, m, h, seed, u, l, NULL);
  for (uint32_t t = 0; t < nnz; ++t) {
    upper[t] = orc_decode_upper(u, coords[t], m, h, seed);
    lower[t] = orc_decode_lower(l, coords[t], m, h, seed);
  }
  free(u);
  free(l);
}

/* ------------------------------------------------------------------------- */
/* Query preparation (Alg. 6, first two steps)                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
  uint32_t j;
  double q;
} orc_qterm;

static int orc_qterm_cmp(const void *a, const void *b) {
  const orc_qterm *x = (const orc_qterm *)a, *y = (const orc_qterm *)b;
  double ax = fabs(x->q), ay = fabs(y->q);
  if (ax > ay) return -1;
  if (ax < ay) return 1;
  return (x->j < y->j) ? -1 : (x->j > y->j);
}

/* nz(q) sorted by |q_j| descending, ties by lower coordinate. Returns the count. */
static uint32_t orc_sorted_query(uint32_t nnz, const uint32_t *c, const float *v, orc_qterm *out) {
  uint32_t t = 0;
  for (uint32_t i = 0; i < nnz; ++i)
    if (v[i] != 0.0f) {
      out[t].j = c[i];
      out[t].q = (double)v[i];
      ++t;
    }
  qsort(out, t, sizeof(orc_qterm), orc_qterm_cmp);
  return t;
}

/* ------------------------------------------------------------------------- */
/* Doc-at-a-time definition (mode O-def): one (query, document) pair.          */
/* ------------------------------------------------------------------------- */

static int orc_find(uint32_t nnz, const uint32_t *c, uint32_t j) {
  for (uint32_t t = 0; t < nnz; ++t)
    if (c[t] == j) return (int)t;
  return -1;
}

/* Sinnamon estimate of <q, x> from x's own sketch, the terms taken in the
 * order of Alg. 6. *abs_sum receives the sum of |term| (the error scale used by
 * the comparison tolerance). */
double orc_pair_est(uint32_t qn, const uint32_t *qc, const float *qv, uint32_t dn, const uint32_t *dc,
                    const float *dv, uint32_t m, uint32_t h, uint64_t seed, double *abs_sum) {
  double *u = (double *)malloc(sizeof(double) * m), *l = (double *)malloc(sizeof(double) * m);
  orc_qterm *qs = (orc_qterm *)malloc(sizeof(orc_qterm) * (qn ? qn : 1));
  orc_sketch(dn, dc, dv, m, h, seed, u, l, NULL);
  uint32_t t = orc_sorted_query(qn, qc, qv, qs);
  double s = 0.0, a = 0.0;
  for (uint32_t i = 0; i < t; ++i) {
    int p = orc_find(dn, dc, qs[i].j);
    if (p < 0 || dv[p] == 0.0f) continue; /* the document is not on list I[j] */
    double x = qs[i].q > 0 ? orc_decode_upper(u, qs[i].j, m, h, seed) : orc_decode_lower(l, qs[i].j, m, h, seed);
    double term = qs[i].q * x;
    s += term;
    a += fabs(term);
  }
  if (abs_sum) *abs_sum = a;
  free(u);
  free(l);
  free(qs);
  return s;
}

/* Exact inner product (Eq. 2), same term order. */
double orc_pair_exact(uint32_t qn, const uint32_t *qc, const float *qv, uint32_t dn, const uint32_t *dc,
                      const float *dv) {
  orc_qterm *qs = (orc_qterm *)malloc(sizeof(orc_qterm) * (qn ? qn : 1));
  uint32_t t = orc_sorted_query(qn, qc, qv, qs);
  double s = 0.0;
  for (uint32_t i = 0; i < t; ++i) {
    int p = orc_find(dn, dc, qs[i].j);
    if (p < 0) continue;
    s += qs[i].q * (double)dv[p];
  }
  free(qs);
  return s;
}

/* ------------------------------------------------------------------------- */
/* Coordinate-at-a-time index (mode O-cat): Alg. 5 indexing, Alg. 6 scoring,   */
/* Alg. 2 exact scoring, Alg. 3 selection.                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
  uint32_t N, n, m, h;
  uint64_t seed;
  uint64_t *list_ptr; /* n + 1 offsets into list_doc / list_val */
  uint32_t *list_doc; /* document positions, ascending within a list */
  float *list_val;    /* the true values, used only by exact scoring */
  double *U, *L;      /* sketch matrix halves, m rows of N columns */
  uint32_t *ids;      /* external id of every position */
  int64_t *vec_ptr;   /* vector storage S of Alg. 7: the documents as given */
  uint32_t *vec_c;
  float *vec_v;
} orc_index;

/* flags & 1: the sketch is stored in bfloat16, U rounded up and L down. */
orc_index *orc_build(uint32_t N, const int64_t *indptr, const uint32_t *coords, const float *vals,
                     const uint32_t *ids, uint32_t n, uint32_t m, uint32_t h, uint64_t seed, uint32_t flags) {
  orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
  ix->N = N;
  ix->n = n;
  ix->m = m;
  ix->h = h;
  ix->seed = seed;
  ix->list_ptr = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  for (uint32_t i = 0; i < N; ++i)
    for (int64_t t = indptr[i]; t < indptr[i + 1]; ++t)
      if (vals[t] != 0.0f) ix->list_ptr[coords[t] + 1]++;
  for (uint32_t j = 0; j < n; ++j) ix->list_ptr[j + 1] += ix->list_ptr[j];
  size_t P = ix->list_ptr[n];
  ix->list_doc = (uint32_t *)malloc(sizeof(uint32_t) * (P ? P : 1));
  ix->list_val = (float *)malloc(sizeof(float) * (P ? P : 1));
  uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  memcpy(fill, ix->list_ptr, sizeof(uint64_t) * ((size_t)n + 1));
  ix->U = (double *)malloc(sizeof(double) * (size_t)m * (N ? N : 1));
  ix->L = (double *)malloc(sizeof(double) * (size_t)m * (N ? N : 1));
  ix->ids = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
  double *u = (double *)malloc(sizeof(double) * m), *l = (double *)malloc(sizeof(double) * m);
  for (uint32_t i = 0; i < N; ++i) {
    ix->ids[i] = ids ? ids[i] : i;
    int64_t a = indptr[i], b = indptr[i + 1];
    /* Alg. 5: insert i into I[j] for every j in nz(x_i) ... */
    for (int64_t t = a; t < b; ++t) {
      if (vals[t] == 0.0f) continue;
      uint64_t p = fill[coords[t]]++;
      ix->list_doc[p] = i;
      ix->list_val[p] = vals[t];
    }
    /* ... then write column i of U and L. */
    orc_sketch((uint32_t)(b - a), coords + a, vals + a, m, h, seed, u, l, NULL);
    for (uint32_t k = 0; k < m; ++k) {
      /* u[k], l[k] are binary32 values (a max / min of the inputs) or 0 */
      ix->U[(size_t)k * N + i] = (flags & 1u) ? orc_bf16_up((float)u[k]) : u[k];
      ix->L[(size_t)k * N + i] = (flags & 1u) ? orc_bf16_down((float)l[k]) : l[k];
    }
  }
  free(u);
  free(l);
  free(fill);
  /* the vector storage keeps every document's (coordinate, value) pairs */
  size_t E = (size_t)(indptr[N] - indptr[0]);
  ix->vec_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)N + 1));
  ix->vec_c = (uint32_t *)malloc(sizeof(uint32_t) * (E ? E : 1));
  ix->vec_v = (float *)malloc(sizeof(float) * (E ? E : 1));
  for (uint32_t i = 0; i <= N; ++i) ix->vec_ptr[i] = indptr[i] - indptr[0];
  if (E) {
    memcpy(ix->vec_c, coords + indptr[0], sizeof(uint32_t) * E);
    memcpy(ix->vec_v, vals + indptr[0], sizeof(float) * E);
  }
  return ix;
}

void orc_free(orc_index *ix) {
  if (!ix) return;
  free(ix->list_ptr);
  free(ix->list_doc);
  free(ix->list_val);
  free(ix->U);
  free(ix->L);
  free(ix->ids);
  free(ix->vec_ptr);
  free(ix->vec_c);
  free(ix->vec_v);
  free(ix);
}

uint64_t orc_postings(const orc_index *ix) { return ix->list_ptr[ix->n]; }

/* Scores of every document for one query. mode 0: Sinnamon estimate (Alg. 6),
 * mode 1: exact (Alg. 2). abs_sum (may be NULL) receives sum |term| per doc.
 * max_coords > 0 is the anytime budget: the walk over the sorted query
 * coordinates stops after that many (the break of Alg. 4 and Alg. 6 taken
 * after a fixed number of coordinates instead of a time budget). */
void orc_score_all(const orc_index *ix, uint32_t qn, const uint32_t *qc, const float *qv, int mode,
                   uint32_t max_coords, double *scores, double *abs_sum) {
  orc_qterm *qs = (orc_qterm *)malloc(sizeof(orc_qterm) * (qn ? qn : 1));
  uint32_t t = orc_sorted_query(qn, qc, qv, qs);
  if (max_coords > 0 && max_coords < t) t = max_coords;
  for (uint32_t i = 0; i < ix->N; ++i) scores[i] = 0.0;
  if (abs_sum)
    for (uint32_t i = 0; i < ix->N; ++i) abs_sum[i] = 0.0;
  uint32_t K[16];
  for (uint32_t c = 0; c < t; ++c) {
    uint32_t j = qs[c].j;
    double q = qs[c].q;
    if (j >= ix->n) continue;
    for (uint32_t o = 0; o < ix->h; ++o) K[o] = orc_bucket(ix->seed, o, j, ix->m);
    for (uint64_t p = ix->list_ptr[j]; p < ix->list_ptr[j + 1]; ++p) {
      uint32_t i = ix->list_doc[p];
      double s;
      if (mode == 1) {
        s = (double)ix->list_val[p] * q;
      } else if (q > 0) {
        double b = ix->U[(size_t)K[0] * ix->N + i];
        for (uint32_t o = 1; o < ix->h; ++o) {
          double w = ix->U[(size_t)K[o] * ix->N + i];
          if (w < b) b = w;
        }
        s = q * b;
      } else {
        double b = ix->L[(size_t)K[0] * ix->N + i];
        for (uint32_t o = 1; o < ix->h; ++o) {
          double w = ix->L[(size_t)K[o] * ix->N + i];
          if (w > b) b = w;
        }
        s = q * b;
      }
      scores[i] += s;
      if (abs_sum) abs_sum[i] += fabs(s);
    }
  }
  free(qs);
}

/* FindLargest (Alg. 3) with k' = k. The heap keeps the k best items seen so far
 * and its root is the worst of them. "a beats b" means a higher score, or an
 * equal score and a lower external id. Returns the count, results best first. */
typedef struct {
  double s;
  uint32_t id;
  uint32_t pos;
} orc_item;

static int orc_beats(const orc_item *a, const orc_item *b) {
  if (a->s > b->s) return 1;
  if (a->s < b->s) return 0;
  return a->id < b->id;
}

static void orc_sift_down(orc_item *hp, uint32_t n, uint32_t i) {
  for (;;) {
    uint32_t w = i, a = 2 * i + 1, b = 2 * i + 2;
    if (a < n && orc_beats(&hp[w], &hp[a])) w = a;
    if (b < n && orc_beats(&hp[w], &hp[b])) w = b;
    if (w == i) return;
    orc_item t = hp[i];
    hp[i] = hp[w];
    hp[w] = t;
    i = w;
  }
}

static void orc_sift_up(orc_item *hp, uint32_t i) {
  while (i > 0) {
    uint32_t p = (i - 1) / 2;
    if (!orc_beats(&hp[p], &hp[i])) return;
    orc_item t = hp[i];
    hp[i] = hp[p];
    hp[p] = t;
    i = p;
  }
}

uint32_t orc_find_largest(uint32_t N, const double *scores, const uint32_t *ids, const uint8_t *live, uint32_t k,
                          uint32_t *out_pos) {
  orc_item *hp = (orc_item *)malloc(sizeof(orc_item) * (k + 1));
  uint32_t n = 0;
  for (uint32_t i = 0; i < N; ++i) {
    if (live && !live[i]) continue;
    orc_item it = {scores[i] == 0.0 ? 0.0 : scores[i], ids ? ids[i] : i, i};
    if (n < k) {
      hp[n] = it;
      orc_sift_up(hp, n);
      ++n;
    } else if (k > 0 && orc_beats(&it, &hp[0])) {
      hp[0] = it;
      orc_sift_down(hp, n, 0);
    }
  }
  /* pop worst-first into the tail of the output */
  uint32_t cnt = n;
  while (n > 0) {
    out_pos[n - 1] = hp[0].pos;
    hp[0] = hp[n - 1];
    --n;
    orc_sift_down(hp, n, 0);
  }
  free(hp);
  return cnt;
}

/* Batched top-k over the index. mode 0: estimate, 1: exact. OpenMP over
 * queries when threads > 1. Outputs are k per query; counts = min(k, N). */
void orc_search(const orc_index *ix, uint32_t nq, const int64_t *qptr, const uint32_t *qc, const float *qv,
                uint32_t k, int mode, uint32_t max_coords, int threads, uint32_t *out_ids, double *out_scores,
                double *out_abs, uint32_t *out_counts) {
#ifdef _OPENMP
  if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
  for (int64_t qi = 0; qi < (int64_t)nq; ++qi) {
    double *sc = (double *)malloc(sizeof(double) * (ix->N ? ix->N : 1));
    double *ab = out_abs ? (double *)malloc(sizeof(double) * (ix->N ? ix->N : 1)) : NULL;
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * (k ? k : 1));
    int64_t a = qptr[qi], b = qptr[qi + 1];
    orc_score_all(ix, (uint32_t)(b - a), qc + a, qv + a, mode, max_coords, sc, ab);
    uint32_t c = orc_find_largest(ix->N, sc, ix->ids, NULL, k, pos);
    out_counts[qi] = c;
    for (uint32_t r = 0; r < c; ++r) {
      out_ids[(size_t)qi * k + r] = ix->ids[pos[r]];
      out_scores[(size_t)qi * k + r] = sc[pos[r]];
      if (out_abs) out_abs[(size_t)qi * k + r] = ab[pos[r]];
    }
    free(sc);
    free(ab);
    free(pos);
  }
}

/* Ranking with k' >= k (Alg. 7) for a batch of queries. Per query: the
 * Sinnamon scores of every document (Alg. 6, stopped after max_coords sorted
 * coordinates when max_coords > 0); V = FindLargest(scores, k');
 * s_v = <q, S.Fetch(v)> for v in V, the exact inner product (Eq. 2) of the
 * query with the stored vector; the result is FindLargest({s_v}, k). Both
 * FindLargest calls break ties by the lower external id. out_scores are the
 * exact scores s_v, out_abs the sums of |q_j x_j| over the shared coordinates
 * (the error scale of the comparison tolerance); counts = min(k, k', N). */
void orc_rerank(const orc_index *ix, uint32_t nq, const int64_t *qptr, const uint32_t *qc, const float *qv,
                uint32_t k, uint32_t kprime, uint32_t max_coords, int threads, uint32_t *out_ids, double *out_scores,
                double *out_abs, uint32_t *out_counts) {
#ifdef _OPENMP
  if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
  for (int64_t qi = 0; qi < (int64_t)nq; ++qi) {
    double *sc = (double *)malloc(sizeof(double) * (ix->N ? ix->N : 1));
    uint32_t *V = (uint32_t *)malloc(sizeof(uint32_t) * (kprime ? kprime : 1));
    double *sv = (double *)malloc(sizeof(double) * (kprime ? kprime : 1));
    double *av = (double *)malloc(sizeof(double) * (kprime ? kprime : 1));
    uint32_t *vid = (uint32_t *)malloc(sizeof(uint32_t) * (kprime ? kprime : 1));
    uint32_t *best = (uint32_t *)malloc(sizeof(uint32_t) * (k ? k : 1));
    int64_t a = qptr[qi], b = qptr[qi + 1];
    uint32_t qn = (uint32_t)(b - a);
    orc_score_all(ix, qn, qc + a, qv + a, 0, max_coords, sc, NULL); /* anytime scoring, then the full q */
    uint32_t nv = orc_find_largest(ix->N, sc, ix->ids, NULL, kprime, V);
    for (uint32_t r = 0; r < nv; ++r) {
      uint32_t d = V[r];
      int64_t d0 = ix->vec_ptr[d], d1 = ix->vec_ptr[d + 1];
      sv[r] = orc_pair_exact(qn, qc + a, qv + a, (uint32_t)(d1 - d0), ix->vec_c + d0, ix->vec_v + d0);
      /* |q_j x_j| summed over the coordinates both vectors hold */
      double s_abs = 0.0;
      for (uint32_t t = 0; t < qn; ++t) {
        if (qv[a + t] == 0.0f) continue;
        int p = orc_find((uint32_t)(d1 - d0), ix->vec_c + d0, qc[a + t]);
        if (p >= 0) s_abs += fabs((double)qv[a + t] * (double)ix->vec_v[d0 + p]);
      }
      av[r] = s_abs;
      vid[r] = ix->ids[d];
    }
    uint32_t c = orc_find_largest(nv, sv, vid, NULL, k, best);
    out_counts[qi] = c;
    for (uint32_t r = 0; r < c; ++r) {
      out_ids[(size_t)qi * k + r] = vid[best[r]];
      out_scores[(size_t)qi * k + r] = sv[best[r]];
      out_abs[(size_t)qi * k + r] = av[best[r]];
    }
    free(sc);
    free(V);
    free(sv);
    free(av);
    free(vid);
    free(best);
  }
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Learned threshold filter: hashed query features and the MLP (FP64).        */
/* Not in the paper. Features: f[g(j)] += xi(j) * q_j with                    */
/* g(j) = mix64(mix64(fseed) ^ j) mod 128 and xi(j) = +-1 from the top bit of  */
/* mix64(mix64(fseed + 1) ^ j) for the first 128 features (signed feature       */
/* hashing, Weinberger et al. 2009), and f[128 + g(j)] += q_j * q_j for the     */
/* second 128 (the squared mass per hash bucket).                              */
/* ------------------------------------------------------------------------- */

void orc_features(uint32_t nnz, const uint32_t *c, const float *v, uint64_t fseed, double *f) {
  for (int t = 0; t < 256; ++t) f[t] = 0.0;
  uint64_t s0 = orc_mix64(fseed), s1 = orc_mix64(fseed + 1);
  for (uint32_t t = 0; t < nnz; ++t) {
    if (v[t] == 0.0f) continue;
    uint32_t g = (uint32_t)(orc_mix64(s0 ^ (uint64_t)c[t]) % 128u);
    double xi = (orc_mix64(s1 ^ (uint64_t)c[t]) >> 63) ? -1.0 : 1.0;
    double q = (double)v[t];
    f[g] += xi * q;
    f[128 + g] += q * q;
  }
}

/* MLP 256 -> 128 -> 128 -> 1 with ReLU. Weights row-major [out][in]:
 * W1[128][256], b1[128], W2[128][128], b2[128], W3[128], b3[1].
 * Forward for B rows of X[B][256]; yhat[B]. */
void orc_mlp_forward(uint32_t B, const double *X, const double *W1, const double *b1, const double *W2,
                     const double *b2, const double *W3, const double *b3, double *yhat) {
  double h1[128], h2[128];
  for (uint32_t r = 0; r < B; ++r) {
    const double *x = X + (size_t)r * 256;
    for (int o = 0; o < 128; ++o) {
      double s = b1[o];
      for (int i = 0; i < 256; ++i) s += W1[o * 256 + i] * x[i];
      h1[o] = s > 0 ? s : 0;
    }
    for (int o = 0; o < 128; ++o) {
      double s = b2[o];
      for (int i = 0; i < 128; ++i) s += W2[o * 128 + i] * h1[i];
      h2[o] = s > 0 ? s : 0;
    }
    double s = b3[0];
    for (int i = 0; i < 128; ++i) s += W3[i] * h2[i];
    yhat[r] = s;
  }
}

/* Loss L = (1/B) sum_r (yhat_r - y_r)^2 and its gradient with respect to every
 * weight and bias (same layouts as the weights). Returns L. */
double orc_mlp_loss_grad(uint32_t B, const double *X, const double *y, const double *W1, const double *b1,
                         const double *W2, const double *b2, const double *W3, const double *b3, double *gW1,
                         double *gb1, double *gW2, double *gb2, double *gW3, double *gb3) {
  memset(gW1, 0, sizeof(double) * 128 * 256);
  memset(gb1, 0, sizeof(double) * 128);
  memset(gW2, 0, sizeof(double) * 128 * 128);
  memset(gb2, 0, sizeof(double) * 128);
  memset(gW3, 0, sizeof(double) * 128);
  gb3[0] = 0;
  double loss = 0;
  double z1[128], h1[128], z2[128], h2[128], d2[128], d1[128];
  for (uint32_t r = 0; r < B; ++r) {
    const double *x = X + (size_t)r * 256;
    for (int o = 0; o < 128; ++o) {
      double s = b1[o];
      for (int i = 0; i < 256; ++i) s += W1[o * 256 + i] * x[i];
      z1[o] = s;
      h1[o] = s > 0 ? s : 0;
    }
    for (int o = 0; o < 128; ++o) {
      double s = b2[o];
      for (int i = 0; i < 128; ++i) s += W2[o * 128 + i] * h1[i];
      z2[o] = s;
      h2[o] = s > 0 ? s : 0;
    }
    double yh = b3[0];
    for (int i = 0; i < 128; ++i) yh += W3[i] * h2[i];
    double e = yh - y[r];
    loss += e * e;
    double dy = 2.0 * e / (double)B; /* dL/dyhat */
    gb3[0] += dy;
    for (int i = 0; i < 128; ++i) {
      gW3[i] += dy * h2[i];
      d2[i] = z2[i] > 0 ? dy * W3[i] : 0.0;
    }
    for (int o = 0; o < 128; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < 128; ++i) gW2[o * 128 + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < 128; ++i) {
      double s = 0;
      for (int o = 0; o < 128; ++o) s += W2[o * 128 + i] * d2[o];
      d1[i] = z1[i] > 0 ? s : 0.0;
    }
    for (int o = 0; o < 128; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < 256; ++i) gW1[o * 256 + i] += d1[o] * x[i];
    }
  }
  return loss / (double)B;
}
