/*
 * CPU oracle for the bulk update of neighborhood-sampling estimators.
 * TEST INFRASTRUCTURE ONLY (see oracle.h): plain sequential C, no sharing
 * with the GPU library.
 *
 * Paper: Tangwongsan, Pavan, Tirthapura, "Parallel Triangle Counting in
 * Massive Streaming Graphs".  Section references are to that paper.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Random protocol.  The paper leaves the random source open (Sec. 4.2 only
 * asks for randInt).  Every decision is drawn from a counter-based
 * generator: the splitmix64 output finalizer (Steele, Lea, Flood, OOPSLA'14)
 * chained over the key (seed, estimator, batch, purpose, attempt), and the
 * bounded integer is Lemire's multiply-shift with rejection (ACM TOMACS
 * 2019), which is exactly uniform on [0, n).                                */
/* ------------------------------------------------------------------------ */
#define GOLDEN 0x9E3779B97F4A7C15ULL

uint64_t orc_mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return z;
}

uint64_t orc_raw(uint64_t seed, uint64_t est, uint64_t batch, uint64_t purpose,
                 uint64_t attempt) {
  uint64_t k = orc_mix64(seed ^ GOLDEN);
  k = orc_mix64(k ^ est);
  k = orc_mix64(k ^ batch);
  return orc_mix64(k ^ (purpose * GOLDEN + attempt));
}

uint64_t orc_lemire_step(uint64_t x, uint64_t n, int *reject) {
  unsigned __int128 p = (unsigned __int128)x * (unsigned __int128)n;
  uint64_t lo = (uint64_t)p;
  *reject = 0;
  if (lo < n) {
    /* threshold = 2^64 mod n: the low halves below it are over-represented */
    uint64_t t = (0 - n) % n;
    if (lo < t) *reject = 1;
  }
  return (uint64_t)(p >> 64);
}

uint64_t orc_uniform(uint64_t seed, uint64_t est, uint64_t batch,
                     uint64_t purpose, uint64_t n) {
  for (uint64_t attempt = 0;; ++attempt) {
    int reject;
    uint64_t v = orc_lemire_step(orc_raw(seed, est, batch, purpose, attempt),
                                 n, &reject);
    if (!reject) return v;
  }
}

static uint64_t draw(const orc_state *s, orc_draw_fn fn, void *ctx,
                     uint32_t est, uint32_t purpose, uint64_t n) {
  if (fn) return fn(ctx, est, purpose, n);
  return orc_uniform(s->seed, est, s->batch, purpose, n);
}

/* ------------------------------------------------------------------------ */
/* Edges                                                                     */
/* ------------------------------------------------------------------------ */
static uint64_t canon(uint32_t a, uint32_t b) {
  uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  return ((uint64_t)lo << 32) | hi;
}
static uint32_t e_lo(uint64_t e) { return (uint32_t)(e >> 32); }
static uint32_t e_hi(uint64_t e) { return (uint32_t)e; }
static int incident(const uint32_t *W, uint32_t j, uint32_t x) {
  return W[2 * (size_t)j] == x || W[2 * (size_t)j + 1] == x;
}

/* The edge that completes the wedge f1, f2 (Invariant 1, item 4): the two
 * endpoints that f1 and f2 do not share.  Empty when they do not form a
 * wedge (equal edges or disjoint edges). */
static uint64_t closing_edge(uint64_t f1, uint64_t f2) {
  uint32_t a = e_lo(f1), b = e_hi(f1), x = e_lo(f2), y = e_hi(f2);
  if (f1 == f2) return ORC_EMPTY;
  uint32_t t, f;
  if (a == x) { t = b; f = y; }
  else if (a == y) { t = b; f = x; }
  else if (b == x) { t = a; f = y; }
  else if (b == y) { t = a; f = x; }
  else return ORC_EMPTY;
  return canon(t, f);
}

/* ------------------------------------------------------------------------ */
/* Bank                                                                      */
/* ------------------------------------------------------------------------ */
orc_state *orc_create(uint32_t r, uint64_t seed) {
  if (r == 0) return NULL;
  orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
  if (!s) return NULL;
  s->r = r;
  s->seed = seed;
  s->r1 = (uint64_t *)malloc(sizeof(uint64_t) * r);
  s->r2 = (uint64_t *)malloc(sizeof(uint64_t) * r);
  s->c = (uint32_t *)calloc(r, sizeof(uint32_t));
  s->closed = (uint8_t *)calloc(r, 1);
  if (!s->r1 || !s->r2 || !s->c || !s->closed) {
    orc_destroy(s);
    return NULL;
  }
  for (uint32_t i = 0; i < r; ++i) s->r1[i] = s->r2[i] = ORC_EMPTY;
  return s;
}

void orc_destroy(orc_state *s) {
  if (!s) return;
  free(s->r1);
  free(s->r2);
  free(s->c);
  free(s->closed);
  free(s);
}

uint64_t orc_sum(const orc_state *s) {
  uint64_t S = 0;
  for (uint32_t i = 0; i < s->r; ++i)
    if (s->closed[i]) S += s->c[i];
  return S;
}

double orc_estimate(const orc_state *s) {
  return (double)orc_sum(s) * (double)s->m / (double)s->r;
}

static int cmp_double(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

double orc_mom(const orc_state *s, uint32_t g, uint64_t *group_sums) {
  if (g == 0 || g > s->r) return NAN;
  double *mean = (double *)malloc(sizeof(double) * g);
  if (!mean) return NAN;
  for (uint32_t k = 0; k < g; ++k) {
    /* group k: estimators floor(k r / g) .. floor((k+1) r / g) - 1 */
    const uint64_t lo = (uint64_t)k * s->r / g;
    const uint64_t hi = (uint64_t)(k + 1) * s->r / g;
    uint64_t S = 0;
    for (uint64_t i = lo; i < hi; ++i)
      if (s->closed[i]) S += s->c[i];
    if (group_sums) group_sums[k] = S;
    mean[k] = (double)S * (double)s->m / (double)(hi - lo);
  }
  qsort(mean, g, sizeof(double), cmp_double);
  const double med = (g & 1u) ? mean[g / 2] : 0.5 * (mean[g / 2 - 1] + mean[g / 2]);
  free(mean);
  return med;
}

uint64_t orc_estimators_needed(double eps, double delta, uint64_t m,
                               uint64_t maxdeg, double tau) {
  if (!(eps > 0.0) || !(delta > 0.0 && delta < 1.0) || !(tau > 0.0)) return 0;
  const double r = 96.0 / (eps * eps) * (double)m * (double)maxdeg / tau * log(1.0 / delta);
  return (uint64_t)ceil(r);
}

static int check_batch(const uint32_t *W, uint32_t w) {
  for (uint32_t j = 0; j < w; ++j)
    if (W[2 * (size_t)j] == W[2 * (size_t)j + 1]) return ORC_EBADEDGE;
  return ORC_OK;
}

/* ======================================================================== */
/* Variant 1: definitions, O(r*w) per batch.                                 */
/* ======================================================================== */

/* |{ j : x in W_j, j > j1 }|, with j1 = NONE read as "before the batch". */
static uint32_t count_later(const uint32_t *W, uint32_t w, uint32_t x,
                            uint32_t j1) {
  uint32_t n = 0;
  uint32_t j0 = (j1 == ORC_NONE) ? 0 : j1 + 1;
  for (uint32_t j = j0; j < w; ++j) n += incident(W, j, x);
  return n;
}

/* Position of the edge on x that has exactly k later W-edges on x. */
static uint32_t kth_from_last(const uint32_t *W, uint32_t w, uint32_t x,
                              uint32_t k) {
  uint32_t seen = 0;
  for (uint32_t j = w; j-- > 0;) {
    if (!incident(W, j, x)) continue;
    if (seen == k) return j;
    ++seen;
  }
  return ORC_NONE;
}

int orc_batch_def(orc_state *s, const uint32_t *W, uint32_t w,
                  orc_draw_fn fn, void *ctx) {
  if (w == 0) return ORC_OK;
  if (!W) return ORC_EINVAL;
  int rc = check_batch(W, w);
  if (rc) return rc;
  const uint64_t m = s->m;
  for (uint32_t i = 0; i < s->r; ++i) {
    uint64_t r1 = s->r1[i], r2 = s->r2[i];
    uint64_t c = s->c[i];
    uint8_t closed = s->closed[i];

    /* Step 1 (Sec. 4.2): with probability w/(w+m) take a uniform edge of W. */
    uint32_t j1 = ORC_NONE;
    uint64_t x = draw(s, fn, ctx, i, 1, m + w);
    if (x >= m) {
      j1 = (uint32_t)(x - m);
      r1 = canon(W[2 * (size_t)j1], W[2 * (size_t)j1 + 1]);
      c = 0;
      r2 = ORC_EMPTY;
      closed = 0;
    }

    /* Step 2 (Sec. 4.3): chi+ = |Gamma_W(f1)| split by endpoint. */
    uint32_t u = e_lo(r1), v = e_hi(r1);
    uint64_t ld = count_later(W, w, u, j1);
    uint64_t rd = count_later(W, w, v, j1);
    uint64_t cplus = ld + rd;
    uint32_t p2 = ORC_NONE;
    if (cplus > 0) {
      /* keep f2 with probability chi-/(chi- + chi+), else a uniform pick
       * from Gamma_W(f1) under the phi naming scheme */
      uint64_t y = draw(s, fn, ctx, i, 2, c + cplus);
      if (y >= c) {
        uint64_t phi = y - c;
        uint32_t src = phi < ld ? u : v;
        uint32_t k = (uint32_t)(phi < ld ? phi : phi - ld);
        uint32_t j2 = kth_from_last(W, w, src, k);
        r2 = canon(W[2 * (size_t)j2], W[2 * (size_t)j2 + 1]);
        closed = 0;
        p2 = j2;
      }
      c += cplus;
      if (c > 0x7FFFFFFFu) return ORC_EOVERFLOW;
    }

    /* Step 3 (Sec. 4.4): a closing edge later than f2. */
    if (r2 != ORC_EMPTY && !closed) {
      uint64_t q = closing_edge(r1, r2);
      if (q != ORC_EMPTY) {
        for (uint32_t j = w; j-- > 0;) {
          if (canon(W[2 * (size_t)j], W[2 * (size_t)j + 1]) != q) continue;
          if (p2 == ORC_NONE || j > p2) closed = 1;
          break; /* the latest occurrence decides */
        }
      }
    }
    s->r1[i] = r1;
    s->r2[i] = r2;
    s->c[i] = (uint32_t)c;
    s->closed[i] = closed;
  }
  s->m += w;
  s->batch += 1;
  return ORC_OK;
}

/* ======================================================================== */
/* Variant 2: the paper's bulk algorithm (Sec. 4.2 - 4.4) with qsort.        */
/* ======================================================================== */

typedef struct {
  uint32_t src, dst, rank, pos;
} arc_rec;

/* rankAll order: src ascending, ties by pos descending (Lemma rankAll). */
static int cmp_src_posdesc(const void *pa, const void *pb) {
  const arc_rec *a = (const arc_rec *)pa, *b = (const arc_rec *)pb;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  if (a->pos != b->pos) return a->pos > b->pos ? -1 : 1;
  return 0;
}

/* F = rankAll(W): map+concat two records per edge, sort, then a scan with
 * resets at the first record of every src (Appendix B, in its sequential
 * form: the running count restarts at each new src). */
static arc_rec *rank_all(const uint32_t *W, uint32_t w) {
  size_t n = 2 * (size_t)w;
  arc_rec *F = (arc_rec *)malloc(sizeof(arc_rec) * (n ? n : 1));
  if (!F) return NULL;
  for (uint32_t j = 0; j < w; ++j) {
    uint32_t a = W[2 * (size_t)j], b = W[2 * (size_t)j + 1];
    F[2 * (size_t)j] = (arc_rec){a, b, 0, j};
    F[2 * (size_t)j + 1] = (arc_rec){b, a, 0, j};
  }
  qsort(F, n, sizeof(arc_rec), cmp_src_posdesc);
  for (size_t i = 0; i < n; ++i)
    F[i].rank = (i == 0 || F[i].src != F[i - 1].src) ? 0 : F[i - 1].rank + 1;
  return F;
}

/* [lo, hi) of records with src == x in F (sorted by src). */
static void src_range(const arc_rec *F, size_t n, uint32_t x, size_t *lo,
                      size_t *hi) {
  size_t a = 0, b = n;
  while (a < b) {
    size_t mid = a + (b - a) / 2;
    if (F[mid].src < x) a = mid + 1; else b = mid;
  }
  *lo = a;
  b = n;
  while (a < b) {
    size_t mid = a + (b - a) / 2;
    if (F[mid].src <= x) a = mid + 1; else b = mid;
  }
  *hi = a;
}

/* Q1 (Sec. 4.3): the record with src == x and the least pos >= p; p = -1
 * asks for the earliest record of x.  Returns its index or -1. */
static long long q1_search(const arc_rec *F, size_t n, uint32_t x,
                           long long p) {
  size_t lo, hi;
  src_range(F, n, x, &lo, &hi);
  /* pos is decreasing on [lo, hi): find the first index with pos < p */
  size_t a = lo, b = hi;
  while (a < b) {
    size_t mid = a + (b - a) / 2;
    if ((long long)F[mid].pos >= p) a = mid + 1; else b = mid;
  }
  return a == lo ? -1 : (long long)a - 1;
}

/* Q2 (Sec. 4.3): the record with src == x and rank == k. */
static long long q2_search(const arc_rec *F, size_t n, uint32_t x,
                           uint32_t k) {
  size_t a = 0, b = n;
  while (a < b) {
    size_t mid = a + (b - a) / 2;
    if (F[mid].src < x || (F[mid].src == x && F[mid].rank < k)) a = mid + 1;
    else b = mid;
  }
  if (a < n && F[a].src == x && F[a].rank == k) return (long long)a;
  return -1;
}

/* Step 3 records: {src=u<v, dst=v, pos}, sorted by (src, dst), then pos. */
static int cmp_src_dst(const void *pa, const void *pb) {
  const arc_rec *a = (const arc_rec *)pa, *b = (const arc_rec *)pb;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  if (a->dst != b->dst) return a->dst < b->dst ? -1 : 1;
  if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
  return 0;
}

/* exact multisearch for (t, f): the latest position of that edge, or -1. */
static long long edge_search(const arc_rec *E, size_t n, uint32_t t,
                             uint32_t f) {
  size_t a = 0, b = n;
  while (a < b) {
    size_t mid = a + (b - a) / 2;
    if (E[mid].src < t || (E[mid].src == t && E[mid].dst <= f)) a = mid + 1;
    else b = mid;
  }
  if (a > 0 && E[a - 1].src == t && E[a - 1].dst == f)
    return (long long)E[a - 1].pos;
  return -1;
}

int orc_batch_bulk(orc_state *s, const uint32_t *W, uint32_t w,
                   orc_draw_fn fn, void *ctx) {
  if (w == 0) return ORC_OK;
  if (!W) return ORC_EINVAL;
  int rc = check_batch(W, w);
  if (rc) return rc;
  const uint32_t r = s->r;
  const uint64_t m = s->m;
  uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * r);
  uint32_t *p2 = (uint32_t *)malloc(sizeof(uint32_t) * r);
  uint64_t *chi_minus = (uint64_t *)malloc(sizeof(uint64_t) * r);
  uint64_t *ld = (uint64_t *)malloc(sizeof(uint64_t) * r);
  uint64_t *rd = (uint64_t *)malloc(sizeof(uint64_t) * r);
  arc_rec *F = NULL, *E = NULL;
  rc = ORC_OK;
  if (!idx || !p2 || !chi_minus || !ld || !rd) { rc = ORC_EINVAL; goto out; }

  /* ---- Step 1: idx = map randInt(|W|+|E|); extract; combine ---------- */
  for (uint32_t i = 0; i < r; ++i) {
    uint64_t x = draw(s, fn, ctx, i, 1, m + w);
    idx[i] = x >= m ? (uint32_t)(x - m) : ORC_NONE;
  }
  for (uint32_t i = 0; i < r; ++i) {
    if (idx[i] == ORC_NONE) continue;
    uint32_t j = idx[i];
    s->r1[i] = canon(W[2 * (size_t)j], W[2 * (size_t)j + 1]);
    s->c[i] = 0;
    s->r2[i] = ORC_EMPTY;
    s->closed[i] = 0;
  }

  /* ---- Step 2: rankAll, Q1 for ld/rd, coin + phi, Q2 ------------------- */
  F = rank_all(W, w);
  if (!F) { rc = ORC_EINVAL; goto out; }
  const size_t nF = 2 * (size_t)w;
  for (uint32_t i = 0; i < r; ++i) {
    chi_minus[i] = s->c[i];
    uint32_t u = e_lo(s->r1[i]), v = e_hi(s->r1[i]);
    if (idx[i] != ORC_NONE) {
      /* f1 = W[idx]: Q1 at p = idx finds the record u->v itself */
      long long a = q1_search(F, nF, u, idx[i]);
      long long b = q1_search(F, nF, v, idx[i]);
      ld[i] = F[a].rank;
      rd[i] = F[b].rank;
    } else {
      /* f1 older than W: Q1 at p = -1 finds the largest rank; the count of
       * W-edges on that endpoint is one more (zero if it has none) */
      long long a = q1_search(F, nF, u, -1);
      long long b = q1_search(F, nF, v, -1);
      ld[i] = a < 0 ? 0 : (uint64_t)F[a].rank + 1;
      rd[i] = b < 0 ? 0 : (uint64_t)F[b].rank + 1;
    }
  }
  for (uint32_t i = 0; i < r; ++i) {
    uint64_t cplus = ld[i] + rd[i];
    p2[i] = ORC_NONE;
    if (cplus == 0) continue;
    uint64_t total = chi_minus[i] + cplus;
    uint64_t y = draw(s, fn, ctx, i, 2, total);
    if (y >= chi_minus[i]) {
      uint64_t phi = y - chi_minus[i];
      uint32_t u = e_lo(s->r1[i]), v = e_hi(s->r1[i]);
      uint32_t src = phi < ld[i] ? u : v;
      uint32_t k = (uint32_t)(phi < ld[i] ? phi : phi - ld[i]);
      long long a = q2_search(F, nF, src, k);
      uint32_t j2 = F[a].pos;
      s->r2[i] = canon(W[2 * (size_t)j2], W[2 * (size_t)j2 + 1]);
      s->closed[i] = 0;
      p2[i] = j2;
    }
    if (total > 0x7FFFFFFFu) { rc = ORC_EOVERFLOW; goto out; }
    s->c[i] = (uint32_t)total;
  }

  /* ---- Step 3: sort W by (src, dst) with src < dst; multisearch -------- */
  E = (arc_rec *)malloc(sizeof(arc_rec) * w);
  if (!E) { rc = ORC_EINVAL; goto out; }
  for (uint32_t j = 0; j < w; ++j) {
    uint64_t e = canon(W[2 * (size_t)j], W[2 * (size_t)j + 1]);
    E[j] = (arc_rec){e_lo(e), e_hi(e), 0, j};
  }
  qsort(E, w, sizeof(arc_rec), cmp_src_dst);
  for (uint32_t i = 0; i < r; ++i) {
    if (s->r2[i] == ORC_EMPTY || s->closed[i]) continue;
    uint64_t q = closing_edge(s->r1[i], s->r2[i]);
    if (q == ORC_EMPTY) continue;
    long long P = edge_search(E, w, e_lo(q), e_hi(q));
    if (P < 0) continue;
    if (p2[i] == ORC_NONE || (uint64_t)P > p2[i]) s->closed[i] = 1;
  }
  s->m += w;
  s->batch += 1;
out:
  free(idx);
  free(p2);
  free(chi_minus);
  free(ld);
  free(rd);
  free(F);
  free(E);
  return rc;
}

/* ======================================================================== */
/* Worked-example helpers (Figs. 1-3).                                        */
/* ======================================================================== */
uint32_t orc_rank(const uint32_t *W, uint32_t w, uint32_t x, uint32_t y) {
  for (uint32_t i = 0; i < w; ++i) {
    uint32_t a = W[2 * (size_t)i], b = W[2 * (size_t)i + 1];
    if ((a == x && b == y) || (a == y && b == x))
      return count_later(W, w, x, i);
  }
  return count_later(W, w, x, ORC_NONE); /* deg_W(x) */
}

void orc_rank_all(const uint32_t *W, uint32_t w, uint32_t *src, uint32_t *dst,
                  uint32_t *rank, uint32_t *pos) {
  arc_rec *F = rank_all(W, w);
  if (!F) return;
  for (size_t i = 0; i < 2 * (size_t)w; ++i) {
    src[i] = F[i].src;
    dst[i] = F[i].dst;
    rank[i] = F[i].rank;
    pos[i] = F[i].pos;
  }
  free(F);
}

uint32_t orc_phi_pos(const uint32_t *W, uint32_t w, uint32_t u, uint32_t v,
                     uint32_t phi) {
  uint32_t ld = orc_rank(W, w, u, v);
  if (phi < ld) return kth_from_last(W, w, u, phi);
  return kth_from_last(W, w, v, phi - ld);
}
