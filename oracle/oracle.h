/*
 * CPU oracle for the coordinated bulk update of neighborhood-sampling
 * triangle-count estimators (Tangwongsan, Pavan, Tirthapura, "Parallel
 * Triangle Counting in Massive Streaming Graphs", Sec. 3.1 and Sec. 4).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU path is compared against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Two independent implementations of the same per-batch semantics:
 *   orc_batch_def  : every quantity straight from its definition, O(r*w).
 *   orc_batch_bulk : the paper's algorithm in the paper's order (rankAll by
 *                    sort + segmented scan, Q1/Q2 multisearch, Step 3 sort of
 *                    the batch by (src,dst) + exact multisearch), using the C
 *                    library qsort as the sort primitive.
 *
 * Conventions (the paper is silent on them; both variants and the GPU path
 * follow the same reading):
 *   - an edge {a,b} is encoded canon(a,b) = (min<<32)|max; the empty edge is
 *     UINT64_MAX (cannot collide: min < max for a loop-free edge);
 *   - positions inside a batch are 0-based (the paper's figures are 1-based);
 *   - in the level-2 naming scheme u is the smaller vertex id of f1;
 *   - random decisions come from a counter-based generator keyed by
 *     (seed, estimator index, batch index, purpose, attempt); see orc_raw.
 *
 * Parity status: the specific r1/r2 values are pinned only by this random
 * protocol (the paper does not fix a random source); every other property
 * is pinned by the tests (worked example of Figs. 1-3, brute-force
 * invariants, exact mean/variance, w = 1 reservoir reduction).
 */
#ifndef TC_ORACLE_H
#define TC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_EMPTY UINT64_MAX
#define ORC_NONE UINT32_MAX

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EBADEDGE (-2)  /* a self-loop {a,a} in the batch */
#define ORC_EOVERFLOW (-3) /* an adjacency count c no longer fits 31 bits */

/* Estimator bank: r tuples (f1, f2, f3-found, chi) of Invariant 1 (NBSI). */
typedef struct {
  uint32_t r;
  uint64_t seed;
  uint64_t m;     /* |E|: edges consumed before the next batch */
  uint64_t batch; /* number of non-empty batches consumed */
  uint64_t *r1;   /* level-1 edge f1 (canonical code) */
  uint64_t *r2;   /* level-2 edge f2 (canonical code or ORC_EMPTY) */
  uint32_t *c;    /* chi = |Gamma(f1)| */
  uint8_t *closed;/* 1 iff a closing edge f3 > f2 has been seen */
} orc_state;

/* Optional override of the random source: returns a value in [0, n) for
 * estimator `est` and purpose 1 (Step 1) or 2 (Step 2).  NULL selects the
 * keyed generator.  Used by tests to drive hand-traced examples. */
typedef uint64_t (*orc_draw_fn)(void *ctx, uint32_t est, uint32_t purpose,
                                uint64_t n);

/* --- random protocol ---------------------------------------------------- */
uint64_t orc_mix64(uint64_t z);
uint64_t orc_raw(uint64_t seed, uint64_t est, uint64_t batch, uint64_t purpose,
                 uint64_t attempt);
/* One multiply-shift step: returns high64(x*n); *reject = 1 iff the step
 * falls in the rejection zone of Lemire's method. */
uint64_t orc_lemire_step(uint64_t x, uint64_t n, int *reject);
uint64_t orc_uniform(uint64_t seed, uint64_t est, uint64_t batch,
                     uint64_t purpose, uint64_t n);

/* --- estimator bank ----------------------------------------------------- */
orc_state *orc_create(uint32_t r, uint64_t seed);
void orc_destroy(orc_state *s);
/* W is uint32[2*w] (w edges as pairs), arrival order = position order. */
int orc_batch_def(orc_state *s, const uint32_t *W, uint32_t w,
                  orc_draw_fn draw, void *ctx);
int orc_batch_bulk(orc_state *s, const uint32_t *W, uint32_t w,
                   orc_draw_fn draw, void *ctx);
/* S = sum_i c_i * closed_i, exact. */
uint64_t orc_sum(const orc_state *s);
/* Lemma 1 averaged over the bank: (m / r) * S. */
double orc_estimate(const orc_state *s);

/* Median-of-means (Sec. 3.1, the aggregate named before Theorem 2; the
 * paper does not fix the group layout, this one is a reading): the r
 * estimators are cut into g
 * contiguous groups, group k = [floor(k r / g), floor((k+1) r / g)); each
 * group's mean of Lemma 1's X is (m / size_k) * S_k with S_k the exact sum
 * of c_i * closed_i over the group; the result is the median of the g
 * means (the mean of the two middle ones when g is even).  group_sums
 * (length g, may be NULL) receives S_k.  Returns NaN for g == 0 or g > r. */
double orc_mom(const orc_state *s, uint32_t g, uint64_t *group_sums);

/* Theorem 2: estimators that suffice for an (eps, delta)-approximation,
 * ceil(96 / eps^2 * m * maxdeg / tau * ln(1 / delta)) (log read as the
 * natural logarithm).  0 for arguments out of range. */
uint64_t orc_estimators_needed(double eps, double delta, uint64_t m,
                               uint64_t maxdeg, double tau);

/* --- pieces of Sec. 4.3 exposed for the worked-example pins ------------- */
/* Definition (Rank): rank(x -> y) over batch W. */
uint32_t orc_rank(const uint32_t *W, uint32_t w, uint32_t x, uint32_t y);
/* Lemma (rankAll): 2w records in the paper's output order (src ascending,
 * pos descending); pos is 0-based. */
void orc_rank_all(const uint32_t *W, uint32_t w, uint32_t *src, uint32_t *dst,
                  uint32_t *rank, uint32_t *pos);
/* Level-2 naming scheme for f1 = {u,v} (u,v as given, not canonicalised):
 * phi -> position of the named edge in W, with ld = rank(u -> v). */
uint32_t orc_phi_pos(const uint32_t *W, uint32_t w, uint32_t u, uint32_t v,
                     uint32_t phi);

#ifdef __cplusplus
}
#endif
#endif
