/*
 * tc.h -- C-ABI of the MI355X (gfx950) bulk update of neighborhood-sampling
 * triangle-count estimators.
 *
 * Method: Tangwongsan, Pavan, Tirthapura, "Parallel Triangle Counting in
 * Massive Streaming Graphs".  An estimator is a tuple (f1, f2, f3, chi)
 * satisfying the neighborhood sampling invariant (Sec. 3.1, Invariant 1);
 * one call of tc_process_batch is one bulkUpdateAll (Sec. 4, Theorem 3):
 * Step 1 level-1 reservoir (Sec. 4.2), Step 2 rank-based level-2 resample
 * and chi update (Sec. 4.3), Step 3 closing-edge check (Sec. 4.4).  The
 * estimate is Lemma 1's X = chi * |E| (when closed) averaged over the bank.
 *
 * Conventions shared by every entry point:
 *   - A batch is `uint32_t edges[2*w]`, 8-byte aligned: edge j is
 *     {edges[2j], edges[2j+1]}, arrival order = j.  Edges must come from a simple undirected graph:
 *     each edge once in the whole stream, no self-loops.  A self-loop is
 *     detected on the device and reported as TC_EBADEDGE by the next
 *     synchronising call (the bank is then unspecified).  Repeated edges
 *     are not detected; results stay deterministic.
 *   - An edge is reported as canon(a,b) = ((uint64)min << 32) | max; the
 *     empty edge is TC_EMPTY_EDGE.
 *   - Random decisions come from a counter-based generator keyed by
 *     (seed, estimator index within its bank, batch index of that bank,
 *     purpose, attempt): the splitmix64 finalizer chained over the key and
 *     Lemire's multiply-shift with rejection.  Results therefore depend on
 *     how the stream is cut into batches, and on nothing else (no launch
 *     shape, tile size or device count changes them).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Enqueueing calls return before the GPU work finishes; device buffers
 *     passed to them must stay valid until the stream passes that point.
 *   - Integer returns are TC_OK (0) or a negative TC_E* code; the text of
 *     the last error is available from tc_last_error() (per thread).
 *   - One object must not be used from two host threads, or enqueued on two
 *     streams, at the same time.
 */
#ifndef TC_H
#define TC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_OK 0
#define TC_EINVAL (-1)    /* bad argument (null pointer, size out of range) */
#define TC_EBADEDGE (-2)  /* a self-loop was found in a batch */
#define TC_EOVERFLOW (-3) /* an adjacency count chi reached 2^31 */
#define TC_ENOMEM (-4)    /* device or pinned host allocation failed */
#define TC_EHIP (-5)      /* a HIP runtime call failed */

#define TC_EMPTY_EDGE UINT64_MAX
#define TC_MAX_BATCH (1u << 28) /* largest w accepted by one call */

typedef struct tc_state tc_state; /* one bank of r estimators, one stream */
typedef struct tc_multi tc_multi; /* many independent banks */

/* ---- single bank (the plain method) ------------------------------------ */

/* Allocate a bank of r >= 1 estimators on the current HIP device with every
 * estimator empty (f1 = f2 = empty, chi = 0, not closed), |E| = 0 and batch
 * index 0.  The library owns all device memory.  Returns NULL on r == 0 or
 * allocation failure (see tc_last_error). */
tc_state *tc_create(uint32_t r, uint64_t seed);

/* Enqueue one bulk update (Sec. 4, bulkUpdateAll) of the bank with the batch
 * `edges` (DEVICE pointer to uint32[2w], caller-owned, read-only) on
 * `stream`; afterwards |E| += w and the batch index += 1.  w == 0 is a
 * no-op that does not advance the batch index.  Returns TC_EINVAL for a
 * NULL state, NULL or misaligned edges with w > 0, or w > TC_MAX_BATCH;
 * TC_ENOMEM if scratch for a larger batch cannot be allocated; earlier
 * sticky device errors are returned here once known. */
int tc_process_batch(tc_state *s, const uint32_t *edges, uint32_t w,
                     void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * bulk update as tc_process_batch, with the same kernels and a bit-identical
 * result, but every per-step buffer (arcs, radix counts, directory, Step-3
 * join partitions, per-estimator step words) is carved from a static device
 * array of the library, 64 MiB on each device, held from the first
 * tc_create on that device until the process ends.  The call allocates
 * and frees nothing, never synchronises, and only enqueues kernels on
 * `stream`.  Limits: the batch's and bank's scratch must fit the array and
 * its 2^20-slot directory (every w <= 2^18 with r <= 2^18 fits; a larger
 * pair is checked on the host and refused with TC_EINVAL, nothing enqueued).
 * All calls on one device share the array: calls that overlap in time on
 * one device (different host threads or unordered streams) race and give
 * undefined results; order them, for instance on one stream.  May be mixed
 * with tc_process_batch on the same bank.  TC_EINVAL also for kernel timing
 * switched on; other arguments and errors as tc_process_batch. */
int tc_process_batch_noalloc(tc_state *s, const uint32_t *edges, uint32_t w,
                             void *stream);

/* Enqueue one batch by the per-estimator form that the bulk algorithm
 * improves on (Sec. 4, opening): every estimator scans the whole batch
 * itself, O(r * w) work, from the definitions of Steps 1-3.  It makes the
 * same random draws and the same state transitions as tc_process_batch, so
 * the two may be mixed on one bank and give bit-identical states; it is
 * meant for checking and for small r * w.  Same arguments, lifetime and
 * errors as tc_process_batch. */
int tc_process_batch_naive(tc_state *s, const uint32_t *edges, uint32_t w,
                           void *stream);

/* Enqueue a whole resident stream: the m edges at DEVICE address edges
 * (uint32_t[2*m], 8-byte aligned) cut into ceil(m/w) consecutive batches of
 * w edges (the last one ragged), each one bulkUpdateAll in stream order.
 * The result is bit-identical to that many tc_process_batch calls on the
 * same cuts.  Inside the call, the closing-edge check (Step 3) of batch k
 * runs on an internal stream while batch k+1 is grouped on `stream`; the
 * call joins that stream back before it returns, so work enqueued on
 * `stream` afterwards sees every batch complete, and the call may be
 * captured into a HIP graph.  TC_EINVAL for a NULL state, NULL edges with
 * m > 0, w == 0 or w > TC_MAX_BATCH; on any error the batches before the
 * failing one stay enqueued. */
int tc_process_stream(tc_state *s, const uint32_t *edges, uint64_t m,
                      uint32_t w, void *stream);

/* Enqueue a whole stream held in HOST memory (the paper's input path: its
 * I/O routine reads the edge list from storage while the update runs; Sec.
 * 5, Table 2's I/O column): host_edges is uint32_t[2*m], cut into
 * ceil(m/w) batches of w edges exactly as tc_process_stream cuts a resident
 * stream, with a bit-identical result.  Batch k is copied into one of two
 * library-owned device staging buffers (2 * 8w bytes, kept and reused by
 * later calls, freed by tc_destroy) on an internal copy stream while batch
 * k - 1 is processed on `stream`; each batch's step waits for its copy.
 * Page-locked host memory (hipHostMalloc, or a pinned torch tensor) gives
 * asynchronous full-rate copies; pageable memory works too, but its copies
 * may block the calling thread.  The host array must stay valid and
 * unchanged until `stream` has passed this call's work.  Not capturable
 * (TC_EINVAL while `stream` is being captured).  TC_EINVAL for a NULL
 * state, NULL host_edges with m > 0, w == 0 or w > TC_MAX_BATCH; TC_ENOMEM
 * if the staging buffers cannot be allocated; on any error the batches
 * before the failing one stay enqueued. */
int tc_process_host_stream(tc_state *s, const uint32_t *host_edges,
                           uint64_t m, uint32_t w, void *stream);

/* Declare that every vertex id of this bank's stream is below n
 * (2 <= n <= 2^32; the default is 2^32).  The grouping sort then runs only
 * as many radix passes as n - 1 needs: its bytes in 8-bit digits, or two
 * passes of 10-bit digits when n - 1 has 17 to 20 bits; fewer kernel
 * launches per batch.  An id >= n in a later batch is detected on the device: that step
 * is abandoned and the next synchronising call returns TC_EINVAL (sticky;
 * the bank is then unspecified).  Applies to batches enqueued afterwards.
 * TC_EINVAL for n out of range. */
int tc_set_vertex_bound(tc_state *s, uint64_t n);

/* ---- launch shapes (batched-form tuning) ---------------------------------
 * Shapes of the step's kernels that a tuner may choose; none of them
 * changes any result (the state stays bit-identical, as the tests check).
 *   digit_bits      0: radix digits from the declared vertex bound (two
 *                   passes of 10-bit digits for bounds of 17 to 20 bits,
 *                   else 8-bit digits; the default); 8: always 8-bit
 *   chunk_tiles     radix tiles (of 4096 arcs) per chunk of the reduce-then-
 *                   scan: 8, 16 or 32 (default 32)
 *   part_estimators Step-3 join: waiting estimators per hash partition aimed
 *                   at, a power of two in [512, 8192] (default 2048; at
 *                   most 2048 partitions per bank)
 *   join_edges      Step-3 join: batch edges per join block aimed at, a
 *                   power of two in [1024, 65536] (default 8192)
 *   fused_edges     chunks of at most this many edges (0..2048; default
 *                   2048) run the whole step in one fused launch, in LDS,
 *                   with no scratch (not while the stream is being
 *                   captured, where every chunk takes the chain of kernels)
 * Applies to steps enqueued afterwards; TC_EINVAL for values out of range.
 * tc_step_bytes_max and tc_multi_reserve_max hold for every tuning. */
typedef struct tc_tuning {
  uint32_t digit_bits;
  uint32_t chunk_tiles;
  uint32_t part_estimators;
  uint32_t join_edges;
  uint32_t fused_edges;
} tc_tuning;
int tc_set_tuning(tc_state *s, const tc_tuning *t);
int tc_get_tuning(const tc_state *s, tc_tuning *t);
int tc_multi_set_tuning(tc_multi *s, const tc_tuning *t);
int tc_multi_get_tuning(const tc_multi *s, tc_tuning *t);

/* Pre-size the bank's step scratch for batches of up to max_w edges so that
 * later tc_process_batch calls with w <= max_w allocate nothing (needed
 * before capturing them into a HIP graph: a captured step that needs more
 * scratch than reserved returns TC_EINVAL before it synchronises, allocates
 * or enqueues anything).  Once some step has been captured, a later growth
 * of the scratch keeps the old block alive (captured graphs hold its
 * addresses) until tc_destroy, or tc_multi_graph_reserve for a tc_multi.
 * Blocking.  TC_ENOMEM on failure. */
int tc_reserve(tc_state *s, uint32_t max_w);

/* Enqueue on `stream` a return of every estimator to empty, with |E| = 0
 * and batch index 0 (as after tc_create).  Uses kernels only, so it may be
 * captured into a HIP graph ahead of captured steps. */
int tc_reset(tc_state *s, void *stream);

/* Block until the bank's last enqueued work is done, then return
 * tau_hat = (|E| / r) * S with S = sum_i chi_i * [closed_i] (Lemma 1, mean
 * aggregate).  NaN on error. */
double tc_estimate(tc_state *s);

/* Blocking; writes S (exact, 64-bit), |E| and tau_hat.  Any pointer may be
 * NULL.  Returns TC_OK or a sticky device error. */
int tc_estimate_ex(tc_state *s, uint64_t *S, uint64_t *m, double *tau);

/* Blocking; the median-of-means aggregate the paper applies to its
 * estimators (Sec. 3.1, before Theorem 2; Sec. 5): the r estimators are cut
 * into `groups` contiguous groups, group k = [floor(k r/g), floor((k+1) r/g)),
 * each group's mean of Lemma 1's X is (|E| / size_k) * S_k with S_k the
 * exact sum of chi * closed over the group, and *tau receives the median
 * of the g means (the mean of the two middle ones for even g).  group_sums
 * (a HOST array of length g, may be NULL) receives the S_k.  tau may be
 * NULL.  TC_EINVAL unless 1 <= groups <= r. */
int tc_estimate_mom(tc_state *s, uint32_t groups, double *tau,
                    uint64_t *group_sums);

/* Theorem 2: the number of estimators that suffices for an
 * (eps, delta)-approximation of the triangle count of a graph with m edges,
 * maximum degree maxdeg and tau triangles:
 * ceil(96 / eps^2 * m * maxdeg / tau * ln(1 / delta)) (the logarithm read as
 * natural).  0 unless eps > 0, 0 < delta < 1 and tau > 0.  Pure host
 * function. */
uint64_t tc_estimators_needed(double eps, double delta, uint64_t m,
                              uint64_t maxdeg, double tau);

/* ---- device memory accounting (admission by memory budget) -------------
 * tc_bank_bytes: device bytes one bank of r estimators holds for its life
 * (36 per estimator: f1, f2, the packed chi/closed word and three per-step
 * words, plus 16 per bank).  tc_step_bytes: the step scratch a step made of
 * these nchunks chunks (chunk k: a bank of r[k] estimators, w[k] edges)
 * needs; an object's scratch grows to the largest step it has run and is
 * then reused.  0 for invalid arguments (w[k] > TC_MAX_BATCH or r[k] == 0).
 * Pure host functions.  tc_device_bytes / tc_multi_device_bytes: the bytes
 * the object holds on the device now (banks, step scratch, blocks kept for
 * captured graphs, host-ingest staging), as requested from hipMalloc
 * (the allocator may round each allocation up). */
uint64_t tc_bank_bytes(uint32_t r);
uint64_t tc_step_bytes(uint32_t nchunks, const uint32_t *r, const uint32_t *w);

/* tc_step_bytes_max: bytes of a step scratch that holds EVERY step of at
 * most nchunks chunks of banks of at most r_max estimators with at most
 * total_w edges in all (0 if an argument is 0).  tc_multi_reserve_max
 * grows the object's scratch to that size (r_max = its largest bank), so
 * that such steps never allocate afterwards: a server that caps its steps
 * at nchunks chunks and total_w edges holds at most
 * sum_b tc_bank_bytes(r_b) + 16 + tc_step_bytes_max(...) bytes of device
 * memory.  Blocking; TC_EINVAL if nchunks exceeds the banks; TC_ENOMEM. */
uint64_t tc_step_bytes_max(uint32_t nchunks, uint32_t r_max, uint64_t total_w);
int tc_multi_reserve_max(tc_multi *s, uint32_t nchunks, uint64_t total_w);
int tc_device_bytes(const tc_state *s, uint64_t *bytes);
int tc_multi_device_bytes(const tc_multi *s, uint64_t *bytes);

/* Blocking; copies the bank into caller-owned HOST arrays of length r:
 * f1, f2 (canonical codes), chi and closed (0/1).  Any pointer may be NULL. */
int tc_read_state(tc_state *s, uint64_t *r1, uint64_t *r2, uint32_t *c,
                  uint8_t *closed);

/* Blocking; waits for the bank's enqueued work and returns any device error. */
int tc_sync(tc_state *s);

/* Number of estimators, edges seen and batches consumed so far. */
uint32_t tc_num_estimators(const tc_state *s);
uint64_t tc_edges_seen(const tc_state *s);
uint64_t tc_batches_seen(const tc_state *s);

/* Wait for outstanding work, then free every resource.  NULL is a no-op. */
void tc_destroy(tc_state *s);

/* Text of the calling thread's last error ("" if none). */
const char *tc_last_error(void);

/* ---- many independent banks (batched and served forms) ----------------- */

/* nbanks banks; bank b has r[b] >= 1 estimators and seed seeds[b].  Each
 * bank behaves exactly as a tc_state fed the same batches. */
tc_multi *tc_multi_create(uint32_t nbanks, const uint32_t *r,
                          const uint64_t *seeds);

/* Enqueue one step: chunk k (k < nchunks) is a batch of w[k] edges at DEVICE
 * address edges[k] for bank bank_ids[k].  Bank ids must be distinct within
 * a call (one batch per bank per step); banks not named are untouched.  All
 * chunks advance in one set of kernel launches.  The three arrays are
 * HOST arrays read before the call returns. */
int tc_multi_process(tc_multi *s, uint32_t nchunks, const uint32_t *bank_ids,
                     const uint32_t *const *edges, const uint32_t *w,
                     void *stream);

/* Pre-size the step scratch as a tc_multi_process call with these chunks
 * would (edge pointers are not needed).  Blocking. */
int tc_multi_reserve(tc_multi *s, uint32_t nchunks, const uint32_t *bank_ids,
                     const uint32_t *w);

/* Enqueue a reset of every bank (see tc_reset). */
int tc_multi_reset(tc_multi *s, void *stream);

/* Enqueue a restart of bank `bank` as an empty bank with a new seed (|E| = 0,
 * batch index 0; its size r stays).  Lets a serving loop hand a bank slot
 * to a new stream once the previous stream is finished and read out. */
int tc_multi_assign(tc_multi *s, uint32_t bank, uint64_t seed, void *stream);

/* As tc_set_vertex_bound, for every bank of the object. */
int tc_multi_set_vertex_bound(tc_multi *s, uint64_t n);

/* Prepare to capture up to nsteps tc_multi_process calls into a HIP graph:
 * each captured step gets its own pinned descriptor buffer, left unchanged
 * so that every replay of the graph reads the step it captured.  Call after
 * tc_multi_reserve and before capturing; calling it again discards the
 * buffers of earlier captures (their graphs must not be replayed after).
 * A captured graph that starts with tc_multi_reset replays the same
 * computation every time; without the reset each replay continues the
 * banks with the captured batch indices. */
int tc_multi_graph_reserve(tc_multi *s, uint32_t nsteps);

/* Blocking; per-bank S, |E| and tau_hat into HOST arrays of length nbanks
 * (any may be NULL). */
int tc_multi_estimate(tc_multi *s, uint64_t *S, uint64_t *m, double *tau);

/* Blocking; tc_estimate_mom for bank `bank`. */
int tc_multi_estimate_mom(tc_multi *s, uint32_t bank, uint32_t groups,
                          double *tau, uint64_t *group_sums);

/* Blocking; like tc_read_state for bank `bank`. */
int tc_multi_read_state(tc_multi *s, uint32_t bank, uint64_t *r1, uint64_t *r2,
                        uint32_t *c, uint8_t *closed);

int tc_multi_sync(tc_multi *s);
uint32_t tc_multi_num_banks(const tc_multi *s);
void tc_multi_destroy(tc_multi *s);

/* ---- input: text edge lists ------------------------------------------------
 * Parse a text edge list held in DEVICE memory (the graphs the paper streams
 * are text edge lists, read by its I/O routine: Sec. 5, Table 2): one edge
 * per line, two unsigned decimal vertex ids separated by any non-digit
 * bytes; lines starting with '#' or '%' are comments; '\r\n' and a missing
 * final newline are accepted.  Writes the edges in file order to the DEVICE
 * array edges (uint32_t[2 * max_edges], caller-owned) and their number to
 * *nedges (HOST).  Blocking (it returns the count).  TC_EINVAL for NULL
 * pointers, an odd number of ids, an id above 2^32 - 1, a line longer than
 * 4096 bytes, or more than max_edges edges (nothing useful is written
 * then); TC_ENOMEM if its scratch cannot be allocated.  Its device
 * scratch (about a sixteenth of the text size) is kept per device, grown to
 * the largest text parsed so far and reused by later calls until the
 * process ends; calls from several host threads are serialised.  It waits
 * for `stream`, so it cannot be captured into a HIP graph. */
int tc_parse_edges(const char *text, uint64_t nbytes, uint32_t *edges,
                   uint64_t max_edges, uint64_t *nedges, void *stream);

/* ---- diagnostics: per-kernel device time --------------------------------
 * mask: bit k (k < tc_num_kernels()) times kernel k; TC_TIME_ALL times every
 * kernel; 0 turns timing off.  While on, every step records a HIP event
 * before and after each timed kernel on the stream that kernel runs on
 * (about 2 us of device time per event, so time few kernels when the step
 * time itself matters).  Changing the mask resets the totals.
 * tc_kernel_times blocks, then writes the accumulated milliseconds of each
 * of the tc_num_kernels() launches of a step (launch order; names from
 * tc_kernel_name; 0 for untimed kernels) into the HOST array `ms` and the
 * number of timed steps into *steps.  Timing must be off while a stream is
 * being captured into a HIP graph (TC_EINVAL otherwise). */
#define TC_TIME_ALL 0xFFFFFFFFu
int tc_set_kernel_timing(tc_state *s, uint32_t mask);
int tc_kernel_times(tc_state *s, double *ms, uint64_t *steps);
int tc_multi_set_kernel_timing(tc_multi *s, uint32_t mask);
int tc_multi_kernel_times(tc_multi *s, double *ms, uint64_t *steps);
int tc_num_kernels(void);
const char *tc_kernel_name(int k);

/* ---- diagnostics: random cache-line read rate ---------------------------
 * Not part of the method: measures how many random cache-line reads per
 * second the device serves, the ceiling of a kernel whose time goes to
 * independent random line reads (Step 2's directory, inverse-index, arc and
 * edge lookups, Sec. 4.3).  table: DEVICE buffer of table_bytes (a multiple
 * of 128; only read, contents arbitrary); sink: DEVICE uint32_t[n], written
 * (caller-owned).  n threads each read per_thread (1..8) words, each the
 * first word of a 128-byte line of the table chosen by a counter-based
 * hash; dependent = 1 makes each address depend on the word read before.
 * The kernel runs once untimed, then reps times between two events on
 * `stream`; *lines_per_s (HOST) gets n * per_thread * reps / elapsed.
 * Blocking.  TC_EINVAL for NULL pointers, table_bytes 0 or not a multiple
 * of 128, n == 0, per_thread outside 1..8 or reps == 0; TC_EHIP if a HIP
 * call fails. */
int tc_probe_line_rate(const void *table, uint64_t table_bytes, uint32_t n,
                       uint32_t per_thread, uint32_t dependent, uint32_t reps,
                       uint32_t *sink, double *lines_per_s, void *stream);

#ifdef __cplusplus
}
#endif
#endif
