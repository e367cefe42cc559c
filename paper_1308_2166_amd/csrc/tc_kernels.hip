// Device kernels of the bulk estimator update (Tangwongsan, Pavan,
// Tirthapura, Sec. 4: bulkUpdateAll) for gfx950.
//
// One step = k_hist -> k_fold_step1 -> k_cscan<0> -> k_scat<0> -> up to
// 3 x (k_cnt -> k_csum -> k_cscan -> k_scat) -> k_dir -> k_est -> k_pcnt ->
// k_pscan -> k_pscat -> k_pjoin.
//
//  k_hist   per-tile counts of digit 0 of the 2w arcs (+ max id, self-loop
//           check)
//  k_fold_step1
//           chunk sums and per-segment digit histograms from the per-tile
//           counts (which become prefixes within their chunk); Step 1
//           (which estimators take a new f1, from where)
//  k_cnt, k_csum, k_cscan, k_scat
//           stable LSD radix pass over D bits of the vertex id (D = 8, or
//           10 when a declared vertex bound makes that two passes not three)
//           (reduce-then-scan: tile counts, chunk sums and in-chunk tile
//           prefixes, chunk bases, and a scatter that reads its offsets in
//           two rows, ranks with wave64 ballots and writes through LDS,
//           coalesced).  Arcs are (vertex << 32 | 2 pos + side); stability keeps every
//           vertex's arcs in arrival order, which is the rankAll grouping
//           of the Lemma on rankAll read in increasing pos (rank = arcs
//           after it in the segment).  A pass whose digit is zero for
//           every arc of a segment (above its largest id) is skipped on the
//           device, and passes above a declared vertex bound are not
//           launched.
//  k_dir    vertex -> [start, end) of its arcs (CSR offsets, or a
//           tag-versioned hashed directory for sparse ids), and the sorted
//           index of the arcs of positions Step 1 picked
//  k_est    Step 2 for every estimator; records its Step-3 closing edge
//  k_pcnt, k_pscan, k_pscat
//           Step 3: batch edges and waiting estimators counted, offset and
//           scattered into hash partitions of their (closing) edge
//  k_pjoin  Step 3: per partition, the waiting estimators in an LDS hash
//           table, the partition's batch edges streamed through it
#include <algorithm>

#include "tc_internal.h"

namespace tc {

static_assert(kHistTiles == 1, "k_hist rows double as per-tile radix counts");

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // splitmix64 output finalizer (Steele, Lea, Flood 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // a 32-bit bijective avalanche mixer (xorshift-multiply rounds)
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint64_t canon(uint32_t a, uint32_t b) {
  return a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
}

// Uniform integer in [0, n), n >= 1: Lemire's multiply-shift with rejection
// over the keyed stream mix64(kb ^ (purpose * golden + attempt)).
__device__ __forceinline__ uint64_t bounded(uint64_t kb, uint64_t purpose,
                                            uint64_t n) {
  for (uint64_t att = 0;; ++att) {
    const uint64_t x = mix64(kb ^ (purpose * kGolden + att));
    const uint64_t lo = x * n;
    const uint64_t hi = __umul64hi(x, n);
    if (lo >= n) return hi;  // outside the zone that needs the threshold
    const uint64_t t = (0ull - n) % n;
    if (lo >= t) return hi;
  }
}

// the edge closing the wedge f1, f2 (the endpoints they do not share)
__device__ __forceinline__ uint64_t closing(uint64_t f1, uint64_t f2) {
  if (f1 == f2) return kEmpty;
  const uint32_t a = (uint32_t)(f1 >> 32), b = (uint32_t)f1;
  const uint32_t x = (uint32_t)(f2 >> 32), y = (uint32_t)f2;
  if (a == x || a == y) return canon(b, a == x ? y : x);
  if (b == x || b == y) return canon(a, b == x ? y : x);
  return kEmpty;
}


// segment of a global tile: the last segment whose tile_off <= gtile
__device__ __forceinline__ uint32_t seg_of_tile(const StepArgs& a,
                                                uint32_t gtile) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].tile_off <= gtile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// segment of a k_hist block
__device__ __forceinline__ uint32_t seg_of_hblk(const StepArgs& a,
                                                uint32_t b) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].hblk_off <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// segment of a flat estimator thread
__device__ __forceinline__ uint32_t seg_of_est(const StepArgs& a,
                                               uint64_t gid) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].gest_off <= gid) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// descriptor by value: kept in registers (scalar ones when s is uniform),
// never re-read through a pointer inside the loops
__device__ __forceinline__ SegDesc seg_desc(const StepArgs& a, uint32_t s) {
  return a.nseg == 1 ? a.seg0 : a.segs[s];
}

// Kernels with one thread per estimator index the descriptor per thread,
// which the compiler turns into vector loads through a pointer for both
// cases; their single-segment builds (kOne) take the descriptor straight
// from the kernel arguments instead (scalar loads issued at the start).
template <bool kOne>
__device__ __forceinline__ SegDesc est_seg_desc(const StepArgs& a, uint32_t s) {
  if constexpr (kOne) return a.seg0;
  return a.segs[s];
}

// Segment of estimator thread gid in a block of consecutive estimator
// threads starting at gid0 (every thread of the block calls it): thread 0
// searches gid0's segment and the start of the one after it, and only a
// thread at or past that start (a block that crosses a segment's end)
// searches for itself.
__device__ __forceinline__ uint32_t block_seg_of_est(const StepArgs& a, uint64_t gid0,
                                                     uint64_t gid, uint32_t* s_seg,
                                                     uint64_t* s_next) {
  if (threadIdx.x == 0) {
    const uint32_t s = seg_of_est(a, gid0);
    *s_seg = s;
    *s_next = s + 1 < a.nseg ? a.segs[s + 1].gest_off : ~0ull;
  }
  __syncthreads();
  return gid < *s_next ? *s_seg : seg_of_est(a, gid);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// The hardware deals a launch's workgroups to the eight XCDs in turn (XCD =
// index mod 8), each XCD with its own L2.  The radix kernels map their tile
// index through this bijection of [0, n) so that the tiles one XCD receives
// come in runs of eight: neighbouring tiles' runs of a digit then mostly
// meet in the same L2.  (The kernels with random accesses keep the plain order, which spreads
// a segment's tables over all eight L2s.)
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
  // groups of 64 blocks: within a group XCD x takes its 8 consecutive tiles,
  // so the launch's window of active tiles stays contiguous; the last,
  // partial group keeps the plain order
  if (b >= (n & ~63u)) return b;
  return (b & ~63u) + ((b & 7u) << 3) + ((b >> 3) & 7u);
}

// exclusive scan of one value per thread over the block (kBlock threads)
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v,
                                                    uint32_t* s_tmp,
                                                    uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t t = s_tmp[w];
    off += (w < wave) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// ---------------------------------------------------------------------------
// Radix layout for D-bit digits: kBins bins; in every per-digit step thread
// t owns the kPer consecutive bins [kPer t, kPer t + kPer), moved as one
// word or one uint4.  A tile's (chunk's, segment's) counts of pass P start
// at word P << D of its kRowWords-word row.
// ---------------------------------------------------------------------------
template <int D>
struct Rdx {
  static constexpr int kBins = 1 << D;
  static constexpr int kPer = kBins / kBlock;
  static constexpr uint32_t kMask = kBins - 1;
  static_assert(kPer == 1 || kPer == 4, "one word or one uint4 of bins per thread");
  static_assert(kPasses * 8 >= 32 && kWidePasses * kWideBits <= 32, "id widths");
};

// this thread's kPer bins at p + kPer * tid (global or LDS, 16-byte aligned)
template <int N>
__device__ __forceinline__ void ld_bins(const uint32_t* p, uint32_t (&v)[N]) {
  if constexpr (N == 1) {
    v[0] = p[threadIdx.x];
  } else {
    static_assert(N == 4, "bins per thread");
    const uint4 q = reinterpret_cast<const uint4*>(p)[threadIdx.x];
    v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
  }
}
template <int N>
__device__ __forceinline__ void st_bins(uint32_t* p, const uint32_t (&v)[N]) {
  if constexpr (N == 1) {
    p[threadIdx.x] = v[0];
  } else {
    static_assert(N == 4, "bins per thread");
    reinterpret_cast<uint4*>(p)[threadIdx.x] = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// ---------------------------------------------------------------------------
// k_hist: per-tile counts of digit 0 of the arc keys
// ---------------------------------------------------------------------------
// add one to bin `dg`; a digit shared by the whole wave costs one atomic
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t dg, bool valid) {
  const uint32_t d0 = __shfl(dg, 0);
  const uint64_t act = __ballot(valid);
  if (__all(!valid || dg == d0) && act) {
    if ((threadIdx.x & 63) == (uint32_t)(__ffsll((long long)act) - 1))
      atomicAdd(&h[d0], (uint32_t)__popcll(act));
  } else if (valid) {
    atomicAdd(&h[dg], 1u);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_hist(StepArgs a) {
  using R = Rdx<D>;
  __shared__ __align__(16) uint32_t h[R::kBins];
  __shared__ uint32_t s_max;
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x;
  const uint32_t hb = blockIdx.x;
  if (tid == 0) {
    s_seg = seg_of_hblk(a, hb);
    s_max = 0;
  }
  // this step's directory entries get a fresh tag (0 means empty); every
  // reader of the tag runs after this kernel
  if (hb == 0 && tid == 0) {
    const uint32_t t = *a.tagp + 1u;
    *a.tagp = t ? t : 1u;
  }
#pragma unroll
  for (int j = 0; j < R::kPer; ++j) h[tid + j * kBlock] = 0;
  __syncthreads();
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  const uint32_t n = 2u * S.w;
  const uint32_t abase = (hb - S.hblk_off) * (uint32_t)(kHistTiles * kTile);
  const uint32_t aend = min(abase + (uint32_t)(kHistTiles * kTile), n);
  uint32_t vmax = 0;
  bool loop = false;
  const bool vec = (reinterpret_cast<uintptr_t>(S.edges) & 15u) == 0;
  // four arcs (two edges) per thread and round; every round's load is
  // issued before the first is used
  constexpr int kRounds = kHistTiles * kTile / (4 * kBlock);
  uint4 xs[kRounds];
  if (vec && abase + kHistTiles * kTile <= aend) {
    // a whole aligned tile: no conditions, so all loads are in flight at once
    const uint4* e4 = reinterpret_cast<const uint4*>(S.edges + abase);
#pragma unroll
    for (int it = 0; it < kRounds; ++it) xs[it] = e4[tid + it * kBlock];
  } else {
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
      const uint32_t i = abase + 4 * tid + it * 4 * kBlock;
      uint4 x = make_uint4(0, 0, 0, 0);
      const bool full = i + 4 <= aend;
      if (full && vec) {
        x = *reinterpret_cast<const uint4*>(S.edges + i);
      } else if (full) {
        const uint2 e0 = *reinterpret_cast<const uint2*>(S.edges + i);
        const uint2 e1 = *reinterpret_cast<const uint2*>(S.edges + i + 2);
        x = make_uint4(e0.x, e0.y, e1.x, e1.y);
      } else if (i < aend) {  // ragged tail: i is even, so i + 1 < aend
        const uint2 e0 = *reinterpret_cast<const uint2*>(S.edges + i);
        x.x = e0.x;
        x.y = e0.y;
      }
      xs[it] = x;
    }
  }
  // clear the need bytes (Step 1 marks them next) while the loads above
  // are in flight
  {
    uint4* n4 = reinterpret_cast<uint4*>(a.need);
    for (uint64_t t = (uint64_t)hb * kBlock + tid; t < a.need_bytes / 16;
         t += (uint64_t)a.nhblk * kBlock)
      n4[t] = make_uint4(0, 0, 0, 0);
  }
#pragma unroll
  for (int it = 0; it < kRounds; ++it) {
    const uint32_t i = abase + 4 * tid + it * 4 * kBlock;
    const uint4 x = xs[it];
    const bool v01 = i < aend, v23 = i + 4 <= aend;
    if (v01) {
      loop |= x.x == x.y;
      vmax = max(vmax, max(x.x, x.y));
    }
    if (v23) {
      loop |= x.z == x.w;
      vmax = max(vmax, max(x.z, x.w));
    }
    // digit 0 only: the later passes count their own input order
    hist_add(h, x.x & R::kMask, v01);
    hist_add(h, x.y & R::kMask, v01);
    hist_add(h, x.z & R::kMask, v23);
    hist_add(h, x.w & R::kMask, v23);
  }
  if (loop) atomicOr(a.err, kErrSelfLoop);
  if (vmax > a.id_limit) atomicOr(a.err, kErrRange);
  atomicMax(&s_max, vmax);
  __syncthreads();
  // the block's counts go out with plain stores; the fold sums them, so
  // no global bin takes one atomic per block
  uint32_t v[R::kPer];
  ld_bins(h, v);
  st_bins(a.hpart + (size_t)hb * kRowWords, v);
  if (tid == 0) a.mpart[hb] = s_max;
}

// ---------------------------------------------------------------------------
// k_fold (in the k_fold_step1 launch): per radix chunk, the digit-0 sums of its
// tiles (the chunk sums of the first radix pass), added into the segment's
// digit-0 histogram; and the largest vertex id
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t seg_of_chunk(const StepArgs& a, uint32_t c) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].chunk_off <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// row of chunk c's digit sums (pass P) in the chunk-sum array
template <int D>
__device__ __forceinline__ uint32_t* csum_row(const StepArgs& a, uint32_t c, int P) {
  return a.csum + (size_t)c * kRowWords + ((size_t)P << D);
}

// row of tile t's digit counts (pass P) in the partial-count array
template <int D>
__device__ __forceinline__ uint32_t* cnt_row(const StepArgs& a, uint32_t t, int P) {
  return a.hpart + (size_t)t * kRowWords + ((size_t)P << D);
}

// What a count-sum block stores for its chunk: the chunk's sum of the
// thread's digit (k_cscan turns it into the chunk's base), or, when every
// segment is a single chunk and one block holds all 256 (8-bit) digits,
// the base itself: the digit's bin start, an exclusive scan of those sums.
template <int D>
__device__ __forceinline__ uint32_t single_chunk_base(const StepArgs& a, uint32_t tot) {
  if constexpr (D == 8) {
    __shared__ uint32_t s_tmp[kWaves];
    if (a.single_chunk) {
      uint32_t all;
      return block_excl_scan(tot, s_tmp, &all);
    }
  }
  return tot;
}

// Rows [r0, r1) (at most kChunk, kRowWords apart from `rows`) of one chunk,
// word d: each row is replaced by the exclusive prefix of the rows before
// it, and their total is returned.  All loads are in flight at once.
__device__ __forceinline__ uint32_t chunk_prefix(uint32_t* rows, uint32_t r0, uint32_t r1,
                                                 uint32_t d) {
  uint32_t v[kChunk];
#pragma unroll
  for (uint32_t i = 0; i < kChunk; ++i)
    v[i] = r0 + i < r1 ? rows[(size_t)(r0 + i) * kRowWords + d] : 0u;
  uint32_t run = 0;
#pragma unroll
  for (uint32_t i = 0; i < kChunk; ++i) {
    if (r0 + i < r1) rows[(size_t)(r0 + i) * kRowWords + d] = run;
    run += v[i];
  }
  return run;
}

// block b of the fold: chunk b / kPer, digits (b % kPer) kBlock + [0, kBlock)
template <int D>
__device__ void fold_chunk(const StepArgs& a, uint32_t b) {
  using R = Rdx<D>;
  __shared__ uint32_t s_seg, s_max;
  const int tid = threadIdx.x;
  const uint32_t c = b / R::kPer, q = b % R::kPer;
  if (tid == 0) {
    s_seg = seg_of_chunk(a, c);
    s_max = 0;
  }
  __syncthreads();
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  const uint32_t r0 = S.hblk_off + ((c - S.chunk_off) << a.chunk_log2);
  const uint32_t r1 = min(r0 + (1u << a.chunk_log2), S.hblk_off + S.nhblk);
  const uint32_t d = q * kBlock + tid;
  const uint32_t tot = chunk_prefix(a.hpart, r0, r1, d);
  if (q == 0 && (uint32_t)tid < r1 - r0) atomicMax(&s_max, a.mpart[r0 + tid]);
  __syncthreads();
  SegWork* wk = a.work + sidx;
  csum_row<D>(a, c, 0)[d] = single_chunk_base<D>(a, tot);
  if (tot) atomicAdd(&wk->hist[d], tot);
  if (q == 0 && tid == 0) atomicMax(&wk->maxid, s_max);
}

// ---------------------------------------------------------------------------
// Radix passes.  Pass P orders the arcs stably by bits DP..DP+D-1 of the
// vertex id (LSD), by reduce-then-scan: k_cnt<P> counts the digits of every
// tile, k_csum<P> sums the counts of every chunk of tiles (and the
// segment's digit histogram) and turns each tile's counts into the prefix
// of its chunk's earlier tiles, k_cscan<P> turns the chunk sums into chunk
// bases, and k_scat<P> adds its two offset rows and moves its arcs.  No
// block waits for another.  Passes above the largest vertex id's top digit
// are skipped on the device; pass 0 takes its counts from k_hist and the
// fold.
// ---------------------------------------------------------------------------

// Pass P runs for a segment iff some vertex id has a nonzero digit at or
// above P (max id >= 2^(DP)); otherwise digit P is zero for every arc and
// the pass would leave the order unchanged.  Pass 0 always runs (an edge
// has two distinct ids), so the passes that run are 0 .. K-1 and pass P
// reads buffer (P+1)&1 (W for P = 0) and writes buffer P&1.
template <int D>
__device__ __forceinline__ bool pass_runs(uint32_t maxid, int P) {
  return P == 0 || (maxid >> (D * P)) != 0u;
}

// bits of digit P that can be nonzero (the match needs only those; used
// from pass 2 on with 8-bit digits, where ids often stop short of the
// digit's top -- on the lower passes the early exit costs more than it
// saves -- and on every pass of wide digits)
template <int D>
__device__ __forceinline__ int digit_bits(uint32_t maxid, int P) {
  const uint32_t top = maxid >> (D * P);
  return top == 0u ? 1 : min(D, 32 - __clz(top));
}
template <int D>
__device__ __forceinline__ bool match_stops(int P) {
  return P >= 2;
}

template <int P, int D>
__global__ __launch_bounds__(kBlock) void k_cnt(StepArgs a) {
  static_assert(P >= 1, "k_hist counts the first pass");
  using R = Rdx<D>;
  __shared__ __align__(16) uint32_t s_h[R::kBins];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  if (tid == 0) s_seg = seg_of_tile(a, blk);
#pragma unroll
  for (int j = 0; j < R::kPer; ++j) s_h[tid + j * kBlock] = 0;
  __syncthreads();
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  const uint32_t n = 2u * S.w;
  const uint32_t maxid = uniform(a.work[sidx].maxid);
  if (!pass_runs<D>(maxid, P)) return;
  const int nbits = digit_bits<D>(maxid, P);
  const uint32_t base = (blk - S.tile_off) * kTile;
  const uint32_t nv = min((uint32_t)kTile, n - base);
  // high words (vertex ids) of the pass input, read in order
  const uint32_t* hi = reinterpret_cast<const uint32_t*>(a.arcs[(P + 1) & 1] + S.arc_off + base) + 1;
  uint32_t v[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) v[i] = hi[2u * min((uint32_t)(i * kBlock + tid), nv - 1)];
  uint32_t row[R::kPer];
  if (P == 1 && nbits >= 7) {
    // the second digit of arcs ordered by their first: most lanes of a
    // wave differ, and one LDS atomic per arc is cheaper than matching
    // equal digits first.  (From the third 8-bit digit on, arcs arrive
    // grouped by their low 16 bits, so a high-degree vertex fills many
    // lanes with one digit.)
#pragma unroll
    for (int i = 0; i < kItems; ++i)
      if ((uint32_t)(i * kBlock + tid) < nv) atomicAdd(&s_h[(v[i] >> (D * P)) & R::kMask], 1u);
    __syncthreads();
    ld_bins(s_h, row);
    st_bins(cnt_row<D>(a, blk, P), row);
    return;
  }
  // few digits: lanes with equal digits add once (one atomic per lane
  // would serialize on the few bins)
  const int lane = tid & 63;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = (uint32_t)(i * kBlock + tid) < nv;
    const uint32_t dg = (v[i] >> (D * P)) & R::kMask;
    const uint64_t vm = __ballot(valid);
    uint32_t lo = (uint32_t)vm, hi2 = (uint32_t)(vm >> 32);
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (match_stops<D>(P) && b >= nbits) break;  // higher digit bits are zero in every arc
      const uint32_t t = (uint32_t)((int32_t)(dg << (31 - b)) >> 31);
      const uint64_t bb = __ballot(t != 0u);
      lo = __builtin_amdgcn_bitop3_b32(lo, t, (uint32_t)bb, 0x90);
      hi2 = __builtin_amdgcn_bitop3_b32(hi2, t, (uint32_t)(bb >> 32), 0x90);
    }
    const uint64_t mm = ((uint64_t)hi2 << 32) | lo;
    if (valid && __popcll(mm & ((1ull << lane) - 1ull)) == 0)
      atomicAdd(&s_h[dg], (uint32_t)__popcll(mm));
  }
  __syncthreads();
  ld_bins(s_h, row);
  st_bins(cnt_row<D>(a, blk, P), row);
}

// block b: chunk b / kPer, digits (b % kPer) kBlock + [0, kBlock): the
// chunk's tile rows become prefixes, its sums go to csum and into the
// segment's digit-P histogram
template <int P, int D>
__global__ __launch_bounds__(kBlock) void k_csum(StepArgs a) {
  static_assert(P >= 1, "the fold sums the first pass");
  using R = Rdx<D>;
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x;
  const uint32_t c = blockIdx.x / R::kPer, q = blockIdx.x % R::kPer;
  if (tid == 0) s_seg = seg_of_chunk(a, c);
  __syncthreads();
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  SegWork* wk = a.work + sidx;
  if (!pass_runs<D>(uniform(wk->maxid), P)) return;
  const uint32_t t0 = S.tile_off + ((c - S.chunk_off) << a.chunk_log2);
  const uint32_t t1 = min(t0 + (1u << a.chunk_log2), S.tile_off + S.ntiles);
  const uint32_t d = q * kBlock + tid;
  const uint32_t tot = chunk_prefix(cnt_row<D>(a, 0, P), t0, t1, d);
  csum_row<D>(a, c, P)[d] = single_chunk_base<D>(a, tot);
  if (tot) atomicAdd(&wk->hist[(P << D) + d], tot);
}

// Each chunk sum of pass P becomes the chunk's base: the digit's bin start
// (an exclusive scan of the segment's digit histogram) plus the digit's
// arcs in the segment's earlier chunks.  A scatter block then finds its
// offsets in two rows.  Block b serves segment b / (kBins / 64) and the 64
// digits 64 (b % (kBins / 64)) + lane; wave w takes the w-th quarter of the
// segment's chunks, whose first kCscanBatch sums are loaded before the scan
// of the histogram (so the two waits overlap) and stay in registers (a
// quarter of more chunks loads the rest twice, in smaller batches).
constexpr uint32_t kCscanBatch = 64;
constexpr uint32_t kCscanMore = 16;  // loads per batch past the first

template <int P, int D>
__global__ __launch_bounds__(kBlock) void k_cscan(StepArgs a) {
  using R = Rdx<D>;
  constexpr uint32_t kGroups = R::kBins / 64;  // 64-digit groups per segment
  __shared__ __align__(16) uint32_t s_bin[R::kBins];
  __shared__ uint32_t s_part[kWaves][64];
  __shared__ uint32_t s_tmp[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t sidx = blockIdx.x / kGroups;
  const uint32_t d = (blockIdx.x % kGroups) * 64 + lane;
  const SegDesc S = seg_desc(a, sidx);
  SegWork* wk = a.work + sidx;
  if (!pass_runs<D>(uniform(wk->maxid), P)) return;
  const uint32_t nc = S.nchunks;
  const uint32_t per = (nc + kWaves - 1) / kWaves;
  const uint32_t c_lo = min((uint32_t)wave * per, nc), c_hi = min(c_lo + per, nc);
  uint32_t* col = csum_row<D>(a, S.chunk_off, P) + d;
  uint32_t v[kCscanBatch], sum = 0;
#pragma unroll
  for (uint32_t i = 0; i < kCscanBatch; ++i)
    v[i] = c_lo + i < c_hi ? col[(size_t)(c_lo + i) * kRowWords] : 0u;
  uint32_t h[R::kPer], bins[R::kPer], t = 0, tot;
  ld_bins(wk->hist + (P << D), h);
#pragma unroll
  for (int j = 0; j < R::kPer; ++j) t += h[j];
#pragma unroll
  for (uint32_t i = 0; i < kCscanBatch; ++i) sum += v[i];
  for (uint32_t c0 = c_lo + kCscanBatch; c0 < c_hi; c0 += kCscanMore) {
    uint32_t u[kCscanMore];
#pragma unroll
    for (uint32_t i = 0; i < kCscanMore; ++i)
      u[i] = c0 + i < c_hi ? col[(size_t)(c0 + i) * kRowWords] : 0u;
#pragma unroll
    for (uint32_t i = 0; i < kCscanMore; ++i) sum += u[i];
  }
  uint32_t bin = block_excl_scan(t, s_tmp, &tot);
#pragma unroll
  for (int j = 0; j < R::kPer; ++j) {
    bins[j] = bin;
    bin += h[j];
  }
  st_bins(s_bin, bins);
  s_part[wave][lane] = sum;
  __syncthreads();
  uint32_t run = s_bin[d];
#pragma unroll
  for (int k = 0; k < kWaves; ++k) run += k < wave ? s_part[k][lane] : 0u;
#pragma unroll
  for (uint32_t i = 0; i < kCscanBatch; ++i) {
    if (c_lo + i < c_hi) col[(size_t)(c_lo + i) * kRowWords] = run;
    run += v[i];
  }
  for (uint32_t c0 = c_lo + kCscanBatch; c0 < c_hi; c0 += kCscanMore) {
    uint32_t u[kCscanMore];
#pragma unroll
    for (uint32_t i = 0; i < kCscanMore; ++i)
      u[i] = c0 + i < c_hi ? col[(size_t)(c0 + i) * kRowWords] : 0u;
#pragma unroll
    for (uint32_t i = 0; i < kCscanMore; ++i) {
      if (c0 + i < c_hi) col[(size_t)(c0 + i) * kRowWords] = run;
      run += u[i];
    }
  }
}

template <int P, int D>
__device__ __forceinline__ void scat_body(const StepArgs& a) {
  using R = Rdx<D>;
  constexpr int kBins = R::kBins, kPer = R::kPer;
  // 8-bit digits: the per-wave bins and the tile's digit offsets have
  // arrays of their own (38 KB in all).  Wide digits: both live in the
  // staging buffer, whose use they precede, so a block still takes 36 KB
  // rather than 56 and a CU still holds four.
  constexpr bool kAlias = D > 8;
  static_assert((kWaves + 1) * kBins * 4 <= kTile * 8, "aliased bins fit the staging buffer");
  __shared__ __align__(16) uint64_t s_el[kTile];
  __shared__ __align__(16) uint32_t s_wh_own[kAlias ? 1 : kWaves * kBins];
  __shared__ __align__(16) uint32_t s_loc_own[kAlias ? 1 : kBins];
  __shared__ __align__(16) uint32_t s_dst[kBins];
  __shared__ uint32_t s_tmp[kWaves];
  __shared__ uint32_t s_seg;
  // s_wh[w * kBins + d]: wave w's arcs of digit d, then the offset of that
  // wave's first one among the tile's; s_loc[d]: the tile's first arc of d
  uint32_t* const s_wh = kAlias ? reinterpret_cast<uint32_t*>(s_el) : s_wh_own;
  uint32_t* const s_loc = kAlias ? reinterpret_cast<uint32_t*>(s_el) + kWaves * kBins : s_loc_own;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  if (tid == 0) s_seg = seg_of_tile(a, blk);
  __syncthreads();
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  SegWork* wk = a.work + sidx;
  const uint32_t n = 2u * S.w;
  const uint32_t maxid = uniform(wk->maxid);
  if (P == 0 && blk == S.tile_off && tid == 0) {
    int K = 0;  // passes run (the launched ones that do not skip)
#pragma unroll
    for (int d = 0; d < kPasses; ++d) K += (d < (int)a.npass && pass_runs<D>(maxid, d)) ? 1 : 0;
    wk->final_buf = (uint32_t)((K + 1) & 1);  // (K - 1) & 1, K >= 1
    const uint64_t span = (uint64_t)maxid + 1;
    wk->dense = span <= (1ull << S.dir_log2) ? 1u : 0u;
  }
  if (!pass_runs<D>(maxid, P)) return;
  const int nbits = digit_bits<D>(maxid, P);
  const uint32_t ltile = blk - S.tile_off;
  const uint64_t* src = a.arcs[(P + 1) & 1] + S.arc_off;
  uint64_t* dst = a.arcs[P & 1] + S.arc_off;
  const uint32_t base = ltile * kTile;
  const uint32_t nv = min((uint32_t)kTile, n - base);

  // load: wave w owns arcs [w*64*kItems, (w+1)*64*kItems) of the tile,
  // iteration i covers 64 consecutive arcs (original order = (i, lane))
  // branch-free loads (a clamped index past the ragged end) so that all
  // kItems loads are in flight together
  uint64_t el[kItems];
  uint32_t rk[kItems];
  if (P == 0) {
    // arcs straight from W: arc id = 2 pos + side, flagged when Step 1
    // takes some f1 from that position (read in order, so coalesced)
    const uint32_t* E = S.edges;
    const uint8_t* need = a.need + S.need_off;
    uint32_t ev[kItems], nb[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t gi = min(base + wave * 64 * kItems + i * 64 + lane, n - 1);
      ev[i] = E[gi];
      nb[i] = need[gi >> 1];
    }
    // (the arc id is recomputed, not kept; past the ragged end it is
    // never used)
#pragma unroll
    for (int i = 0; i < kItems; ++i)
      el[i] = ((uint64_t)ev[i] << 32) | (base + wave * 64 * kItems + i * 64 + lane) |
              (nb[i] ? kNeedFlag : 0u);
  } else {
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t gi = min(base + wave * 64 * kItems + i * 64 + lane, n - 1);
      el[i] = src[gi];
    }
  }
  // this tile's first arc of each of the thread's digits goes to: its
  // chunk's base for the digit (bin start + the segment's earlier chunks)
  // + the chunk's earlier tiles (both loads overlap the ranking below)
  uint32_t off[kPer], pre_t[kPer];
  ld_bins(csum_row<D>(a, S.chunk_off + (ltile >> a.chunk_log2), P), off);
  ld_bins(cnt_row<D>(a, S.tile_off + ltile, P), pre_t);
#pragma unroll
  for (int j = 0; j < kPer; ++j) off[j] += pre_t[j];
  // wide digits: parked in the thread's own words of s_dst until the scan
  // (issued after the arc loads, so the wait costs nothing the ranking
  // would not wait for anyway), which leaves the ranking more registers
  if constexpr (kAlias) st_bins(s_dst, off);
#pragma unroll
  for (int i = 0; i < kWaves * kPer; ++i) s_wh[tid + i * kBlock] = 0;
  __syncthreads();

  // stable rank of each arc among equal digits of its wave: a ballot match
  // finds the lanes sharing the digit (per digit bit one ballot and one
  // three-input bit operation per mask half: mask &= ~(bit ^ ballot)); the
  // lowest of them adds the group size to the wave's bin with a returning
  // LDS atomic (the atomics of the kItems rounds are issued back to back
  // and land in program order, so each returns the count of earlier equal
  // digits); the group then reads the returned base from its leader lane
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint32_t lb[kItems];  // leader lane | (equal digits in lower lanes) << 8
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t li = wave * 64 * kItems + i * 64 + lane;
    const bool valid = li < nv;
    const uint32_t dg = (uint32_t)(el[i] >> (32 + D * P)) & R::kMask;
    const uint64_t vm = __ballot(valid);
    uint32_t lo = (uint32_t)vm, hi = (uint32_t)(vm >> 32);
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (match_stops<D>(P) && b >= nbits) break;  // higher digit bits are zero in every arc
      const uint32_t t = (uint32_t)((int32_t)(dg << (31 - b)) >> 31);  // 0 or ~0
      const uint64_t bb = __ballot(t != 0u);
      lo = __builtin_amdgcn_bitop3_b32(lo, t, (uint32_t)bb, 0x90);
      hi = __builtin_amdgcn_bitop3_b32(hi, t, (uint32_t)(bb >> 32), 0x90);
    }
    const uint64_t mm = ((uint64_t)hi << 32) | lo;
    const uint32_t below = __popcll(mm & lt_mask);
    uint32_t bse = 0;
    if (valid && below == 0) bse = atomicAdd(&s_wh[wave * kBins + dg], (uint32_t)__popcll(mm));
    rk[i] = bse;
    lb[i] = (((uint32_t)__ffsll((long long)mm) - 1u) & 63u) | (below << 8);
  }
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    rk[i] = __shfl(rk[i], (int)(lb[i] & 63u)) + (lb[i] >> 8);
  __syncthreads();

  // per digit (thread = kPer digits): wave offsets, tile counts, tile
  // offsets and the global destination of the tile's first arc of each
  uint32_t cnt[kPer] = {};
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    uint32_t cw[kPer], pre[kPer];
    ld_bins(s_wh + w * kBins, cw);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      pre[j] = cnt[j];
      cnt[j] += cw[j];
    }
    st_bins(s_wh + w * kBins, pre);
  }
  if constexpr (kAlias) ld_bins(s_dst, off);
  uint32_t ctot = 0, tot;
#pragma unroll
  for (int j = 0; j < kPer; ++j) ctot += cnt[j];
  uint32_t loc = block_excl_scan(ctot, s_tmp, &tot);
  uint32_t locs[kPer], dsts[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    locs[j] = loc;
    dsts[j] = off[j] - loc;
    loc += cnt[j];
  }
  st_bins(s_loc, locs);
  st_bins(s_dst, dsts);
  __syncthreads();

  // scatter into LDS in digit order, then write runs out coalesced
  if constexpr (kAlias) {
    // every position is read before the staging buffer is overwritten
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t dg = (uint32_t)(el[i] >> (32 + D * P)) & R::kMask;
      rk[i] += s_loc[dg] + s_wh[wave * kBins + dg];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t li = wave * 64 * kItems + i * 64 + lane;
      if (li < nv) s_el[rk[i]] = el[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t li = wave * 64 * kItems + i * 64 + lane;
      if (li < nv) {
        const uint32_t dg = (uint32_t)(el[i] >> (32 + D * P)) & R::kMask;
        s_el[s_loc[dg] + s_wh[wave * kBins + dg] + rk[i]] = el[i];
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < nv; i += kBlock) {
    const uint64_t e = s_el[i];
    const uint32_t dg = (uint32_t)(e >> (32 + D * P)) & R::kMask;
    dst[s_dst[dg] + i] = e;
  }
}

// The body needs about 140 registers; passes whose build fits in 128
// without spilling run with four waves per SIMD (one more block per CU),
// the others (the first pass reads W and the need bytes and sets up the
// directory mode; the last 8-bit one) with three.
template <int P, int D>
__global__ __launch_bounds__(kBlock) void k_scat(StepArgs a) {
  scat_body<P, D>(a);
}
template <int P, int D>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_scat4(StepArgs a) {
  scat_body<P, D>(a);
}


// ---------------------------------------------------------------------------
// k_step1: Step 1 (Sec. 4.2) draws for every estimator; the replacement
// index goes to j1[] and its batch position is marked as needed
// ---------------------------------------------------------------------------
template <bool kOne>
__device__ void step1_block(const StepArgs& a, uint32_t blk) {
  const uint64_t gid = (uint64_t)blk * kBlock + threadIdx.x;
  uint32_t sidx = 0;
  if constexpr (!kOne) {
    __shared__ uint32_t s_seg;
    __shared__ uint64_t s_next;
    sidx = block_seg_of_est(a, (uint64_t)blk * kBlock, gid, &s_seg, &s_next);
  }
  if (gid >= a.nest) return;
  const SegDesc S = est_seg_desc<kOne>(a, sidx);
  const uint32_t i = (uint32_t)(gid - S.gest_off);
  const uint64_t kb = mix64(mix64(S.key0 ^ (uint64_t)i) ^ S.batch);
  // replace f1 with probability w / (m + w): x uniform on [0, m + w)
  const uint64_t x = bounded(kb, 1, S.m + S.w);
  uint32_t j1 = kNone;
  if (x >= S.m) {
    const uint32_t p = (uint32_t)(x - S.m);
    a.need[S.need_off + p] = 1;  // idempotent byte store: no atomic needed
    const uint2 ed = reinterpret_cast<const uint2*>(S.edges)[p];
    a.r1[S.est_off + i] = canon(ed.x, ed.y);
    j1 = p | (ed.x < ed.y ? 0u : kSideV);
  }
  a.j1[S.est_off + i] = j1;
}

// one launch for two independent jobs: blocks [0, nchunk) fold the k_hist
// counts, the rest run Step 1
template <int D, bool kOne>
__global__ __launch_bounds__(kBlock) void k_fold_step1(StepArgs a) {
  const uint32_t nfold = a.nchunk * (uint32_t)Rdx<D>::kPer;
  if (blockIdx.x < nfold) fold_chunk<D>(a, blockIdx.x);
  else step1_block<kOne>(a, blockIdx.x - nfold);
}

// ---------------------------------------------------------------------------
// vertex directory
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t dir_claim(DirSlot* dir, uint32_t mask,
                                              uint32_t x, uint32_t tag,
                                              uint32_t* err) {
  const uint64_t want = ((uint64_t)tag << 32) | x;
  uint32_t h = mix32(x) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    unsigned long long* kt = reinterpret_cast<unsigned long long*>(&dir[h]);
    const uint64_t cur = __hip_atomic_load(kt, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    if (cur == want) return h;
    if ((uint32_t)(cur >> 32) != tag) {
      const uint64_t old = atomicCAS(kt, (unsigned long long)cur,
                                     (unsigned long long)want);
      if (old == cur || old == want) return h;
      // otherwise another key took the slot this step: move on
    }
    h = (h + 1) & mask;
  }
  atomicOr(err, kErrProbe);
  return kNone;
}

// [start, end) of x's arcs, or an empty range.  Dense directory: two
// words of the CSR offsets (one line unless x + 1 starts the next), both
// loads issued before either is used; ids above the largest are absent.
__device__ __forceinline__ uint2 dir_find_dense(const uint32_t* off, uint32_t maxid,
                                                uint32_t x) {
  const uint32_t xc = min(x, maxid);
  const uint32_t s = off[xc], e = off[xc + 1];
  const bool ok = x <= maxid;
  return make_uint2(ok ? s : 0u, ok ? e : 0u);
}

// hashed directory: linear probing from x's hash to its key or a slot that
// is not live this step
__device__ __forceinline__ uint2 dir_find_hashed(const DirSlot* dir, uint32_t mask,
                                                 uint32_t x, uint32_t tag) {
  uint32_t h = mix32(x) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const uint4 e = *reinterpret_cast<const uint4*>(&dir[h]);
    if (e.y != tag) break;
    if (e.x == x) return make_uint2(e.z, e.w);
    h = (h + 1) & mask;
  }
  return make_uint2(0, 0);
}

// Vertex ids per window of the dense offsets that k_dir fills at a time.
constexpr uint32_t kDirWin = 16u * kBlock;
static_assert(kTile < 0xFFFFu, "tile indices and the empty mark fit 16 bits");

// suffix minimum over a kBlock block of one value per thread: the minimum
// of the values of the threads above this one (0xFFFF when there is none)
__device__ __forceinline__ uint32_t block_excl_suffix_min(uint32_t v, uint32_t* s_tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_down(x, d);
    if (lane + d < 64) x = min(x, y);
  }
  if (lane == 0) s_tmp[wave] = x;
  uint32_t above = __shfl_down(x, 1);
  if (lane == 63) above = 0xFFFFu;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kWaves; ++k)
    if (k > wave) above = min(above, s_tmp[k]);
  return above;
}

// The block's tile of sorted arcs keeps its arcs in registers and their
// vertices (plus the arc on each side) in LDS.  Dense directory: the tile
// writes the CSR offsets of the vertex ids from one past the arc before the
// tile to its last arc's (to max id + 1 for the last tile), so every id up
// to max id + 1 is written by exactly one tile.  Offset y is the tile's
// first arc of a vertex >= y: a suffix minimum, over the window of ids, of
// the marks that each vertex's first arc in the tile leaves at its id; the
// windows go from the top down, each written out in consecutive words.
__global__ __launch_bounds__(kBlock) void k_dir(StepArgs a) {
  __shared__ uint32_t s_vtx[kTile + 2];  // s_vtx[1 + t] = vertex of arc base + t
  __shared__ __align__(16) uint16_t s_win[kDirWin];
  __shared__ uint32_t s_tmp[kWaves];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x;
  const uint32_t gtile = blockIdx.x;
  if (tid == 0) s_seg = seg_of_tile(a, gtile);
  __syncthreads();
  if (*a.err & kErrFatal) return;
  const uint32_t sidx = uniform(s_seg);
  const SegDesc S = seg_desc(a, sidx);
  const SegWork* wk = a.work + sidx;
  // (a select, not an index into the argument array: see k_est)
  const uint64_t* arc = (wk->final_buf ? a.arcs[1] : a.arcs[0]) + S.arc_off;
  const uint32_t n = 2u * S.w;
  const uint32_t base = (gtile - S.tile_off) * kTile;
  const uint32_t nv = min((uint32_t)kTile, n - base);
  // clamped loads past the ragged end are never used as arcs
  uint64_t v[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) v[k] = arc[min(base + k * kBlock + tid, n - 1)];
  if (tid == 0) s_vtx[0] = (uint32_t)(arc[base > 0 ? base - 1 : 0] >> 32);
  if (tid == 1) s_vtx[kTile + 1] = (uint32_t)(arc[min(base + kTile, n - 1)] >> 32);
#pragma unroll
  for (int k = 0; k < kItems; ++k) s_vtx[1 + k * kBlock + tid] = (uint32_t)(v[k] >> 32);
  __syncthreads();
  const bool dense = wk->dense != 0;
  uint32_t* inv = a.inv + S.arc_off;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t t = k * kBlock + tid;
    const uint32_t id = (uint32_t)v[k];
    if (t < nv && (id & kNeedFlag)) inv[id & kIdMask] = base + t;
  }
  if (dense) {
    uint32_t* off = a.doff + S.doff_off;
    const uint64_t lo = base == 0 ? 0u : (uint64_t)s_vtx[0] + 1u;
    const uint64_t hi = base + nv == n ? (uint64_t)uniform(wk->maxid) + 1u
                                       : (uint64_t)s_vtx[nv];
    if (lo > hi) return;  // the whole tile continues the vertex before it
    uint32_t carry = nv;  // first arc at or above the current window's end
    for (uint64_t win = (hi - lo) / kDirWin + 1; win-- > 0;) {
      const uint64_t y0 = lo + win * kDirWin;
      const uint32_t len = hi - y0 + 1 < kDirWin ? (uint32_t)(hi - y0 + 1) : kDirWin;
      uint4* w4 = reinterpret_cast<uint4*>(s_win);
      w4[2 * tid] = make_uint4(~0u, ~0u, ~0u, ~0u);
      w4[2 * tid + 1] = make_uint4(~0u, ~0u, ~0u, ~0u);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const uint32_t t = k * kBlock + tid;
        const uint32_t x = s_vtx[1 + t];
        const bool head = t == 0 || s_vtx[t] != x;
        if (t < nv && head && x >= y0 && x - y0 < len) s_win[x - y0] = (uint16_t)t;
      }
      __syncthreads();
      // the thread's 16 consecutive marks, their suffix minima in place
      const uint4 q0 = w4[2 * tid], q1 = w4[2 * tid + 1];
      uint32_t m[16] = {q0.x & 0xFFFFu, q0.x >> 16, q0.y & 0xFFFFu, q0.y >> 16,
                        q0.z & 0xFFFFu, q0.z >> 16, q0.w & 0xFFFFu, q0.w >> 16,
                        q1.x & 0xFFFFu, q1.x >> 16, q1.y & 0xFFFFu, q1.y >> 16,
                        q1.z & 0xFFFFu, q1.z >> 16, q1.w & 0xFFFFu, q1.w >> 16};
#pragma unroll
      for (int j = 14; j >= 0; --j) m[j] = min(m[j], m[j + 1]);
      const uint32_t above = min(block_excl_suffix_min(m[0], s_tmp), carry);
#pragma unroll
      for (int j = 0; j < 16; ++j) m[j] = min(m[j], above);
      __syncthreads();  // every thread has read its marks
      w4[2 * tid] = make_uint4(m[0] | m[1] << 16, m[2] | m[3] << 16, m[4] | m[5] << 16,
                               m[6] | m[7] << 16);
      w4[2 * tid + 1] = make_uint4(m[8] | m[9] << 16, m[10] | m[11] << 16,
                                   m[12] | m[13] << 16, m[14] | m[15] << 16);
      __syncthreads();
      for (uint32_t k = tid; k < len; k += kBlock) off[y0 + k] = base + s_win[k];
      carry = s_win[0];
      __syncthreads();  // before the next window overwrites the marks
    }
    return;
  }
  DirSlot* dir = a.dir + S.dir_off;
  const uint32_t mask = (1u << S.dir_log2) - 1u;
  const uint32_t tag = uniform(*a.tagp);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t t = k * kBlock + tid;
    if (t >= nv) continue;
    const uint32_t i = base + t;
    const uint32_t x = s_vtx[1 + t];
    const bool head = i == 0 || s_vtx[t] != x;
    const bool tail = i + 1 == n || s_vtx[t + 2] != x;
    if (!head && !tail) continue;
    const uint32_t slot = dir_claim(dir, mask, x, tag, a.err);
    if (slot == kNone) continue;
    if (head) dir[slot].start = i;
    if (tail) dir[slot].end = i + 1;
  }
}

// ---------------------------------------------------------------------------
// k_est: Steps 1 and 2 per estimator, Step-3 query posted
// ---------------------------------------------------------------------------
template <bool kOne>
__global__ __launch_bounds__(kBlock) void k_est(StepArgs a) {
  const uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t sidx = 0;
  if constexpr (!kOne) {
    __shared__ uint32_t s_seg;
    __shared__ uint64_t s_next;
    sidx = block_seg_of_est(a, (uint64_t)blockIdx.x * kBlock, gid, &s_seg, &s_next);
  }
  if (gid >= a.nest) return;
  if (*a.err & kErrFatal) return;
  const SegDesc S = est_seg_desc<kOne>(a, sidx);
  const SegWork* wk = a.work + sidx;
  const uint32_t i = (uint32_t)(gid - S.gest_off);  // index within the bank
  const uint64_t e = S.est_off + i;
  const uint2* W = reinterpret_cast<const uint2*>(S.edges);

  // every load that does not depend on another is issued here: the
  // estimator's state and the segment's words (its sorted-arc buffer, the
  // directory mode, the step's tag)
  const uint64_t r1 = a.r1[e];  // Step 1 (k_step1) already wrote a new f1
  uint64_t r2 = a.r2[e];
  const uint32_t ccw = a.cc[e];
  const uint32_t jw = a.j1[e];
  const uint32_t fbuf = wk->final_buf;
  const bool dense = wk->dense != 0;
  const uint32_t maxid = wk->maxid;
  const uint32_t tag = *a.tagp;
  uint64_t c = ccw & kChiMax;
  bool closed = (ccw & kClosed) != 0;
  const uint64_t kb = mix64(mix64(S.key0 ^ (uint64_t)i) ^ S.batch);

  // Step 1 (Sec. 4.2): a new f1 = W[j1] starts with chi = 0 and no f2
  const uint32_t j1 = jw == kNone ? kNone : (jw & kPosMask);
  const uint32_t side_u = (jw != kNone && (jw & kSideV)) ? 1u : 0u;
  if (j1 != kNone) {
    c = 0;
    r2 = kEmpty;
    closed = false;
  }

  // Step 2 (Sec. 4.3): chi+ = rank(u->v) + rank(v->u) with u < v.  The
  // inverse-index pair of W[j1] is loaded together with the two directory
  // slots (an unused, always valid pair when there is no new f1)
  const uint32_t u = (uint32_t)(r1 >> 32), v = (uint32_t)r1;
  const uint2 iv2 = *reinterpret_cast<const uint2*>(
      a.inv + S.arc_off + 2ull * (j1 == kNone ? 0u : j1));
  uint2 su, sv;
  if (dense) {
    const uint32_t* off = a.doff + S.doff_off;
    su = dir_find_dense(off, maxid, u);
    sv = dir_find_dense(off, maxid, v);
  } else {
    const DirSlot* dir = a.dir + S.dir_off;
    const uint32_t dmask = (1u << S.dir_log2) - 1u;
    su = dir_find_hashed(dir, dmask, u, tag);
    sv = dir_find_hashed(dir, dmask, v, tag);
  }
  // (a select of the two buffer pointers: indexing the argument array by
  // a value read at run time would load the pointer from memory)
  const uint64_t* arc = (fbuf ? a.arcs[1] : a.arcs[0]) + S.arc_off;
  uint32_t ld, rd;
  if (j1 != kNone) {
    // f1 is W[j1]: the arcs after it on each endpoint are those after its
    // own arcs in their segments (the guard only keeps every later index
    // inside the segment)
    const uint32_t iu = side_u ? iv2.y : iv2.x;
    const uint32_t iv = side_u ? iv2.x : iv2.y;
    const bool ok = iu >= su.x && iu < su.y && iv >= sv.x && iv < sv.y;
    if (!ok) atomicOr(a.err, kErrIndex);
    ld = ok ? su.y - 1 - iu : 0u;
    rd = ok ? sv.y - 1 - iv : 0u;
  } else {
    ld = su.y - su.x;
    rd = sv.y - sv.x;
  }
  const uint64_t cplus = (uint64_t)ld + rd;
  uint32_t p2 = kNone;
  if (cplus != 0) {
    const uint64_t tot = c + cplus;
    const uint64_t y = bounded(kb, 2, tot);
    if (y >= c) {
      // phi names the (phi)-th candidate: rank phi on u, else phi-ld on v;
      // rank k on a vertex is the arc with k later arcs of that vertex
      const uint64_t phi = y - c;
      const uint32_t idx = phi < ld ? su.y - 1 - (uint32_t)phi
                                    : sv.y - 1 - (uint32_t)(phi - ld);
      p2 = ((uint32_t)arc[idx] & kIdMask) >> 1;  // arc id -> batch position
      if (p2 >= S.w) {  // cannot happen: arcs carry positions < w
        atomicOr(a.err, kErrIndex);
        p2 = 0;
      }
      const uint2 ed = W[p2];
      r2 = canon(ed.x, ed.y);
      closed = false;
    }
    if (tot > kChiMax) {
      atomicOr(a.err, kErrOverflow);
      c = kChiMax;
    } else {
      c = tot;
    }
  }

  // Step 3 (Sec. 4.4): the closing edge this estimator waits for in W
  uint64_t q = kEmpty;
  if (r2 != kEmpty && !closed) q = closing(r1, r2);
  a.qq[e] = q;
  a.qthr[e] = (p2 == kNone) ? 0u : p2 + 1;  // closes at a position >= this
  a.r2[e] = r2;
  a.cc[e] = (uint32_t)c | (closed ? kClosed : 0u);
}

// ---------------------------------------------------------------------------
// Step 3 (Sec. 4.4): which waiting estimators' closing edges occur in W at
// or after their position limit.  A hash join: the batch edges and the
// waiting estimators are grouped by partition of their (closing) edge's
// hash, then each partition's estimators go into an LDS hash table that the
// partition's edges are streamed through.  Closed flags are an OR over the
// matches, so the order of records inside a partition does not matter.
// ---------------------------------------------------------------------------

// segment of block b of a launch whose segments' blocks start at `off`
template <uint32_t SegDesc::*Off>
__device__ __forceinline__ uint32_t seg_of_block(const StepArgs& a, uint32_t b) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].*Off <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t part_of(uint64_t h, uint32_t pbits) {
  return pbits ? (uint32_t)(h >> (64u - pbits)) : 0u;
}

// The partition kernels run 1024-thread blocks (sixteen waves) over tiles
// of kPTile elements: enough waves per CU to keep their loads in flight.
constexpr int kPThreads = 1024;
constexpr int kPWaves = kPThreads / 64;

// exclusive scan of one value per thread over a kPThreads block
__device__ __forceinline__ uint32_t pblock_excl_scan(uint32_t v, uint32_t* s_tmp,
                                                     uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kPWaves; ++w) {
    const uint32_t t = s_tmp[w];
    off += (w < wave) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Global (not generic) view of a pointer: its loads are global loads, so
// waiting for them never waits for LDS traffic, nor LDS waits for them.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Up to 2^ptile_log2 elements of one side of a partition tile: edges of W
// (side 0) or estimators (side 1, waiting ones only).  f(h, id, valid) is
// called by every thread for each of its elements, in rounds of kPRound
// loads issued together; h = mix64 of the (closing) edge, id its batch
// position or state index.  Every lane of a wave makes the same calls.
constexpr uint32_t kPRound = 8;

template <class F>
__device__ __forceinline__ void for_tile(const StepArgs& a, const SegDesc& S, uint32_t t,
                                         F&& f) {
  const int tid = threadIdx.x;
  if (t < S.netile) {
    const uint2* W = reinterpret_cast<const uint2*>(S.edges);
    const uint32_t j0 = t << S.ptile_log2, j1 = min(j0 + (1u << S.ptile_log2), S.w);
    for (uint32_t b = j0; b < j1; b += kPRound * kPThreads) {
      uint2 ed[kPRound];
#pragma unroll
      for (uint32_t k = 0; k < kPRound; ++k)
        ed[k] = W[min(b + k * kPThreads + tid, j1 - 1)];
#pragma unroll
      for (uint32_t k = 0; k < kPRound; ++k) {
        const uint32_t j = b + k * kPThreads + tid;
        f(mix64(canon(ed[k].x, ed[k].y)), j, j < j1);
      }
    }
  } else {
    const uint32_t i0 = (t - S.netile) << S.ptile_log2;
    const uint32_t i1 = min(i0 + (1u << S.ptile_log2), S.r);
    const uint64_t* qq = a.qq + S.est_off;
    for (uint32_t b = i0; b < i1; b += kPRound * kPThreads) {
      uint64_t q[kPRound];
#pragma unroll
      for (uint32_t k = 0; k < kPRound; ++k) q[k] = qq[min(b + k * kPThreads + tid, i1 - 1)];
#pragma unroll
      for (uint32_t k = 0; k < kPRound; ++k) {
        const uint32_t i = b + k * kPThreads + tid;
        f(mix64(q[k]), (uint32_t)S.est_off + i, i < i1 && q[k] != kEmpty);
      }
    }
  }
}

// Lanes of the wave whose partitions are equal (nbits low bits compared):
// one ballot and one three-input bit operation per bit and mask half.
__device__ __forceinline__ uint64_t match_lanes(uint32_t p, bool valid, uint32_t nbits) {
  const uint64_t vm = __ballot(valid);
  uint32_t lo = (uint32_t)vm, hi = (uint32_t)(vm >> 32);
  for (uint32_t b = 0; b < nbits; ++b) {
    const uint32_t t = (uint32_t)((int32_t)(p << (31 - b)) >> 31);
    const uint64_t bb = __ballot(t != 0u);
    lo = __builtin_amdgcn_bitop3_b32(lo, t, (uint32_t)bb, 0x90);
    hi = __builtin_amdgcn_bitop3_b32(hi, t, (uint32_t)(bb >> 32), 0x90);
  }
  return ((uint64_t)hi << 32) | lo;
}

// With few partitions (pbits <= kAggBits) a wave's equal partitions are
// counted or ranked once per group (one LDS atomic per distinct partition);
// with more, one LDS atomic per element (they rarely collide).
constexpr uint32_t kAggBits = 4;

// Tiles of one segment and side land on the XCDs in runs of eight (as in the
// radix passes): neighbouring tiles' runs of a partition then mostly meet in
// one L2 before they are written back.
__device__ __forceinline__ uint32_t ptile_block(uint32_t b) {
  return xcd_block(b, gridDim.x);
}

// k_pcnt: per partition tile, the count of its elements in each partition
__global__ __launch_bounds__(kPThreads) void k_pcnt(StepArgs a) {
  __shared__ uint32_t s_h[1u << kMaxPartLog2];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t blk = ptile_block(blockIdx.x);
  if (tid == 0) s_seg = seg_of_block<&SegDesc::ptile_off>(a, blk);
  for (uint32_t p = tid; p < (1u << kMaxPartLog2); p += kPThreads) s_h[p] = 0;
  __syncthreads();
  if (*a.err & kErrFatal) return;
  const SegDesc S = seg_desc(a, uniform(s_seg));
  const uint32_t P = 1u << S.pbits, t = blk - S.ptile_off;
  const bool agg = S.pbits <= kAggBits;
  for_tile(a, S, t, [&](uint64_t h, uint32_t, bool valid) {
    const uint32_t p = part_of(h, S.pbits);
    if (agg) {
      const uint64_t mm = match_lanes(p, valid, S.pbits);
      if (valid && __popcll(mm & ((1ull << lane) - 1ull)) == 0)
        atomicAdd(&s_h[p], (uint32_t)__popcll(mm));
    } else if (valid) {
      atomicAdd(&s_h[p], 1u);
    }
  });
  __syncthreads();
  uint32_t* row = a.prow + S.prow_off + (uint64_t)t * P;
  for (uint32_t p = tid; p < P; p += kPThreads) row[p] = s_h[p];
}

// k_pscan: per (segment, side, 64 partitions), each partition's count rows
// over the side's tiles become exclusive prefixes, and its total is kept.
// Wave w of the sixteen takes the w-th sixteenth of the tiles, loaded in
// batches.
constexpr uint32_t kPScanBatch = 16;

__global__ __launch_bounds__(kPThreads) void k_pscan(StepArgs a) {
  __shared__ uint32_t s_part[kPWaves][64];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_seg = seg_of_block<&SegDesc::pscan_off>(a, blockIdx.x);
  __syncthreads();
  if (*a.err & kErrFatal) return;
  const SegDesc S = seg_desc(a, uniform(s_seg));
  const uint32_t P = 1u << S.pbits, ngroups = (P + 63) / 64;
  const uint32_t b = blockIdx.x - S.pscan_off, side = b / ngroups;
  const uint32_t p = (b % ngroups) * 64 + lane;
  const bool valid = p < P;
  const uint32_t t0 = side ? S.netile : 0u, nt = side ? S.nqtile : S.netile;
  const uint32_t per = (nt + kPWaves - 1) / kPWaves;
  const uint32_t lo = min((uint32_t)wave * per, nt), hi = min(lo + per, nt);
  uint32_t* col = a.prow + S.prow_off + (uint64_t)t0 * P + (valid ? p : 0u);
  uint32_t sum = 0;
  for (uint32_t c = lo; c < hi; c += kPScanBatch) {
    uint32_t v[kPScanBatch];
#pragma unroll
    for (uint32_t i = 0; i < kPScanBatch; ++i)
      v[i] = valid && c + i < hi ? col[(uint64_t)(c + i) * P] : 0u;
#pragma unroll
    for (uint32_t i = 0; i < kPScanBatch; ++i) sum += v[i];
  }
  s_part[wave][lane] = sum;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kPWaves; ++k) {
    run += k < wave ? s_part[k][lane] : 0u;
    total += s_part[k][lane];
  }
  for (uint32_t c = lo; c < hi; c += kPScanBatch) {
    uint32_t v[kPScanBatch];
#pragma unroll
    for (uint32_t i = 0; i < kPScanBatch; ++i)
      v[i] = valid && c + i < hi ? col[(uint64_t)(c + i) * P] : 0u;
#pragma unroll
    for (uint32_t i = 0; i < kPScanBatch; ++i) {
      if (valid && c + i < hi) col[(uint64_t)(c + i) * P] = run;
      run += v[i];
    }
  }
  if (wave == 0 && valid) a.ptot[2ull * (S.part_off + p) + side] = total;
}

// A record: the top 32 bits of h (the partition in their top pbits bits,
// the LDS table index and fingerprint below) over the element's id.
__device__ __forceinline__ uint64_t part_rec(uint64_t h, uint32_t id) {
  return (h & 0xFFFFFFFF00000000ull) | id;
}

// k_pscat: per partition tile, the records of its elements in partition
// order.  Each element takes a place among its partition's records of the
// tile (an LDS atomic: the order inside a partition does not matter) in a
// tile-sized LDS staging array laid out by partition; the staged records
// then go out in order, consecutive lanes writing consecutive records, to
// the partition's start (a scan of the side's totals) plus the tile's
// prefix.  The first tile of each side also stores the starts for the join.
__global__ __launch_bounds__(kPThreads) void k_pscat(StepArgs a) {
  constexpr uint32_t kPer = (1u << kMaxPartLog2) / kPThreads;  // partitions per thread
  __shared__ uint64_t s_el[kPTile];
  __shared__ uint32_t s_base[1u << kMaxPartLog2];  // global slot of the tile's first
  __shared__ uint32_t s_loc[(1u << kMaxPartLog2) + 1];  // staging offsets, then cursors
  __shared__ uint32_t s_tmp[kPWaves];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t blk = ptile_block(blockIdx.x);
  if (tid == 0) s_seg = seg_of_block<&SegDesc::ptile_off>(a, blk);
  __syncthreads();
  if (*a.err & kErrFatal) return;
  const SegDesc S = seg_desc(a, uniform(s_seg));
  const uint32_t P = 1u << S.pbits, t = blk - S.ptile_off;
  const uint32_t side = t < S.netile ? 0u : 1u;
  const bool first = t == 0 || t == S.netile;
  const bool last = t + 1 == S.netile || t + 1 == S.netile + S.nqtile;
  // thread tid holds partitions [kPer tid, kPer tid + kPer): their starts
  // (scan of the totals), the tile's prefix and its own count (the next
  // tile's prefix, or the total, minus this one's)
  const uint32_t* tot = a.ptot + 2ull * S.part_off + side;
  const uint32_t* row = a.prow + S.prow_off + (uint64_t)t * P;
  uint32_t v[kPer], pre[kPer], cnt[kPer], sum = 0, csum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t p = kPer * tid + k;
    v[k] = p < P ? tot[2ull * p] : 0u;
    pre[k] = p < P ? row[p] : 0u;
    const uint32_t nxt = p < P ? (last ? v[k] : row[P + p]) : 0u;
    cnt[k] = nxt - pre[k];
    sum += v[k];
    csum += cnt[k];
  }
  uint32_t all, n;
  uint32_t run = pblock_excl_scan(sum, s_tmp, &all);
  uint32_t loc = pblock_excl_scan(csum, s_tmp, &n);
  uint32_t* st = a.pstart + 2ull * S.part_off + side;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t p = kPer * tid + k;
    if (p < P) {
      if (first) st[2ull * p] = run;
      s_base[p] = run + pre[k];
      s_loc[p] = loc;
    }
    run += v[k];
    loc += cnt[k];
  }
  if (tid == 0) s_loc[P] = n;
  __syncthreads();
  // staging offsets of the partitions, kept for the write-out below
  uint32_t lo[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) lo[k] = kPer * tid + k < P ? s_loc[kPer * tid + k] : 0u;
  const bool agg = S.pbits <= kAggBits;
  for_tile(a, S, t, [&](uint64_t h, uint32_t id, bool valid) {
    const uint32_t p = part_of(h, S.pbits);
    uint32_t slot;
    if (agg) {
      const uint64_t mm = match_lanes(p, valid, S.pbits);
      const uint32_t below = __popcll(mm & ((1ull << lane) - 1ull));
      uint32_t bse = 0;
      if (valid && below == 0) bse = atomicAdd(&s_loc[p], (uint32_t)__popcll(mm));
      slot = __shfl(bse, (int)(((uint32_t)__ffsll((long long)mm) - 1u) & 63u)) + below;
    } else {
      slot = valid ? atomicAdd(&s_loc[p], 1u) : 0u;
    }
    if (valid) s_el[slot] = part_rec(h, id);
  });
  __syncthreads();
  // the cursors ran to the next partition's offset: restore the offsets
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k)
    if (kPer * tid + k < P) s_loc[kPer * tid + k] = lo[k];
  __syncthreads();
  uint64_t* out = side ? a.qrec + S.gest_off : a.erec + S.arc_off / 2;
  for (uint32_t i = tid; i < n; i += kPThreads) {
    const uint64_t rec = s_el[i];
    const uint32_t p = part_of(rec, S.pbits);
    out[s_base[p] + (i - s_loc[p])] = rec;
  }
}

// k_pjoin: block (p, slice): the waiting estimators of partition p (in
// rounds of kJoinQ) in an LDS open-addressing table of their records,
// indexed by the low bits of the record's high word, and the slice's edges
// probed against it, kJoinRound loads in flight per thread.  A record whose
// high word equals the edge's closes its estimator iff the edge is the
// estimator's closing edge and comes at or after its limit.  Most edges
// match no record: a bitmap of the records' keys (one LDS read) turns them
// away before the table, whose probe chains (the wave runs as long as its
// longest) are the join's critical path.  Also resets the per-segment work
// area (the step's last kernel).
constexpr int kJoinThreads = 512;
constexpr uint32_t kJoinRound = 8;
constexpr uint32_t kQPer = kJoinQ / kJoinThreads;  // records per thread and round
static_assert(kQPer * kJoinThreads == kJoinQ, "a round's records are whole loads");
constexpr uint64_t kFreeRec = ~0ull;  // no record: ids stay below 2^31
constexpr uint32_t kJoinBitsLog2 = 16;  // key bitmap bits (8 KB)

__device__ __forceinline__ uint32_t join_bit(uint32_t f) {
  return f & ((1u << kJoinBitsLog2) - 1u);
}

__global__ __launch_bounds__(kJoinThreads) void k_pjoin(StepArgs a) {
  __shared__ uint64_t s_tab[kJoinSlots];
  __shared__ uint32_t s_bits[(1u << kJoinBitsLog2) / 32];
  __shared__ uint32_t s_seg;
  const int tid = threadIdx.x;
  if (tid == 0) s_seg = seg_of_block<&SegDesc::jblk_off>(a, blockIdx.x);
  __syncthreads();
  const SegDesc S = seg_desc(a, uniform(s_seg));
  if ((*a.err & kErrFatal) == 0) {
    const uint32_t b = blockIdx.x - S.jblk_off, p = b / S.jslices, sl = b % S.jslices;
    const uint64_t g2 = 2ull * (S.part_off + p);
    const uint32_t qs = a.pstart[g2 + 1], qc = a.ptot[g2 + 1];
    const uint32_t es = a.pstart[g2], ec = a.ptot[g2];
    const uint32_t e_lo = es + (uint32_t)((uint64_t)ec * sl / S.jslices);
    const uint32_t e_hi = es + (uint32_t)((uint64_t)ec * (sl + 1) / S.jslices);
    const auto* qrec = as_global(a.qrec + S.gest_off);
    const auto* erec = as_global(a.erec + S.arc_off / 2);
    const auto* W = as_global(reinterpret_cast<const uint64_t*>(S.edges));
    constexpr uint32_t kStride = kJoinRound * kJoinThreads;
    for (uint32_t r0 = 0; e_hi > e_lo && r0 < qc; r0 += kJoinQ) {
      const uint32_t nq = min(kJoinQ, qc - r0);
      // the round's records and the slice's first edges are loaded before
      // the table is cleared, so their latency overlaps the clear
      uint64_t rec[kQPer], er[kJoinRound];
#pragma unroll
      for (uint32_t k = 0; k < kQPer; ++k)
        rec[k] = qrec[qs + r0 + min(k * kJoinThreads + tid, nq - 1)];
#pragma unroll
      for (uint32_t k = 0; k < kJoinRound; ++k)
        er[k] = erec[min(e_lo + k * kJoinThreads + tid, e_hi - 1)];
      // a table of four times the round's records (load <= 1/4; at most
      // kJoinSlots, so a full round of kJoinQ loads it to 1/2)
      const uint32_t cl = nq > 1 ? 32u - (uint32_t)__clz(nq - 1) : 0u;
      const uint32_t mask = min(kJoinSlots, max(512u, 4u << cl)) - 1u;
      for (uint32_t i = tid; i <= mask; i += kJoinThreads) s_tab[i] = kFreeRec;
      for (uint32_t i = tid; i < (1u << kJoinBitsLog2) / 32; i += kJoinThreads) s_bits[i] = 0;
      __syncthreads();
#pragma unroll
      for (uint32_t k = 0; k < kQPer; ++k) {
        if (k * kJoinThreads + tid >= nq) continue;
        const uint32_t f = (uint32_t)(rec[k] >> 32);
        atomicOr(&s_bits[join_bit(f) >> 5], 1u << (join_bit(f) & 31u));
        uint32_t slot = f & mask;
        while (atomicCAS(reinterpret_cast<unsigned long long*>(&s_tab[slot]),
                         (unsigned long long)kFreeRec,
                         (unsigned long long)rec[k]) != kFreeRec)
          slot = (slot + 1) & mask;
      }
      __syncthreads();
      for (uint32_t j0 = e_lo; j0 < e_hi; j0 += kStride) {
        // the next edges are in flight while these probe the table
        const uint32_t j1 = j0 + kStride;
        uint64_t nx[kJoinRound];
        if (j1 < e_hi) {
#pragma unroll
          for (uint32_t k = 0; k < kJoinRound; ++k)
            nx[k] = erec[min(j1 + k * kJoinThreads + tid, e_hi - 1)];
        }
        // the filter for all of the thread's edges at once, then the table
        // for those that pass
        uint32_t pass = 0;
#pragma unroll
        for (uint32_t k = 0; k < kJoinRound; ++k) {
          const uint32_t f = (uint32_t)(er[k] >> 32);
          const bool in = j0 + k * kJoinThreads + tid < e_hi;
          pass |= (in && (s_bits[join_bit(f) >> 5] >> (join_bit(f) & 31u)) & 1u) ? 1u << k : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kJoinRound; ++k) {
          if (!(pass >> k & 1u)) continue;
          const uint32_t f = (uint32_t)(er[k] >> 32), pos = (uint32_t)er[k];
          for (uint32_t slot = f & mask;; slot = (slot + 1) & mask) {
            const uint64_t qr = s_tab[slot];
            if (qr == kFreeRec) break;
            if ((uint32_t)(qr >> 32) != f) continue;
            const uint32_t e = (uint32_t)qr;
            const uint64_t ed = W[pos];
            if (canon((uint32_t)ed, (uint32_t)(ed >> 32)) == a.qq[e] && pos >= a.qthr[e])
              atomicOr(&a.cc[e], kClosed);
          }
        }
        if (j1 < e_hi) {
#pragma unroll
          for (uint32_t k = 0; k < kJoinRound; ++k) er[k] = nx[k];
        }
      }
      __syncthreads();
    }
  }
  // this step no longer needs the per-segment work area: reset it
  const uint32_t words = a.nseg * (uint32_t)(sizeof(SegWork) / 4);
  uint32_t* wz = reinterpret_cast<uint32_t*>(a.work);
  for (uint32_t t = blockIdx.x * kJoinThreads + tid; t < words; t += a.njblk * kJoinThreads)
    wz[t] = 0;
}

// ---------------------------------------------------------------------------
// k_naive: the per-estimator form the bulk algorithm improves on (Sec. 4):
// every estimator reads the whole batch itself, O(r w) work.  It makes the
// same random draws and state transitions as the bulk step, written from
// the definitions: Step 1 takes W[x - |E|] when x = U(|E|+|W|) >= |E|;
// Step 2 counts the batch edges on each endpoint of f1 after f1's position
// (ld, rd), keeps f2 when y = U(chi + ld + rd) < chi and otherwise takes the
// edge with phi = y - chi later edges on u (phi < ld) or phi - ld later
// edges on v; Step 3 closes when the closing edge occurs in W after f2's
// position (anywhere, for an f2 from an earlier batch).
// ---------------------------------------------------------------------------
// The batch is read in tiles of kNaiveTile edges staged in LDS and shared by
// the block (every estimator reads every edge: broadcast LDS reads); the
// three scans (later edges on f1's endpoints, the phi-th edge, the closing
// edge's latest position) each sweep the tiles, forward or backward.
constexpr uint32_t kNaiveTile = 2048;

__global__ __launch_bounds__(kBlock) void k_naive(NaiveArgs a) {
  __shared__ uint2 s_w[kNaiveTile];
  __shared__ uint32_t s_err;
  const uint2* W = reinterpret_cast<const uint2*>(a.edges);
  const int tid = threadIdx.x;
  if (blockIdx.x == 0) {  // a self-loop invalidates the batch
    bool loop = false;
    for (uint32_t j = tid; j < a.w; j += kBlock) {
      const uint2 ed = W[j];
      loop |= ed.x == ed.y;
    }
    if (loop) atomicOr(a.err, kErrSelfLoop);
  }
  if (tid == 0) s_err = *a.err;  // one read, so the exit is block-uniform
  __syncthreads();
  if (s_err & kErrFatal) return;
  const uint32_t i = blockIdx.x * kBlock + tid;
  const bool live = i < a.r;  // threads past r still help load the tiles
  const uint64_t e = a.est_off + (live ? i : 0u);
  uint64_t r1 = kEmpty, r2 = kEmpty, c = 0;
  bool closed = false;
  uint64_t kb = 0;
  uint32_t j1 = kNone;
  if (live) {
    r1 = a.r1[e];
    r2 = a.r2[e];
    const uint32_t ccw = a.cc[e];
    c = ccw & kChiMax;
    closed = (ccw & kClosed) != 0;
    kb = mix64(mix64(a.key0 ^ (uint64_t)i) ^ a.batch);
    // Step 1
    const uint64_t x = bounded(kb, 1, a.m + a.w);
    if (x >= a.m) {
      j1 = (uint32_t)(x - a.m);
      const uint2 ed = W[j1];
      r1 = canon(ed.x, ed.y);
      c = 0;
      r2 = kEmpty;
      closed = false;
    }
  }
  const uint32_t ntile = (a.w + kNaiveTile - 1) / kNaiveTile;
  auto load_tile = [&](uint32_t t) {
    __syncthreads();
    const uint32_t j0 = t * kNaiveTile, n = min(kNaiveTile, a.w - j0);
    for (uint32_t k = tid; k < n; k += kBlock) s_w[k] = W[j0 + k];
    __syncthreads();
  };

  // Step 2: ld, rd = edges on u, v after f1's position (all of W for an
  // f1 from an earlier batch)
  const uint32_t u = (uint32_t)(r1 >> 32), v = (uint32_t)r1;
  uint32_t ld = 0, rd = 0;
  const uint32_t jstart = j1 == kNone ? 0u : j1 + 1;
  for (uint32_t t = 0; t < ntile; ++t) {
    load_tile(t);
    const uint32_t j0 = t * kNaiveTile, n = min(kNaiveTile, a.w - j0);
    if (!live || jstart >= j0 + n) continue;
    uint32_t k = jstart > j0 ? jstart - j0 : 0u;
    for (; k + 8 <= n; k += 8) {  // eight independent LDS reads per round
      uint2 ed[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) ed[q] = s_w[k + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ld += (ed[q].x == u || ed[q].y == u) ? 1u : 0u;
        rd += (ed[q].x == v || ed[q].y == v) ? 1u : 0u;
      }
    }
    for (; k < n; ++k) {
      const uint2 ed = s_w[k];
      ld += (ed.x == u || ed.y == u) ? 1u : 0u;
      rd += (ed.x == v || ed.y == v) ? 1u : 0u;
    }
  }
  const uint64_t cplus = (uint64_t)ld + rd;
  uint32_t p2 = kNone;
  bool pick = false;  // a new f2 is taken: find the edge with k later
  uint32_t src = 0, kk = 0;  // edges on src
  if (live && cplus != 0) {
    const uint64_t y = bounded(kb, 2, c + cplus);
    if (y >= c) {
      const uint64_t phi = y - c;
      src = phi < ld ? u : v;
      kk = (uint32_t)(phi < ld ? phi : phi - ld);
      pick = true;
    }
    const uint64_t tot = c + cplus;
    if (tot > kChiMax) {
      atomicOr(a.err, kErrOverflow);
      c = kChiMax;
    } else {
      c = tot;
    }
  }
  if (__syncthreads_or(pick)) {
    uint32_t seen = 0;
    for (uint32_t t = ntile; t-- > 0;) {
      load_tile(t);
      if (!pick || p2 != kNone) continue;
      const uint32_t j0 = t * kNaiveTile, n = min(kNaiveTile, a.w - j0);
      uint32_t k = n;
      for (; k >= 8; k -= 8) {  // edges k-8 .. k-1, eight reads per round
        uint32_t hit = 0;  // bit q: edge k-8+q is on src
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint2 ed = s_w[k - 8 + q];
          hit |= (ed.x == src || ed.y == src) ? (1u << q) : 0u;
        }
        const uint32_t cnt = __popc(hit);
        if (seen + cnt <= kk) {
          seen += cnt;
          continue;
        }
        // the (kk - seen)-th set bit counted from the top
        uint32_t need = kk - seen;
        for (int q = 7; q >= 0; --q) {
          if (!((hit >> q) & 1u)) continue;
          if (need == 0) {
            p2 = j0 + k - 8 + q;
            break;
          }
          --need;
        }
        break;
      }
      if (p2 == kNone) {
        for (; k-- > 0;) {
          const uint2 ed = s_w[k];
          if (ed.x != src && ed.y != src) continue;
          if (seen == kk) {
            p2 = j0 + k;
            break;
          }
          ++seen;
        }
      }
    }
    if (pick) {
      if (p2 == kNone) {  // cannot happen: kk < the count just taken
        atomicOr(a.err, kErrIndex);
        pick = false;
      } else {
        const uint2 ed = W[p2];
        r2 = canon(ed.x, ed.y);
        closed = false;
      }
    }
  }

  // Step 3: the latest occurrence of the closing edge decides
  uint64_t q = kEmpty;
  if (live && r2 != kEmpty && !closed) q = closing(r1, r2);
  if (__syncthreads_or(q != kEmpty)) {
    bool found = false;
    for (uint32_t t = ntile; t-- > 0;) {
      load_tile(t);
      if (q == kEmpty || found) continue;
      const uint32_t j0 = t * kNaiveTile, n = min(kNaiveTile, a.w - j0);
      uint32_t k = n;
      for (; k >= 8 && !found; k -= 8) {
        uint32_t hit = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint2 ed = s_w[k - 8 + b];
          hit |= canon(ed.x, ed.y) == q ? (1u << b) : 0u;
        }
        if (hit) {  // the latest of them
          const uint32_t jl = j0 + k - 8 + (31u - __clz(hit));
          closed = p2 == kNone || jl > p2;
          found = true;
        }
      }
      for (; k-- > 0 && !found;) {
        const uint2 ed = s_w[k];
        if (canon(ed.x, ed.y) != q) continue;
        closed = p2 == kNone || j0 + k > p2;
        found = true;
      }
    }
  }
  if (!live) return;
  a.r1[e] = r1;
  a.r2[e] = r2;
  a.cc[e] = (uint32_t)c | (closed ? kClosed : 0u);
}

hipError_t launch_naive(const NaiveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_naive, dim3((a.r + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// estimate and small utilities
// ---------------------------------------------------------------------------
// group of local estimator i of n: with bank offsets, its bank; otherwise
// its median-of-means group k = floor(((i+1) g - 1) / n), i.e. the groups
// [floor(k n / g), floor((k+1) n / g)), k < g <= n
__device__ __forceinline__ uint32_t group_of(uint64_t i, const uint64_t* bank_off,
                                             uint32_t nbanks, uint64_t n, uint32_t g) {
  if (bank_off) {
    uint32_t lo = 0, hi = nbanks - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (bank_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  return (uint32_t)(((i + 1) * (uint64_t)g - 1) / n);
}

// S_k = sum of chi * closed over the estimators of each group k, for the
// estimators e0 .. e0 + n - 1 (groups are consecutive, so a block's
// kGsumChunk estimators fall in at most kGsumChunk groups: summed in LDS
// first, then one global atomic per group the block touches)
constexpr uint32_t kGsumChunk = kBlock * 16;
__global__ __launch_bounds__(kBlock) void k_gsum(const uint32_t* cc, uint64_t e0, uint64_t n,
                                                 const uint64_t* bank_off, uint32_t nbanks,
                                                 uint32_t g, unsigned long long* sums) {
  __shared__ unsigned long long acc[kGsumChunk];
  const int tid = threadIdx.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * kGsumChunk;
  for (uint32_t t = tid; t < kGsumChunk; t += kBlock) acc[t] = 0;
  const uint32_t k0 = group_of(b0, bank_off, nbanks, n, g);
  __syncthreads();
  for (uint32_t t = tid; t < kGsumChunk; t += kBlock) {
    const uint64_t i = b0 + t;
    if (i >= n) break;
    const uint32_t w = cc[e0 + i];
    if (w & kClosed)
      atomicAdd(&acc[group_of(i, bank_off, nbanks, n, g) - k0],
                (unsigned long long)(w & kChiMax));
  }
  __syncthreads();
  for (uint32_t t = tid; t < kGsumChunk; t += kBlock)
    if (acc[t]) atomicAdd(&sums[k0 + t], acc[t]);
}

__global__ __launch_bounds__(kBlock) void k_fill64(uint64_t* p, uint64_t n,
                                                   uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill32(uint32_t* p, uint64_t n,
                                                   uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// k_small: the whole step (Steps 1-3) for chunks of at most kSmallW edges,
// in one launch and in LDS.  Block (chunk, slice) copies W, sorts its 2w
// arcs (vertex << 32 | arc id, unique keys, so the order is the stable
// grouping by vertex: the rankAll order read in increasing position) with
// a bitonic network, builds a table of the chunk's edges and their latest
// positions, and runs every estimator of its slice through the same Steps
// as k_fold_step1 / k_est / the join: the draws, the same ld/rd (segment
// ends found by binary search of the sorted arcs), the same selection and
// the same closing-edge test.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t small_seg(const SmallArgs& a, uint32_t b) {
  if (a.nseg == 1) return 0;
  uint32_t lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (a.descs[mid].blk_off <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// first index in s[0, n) whose key is >= k (s sorted ascending)
__device__ __forceinline__ uint32_t lds_lower_bound(const uint64_t* s, uint32_t n, uint64_t k) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Stable LSD radix sort of the n <= kSmallArcs arcs in s by their vertex
// (the high word), 8 bits a pass over the bits of vmax, through the buffer
// t; the result ends in s.  Wave w ranks elements [w kSmallPerWave, (w+1)
// kSmallPerWave) in order, four rounds of 64: lanes with equal digits find
// each other by ballots, and the lowest adds their number to the wave's
// count of that digit with a returning LDS atomic (a wave's atomics land in
// program order, so each returns the count of earlier equal digits).
constexpr uint32_t kSmallArcs = 2 * kSmallW;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr uint32_t kSmallPerWave = kSmallArcs / kSmallWaves;
static_assert(kSmallPerWave % 64 == 0, "whole rounds of 64 arcs per wave");

__device__ void small_sort(uint64_t* s, uint64_t* t, uint32_t n, uint32_t vmax,
                           uint32_t (*s_wh)[256], uint32_t* s_start, uint32_t* s_part) {
  constexpr int kRounds = (int)(kSmallPerWave / 64);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const int nbits = 32 - __clz(vmax | 1u);
  for (int sh = 0; sh < nbits; sh += 8) {
    for (uint32_t i = tid; i < kSmallWaves * 256u; i += kSmallThreads) (&s_wh[0][0])[i] = 0;
    __syncthreads();
    uint64_t el[kRounds];
    uint32_t dg[kRounds], rk[kRounds];
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
      const uint32_t i = (uint32_t)wave * kSmallPerWave + it * 64 + lane;
      const bool valid = i < n;
      el[it] = valid ? s[i] : 0ull;
      dg[it] = (uint32_t)(el[it] >> (32 + sh)) & 255u;
      uint64_t mm = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((dg[it] >> b) & 1u);
        mm &= ((dg[it] >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t below = (uint32_t)__popcll(mm & lt);
      uint32_t base = 0;
      if (valid && below == 0) base = atomicAdd(&s_wh[wave][dg[it]], (uint32_t)__popcll(mm));
      const int leader = (int)(((uint32_t)__ffsll((long long)mm) - 1u) & 63u);
      rk[it] = valid ? __shfl(base, leader) + below : 0u;
    }
    __syncthreads();
    // per digit: the waves' counts become offsets, the digits' totals an
    // exclusive scan (threads 0..255, one digit each)
    uint32_t tot = 0;
    if (tid < 256) {
#pragma unroll
      for (int w = 0; w < kSmallWaves; ++w) {
        const uint32_t c = s_wh[w][tid];
        s_wh[w][tid] = tot;
        tot += c;
      }
    }
    uint32_t x = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (tid < 256 && lane == 63) s_part[wave] = x;
    __syncthreads();
    if (tid < 256) {
      uint32_t off = 0;
      for (int w = 0; w < wave; ++w) off += s_part[w];
      s_start[tid] = off + x - tot;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
      const uint32_t i = (uint32_t)wave * kSmallPerWave + it * 64 + lane;
      if (i < n) t[s_start[dg[it]] + s_wh[wave][dg[it]] + rk[it]] = el[it];
    }
    __syncthreads();
    uint64_t* u = s;
    s = t;
    t = u;
  }
  // an odd number of passes left the result in the other buffer
  if (((nbits + 7) / 8) & 1) {
    for (uint32_t i = threadIdx.x; i < n; i += kSmallThreads) t[i] = s[i];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSmallThreads) void k_small(SmallArgs a) {
  constexpr uint32_t kArcs = kSmallArcs;
  constexpr uint32_t kTab = 2 * kSmallW;  // edge table slots (load <= 1/2)
  __shared__ uint2 s_w[kSmallW];
  __shared__ uint64_t s_arc[kArcs];
  __shared__ uint64_t s_ek[kTab];  // canonical edge, kEmpty = free (the sort's
                                   // second buffer before that)
  __shared__ uint32_t s_ep[kTab];  // 1 + its latest position
  __shared__ uint32_t s_wh[kSmallWaves][256];
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_part[4];
  __shared__ uint32_t s_seg, s_bad, s_vmax;
  static_assert(kTab == kArcs, "the edge table's keys double as the sort buffer");
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_seg = small_seg(a, blockIdx.x);
    s_bad = 0;
    s_vmax = 0;
  }
  __syncthreads();
  if (*a.err & kErrFatal) return;
  const SmallDesc S = a.nseg == 1 ? a.d0 : a.descs[uniform(s_seg)];
  const uint32_t w = S.w, n = 2u * w;
  const uint2* W = reinterpret_cast<const uint2*>(S.edges);
  bool loop = false;
  uint32_t vmax = 0;
  for (uint32_t j = tid; j < w; j += kSmallThreads) {
    const uint2 ed = W[j];
    s_w[j] = ed;
    loop |= ed.x == ed.y;
    vmax = max(vmax, max(ed.x, ed.y));
    s_arc[2 * j] = ((uint64_t)ed.x << 32) | (2u * j);
    s_arc[2 * j + 1] = ((uint64_t)ed.y << 32) | (2u * j + 1u);
  }
  atomicMax(&s_vmax, vmax);
  if (loop) {
    atomicOr(a.err, kErrSelfLoop);
    s_bad = 1;
  }
  if (vmax > a.id_limit) {
    atomicOr(a.err, kErrRange);
    s_bad = 1;
  }
  __syncthreads();
  if (s_bad) return;
  // the arcs by vertex, stably (arc ids ascend within a vertex, as built)
  small_sort(s_arc, s_ek, n, s_vmax, s_wh, s_start, s_part);
  for (uint32_t i = tid; i < kTab; i += kSmallThreads) {
    s_ek[i] = kEmpty;
    s_ep[i] = 0;
  }
  __syncthreads();
  // the chunk's edges and their latest positions (1 + position, 0 = none)
  constexpr uint32_t kTabMask = kTab - 1;
  for (uint32_t j = tid; j < w; j += kSmallThreads) {
    const uint64_t q = canon(s_w[j].x, s_w[j].y);
    uint32_t h = (uint32_t)mix64(q) & kTabMask;
    for (;;) {
      const unsigned long long prev = atomicCAS(
          reinterpret_cast<unsigned long long*>(&s_ek[h]), (unsigned long long)kEmpty,
          (unsigned long long)q);
      if (prev == kEmpty || prev == q) break;
      h = (h + 1) & kTabMask;
    }
    atomicMax(&s_ep[h], j + 1);
  }
  __syncthreads();

  const uint32_t i0 = (blockIdx.x - S.blk_off) * kSmallR, i1 = min(i0 + kSmallR, S.r);
  for (uint32_t i = i0 + tid; i < i1; i += kSmallThreads) {
    const uint64_t e = S.est_off + i;
    uint64_t r1 = a.r1[e], r2 = a.r2[e];
    const uint32_t ccw = a.cc[e];
    uint64_t c = ccw & kChiMax;
    bool closed = (ccw & kClosed) != 0;
    const uint64_t kb = mix64(mix64(S.key0 ^ (uint64_t)i) ^ S.batch);
    // Step 1 (Sec. 4.2): x uniform on [0, m + w); x >= m takes W[x - m]
    const uint64_t x = bounded(kb, 1, S.m + w);
    uint32_t j1 = kNone, au = 0, av = 0;
    if (x >= S.m) {
      j1 = (uint32_t)(x - S.m);
      const uint2 ed = s_w[j1];
      r1 = canon(ed.x, ed.y);
      c = 0;
      r2 = kEmpty;
      closed = false;
      // arc ids of W[j1]'s endpoints u = min, v = max
      au = ed.x < ed.y ? 2u * j1 : 2u * j1 + 1u;
      av = au ^ 1u;
    }
    // Step 2 (Sec. 4.3): the segments of u and v in the sorted arcs
    const uint32_t u = (uint32_t)(r1 >> 32), v = (uint32_t)r1;
    const uint32_t su = lds_lower_bound(s_arc, n, (uint64_t)u << 32);
    const uint32_t eu = u == 0xFFFFFFFFu ? n : lds_lower_bound(s_arc, n, (uint64_t)(u + 1) << 32);
    const uint32_t sv = lds_lower_bound(s_arc, n, (uint64_t)v << 32);
    const uint32_t ev = v == 0xFFFFFFFFu ? n : lds_lower_bound(s_arc, n, (uint64_t)(v + 1) << 32);
    uint32_t ld, rd;
    if (j1 != kNone) {
      // the arcs after f1's own in their segments
      ld = eu - 1 - lds_lower_bound(s_arc, n, ((uint64_t)u << 32) | au);
      rd = ev - 1 - lds_lower_bound(s_arc, n, ((uint64_t)v << 32) | av);
    } else {
      ld = eu - su;
      rd = ev - sv;
    }
    const uint64_t cplus = (uint64_t)ld + rd;
    uint32_t p2 = kNone;
    if (cplus != 0) {
      const uint64_t tot = c + cplus;
      const uint64_t y = bounded(kb, 2, tot);
      if (y >= c) {
        const uint64_t phi = y - c;
        const uint32_t idx = phi < ld ? eu - 1 - (uint32_t)phi : ev - 1 - (uint32_t)(phi - ld);
        p2 = ((uint32_t)s_arc[idx] & kIdMask) >> 1;
        const uint2 ed = s_w[p2];
        r2 = canon(ed.x, ed.y);
        closed = false;
      }
      if (tot > kChiMax) {
        atomicOr(a.err, kErrOverflow);
        c = kChiMax;
      } else {
        c = tot;
      }
    }
    // Step 3 (Sec. 4.4): closed iff the closing edge comes at or after the
    // first position that may close it
    if (r2 != kEmpty && !closed) {
      const uint64_t q = closing(r1, r2);
      if (q != kEmpty) {
        const uint32_t thr = p2 == kNone ? 0u : p2 + 1u;
        for (uint32_t h = (uint32_t)mix64(q) & kTabMask;; h = (h + 1) & kTabMask) {
          const uint64_t k = s_ek[h];
          if (k == kEmpty) break;
          if (k == q) {
            closed = s_ep[h] > thr;
            break;
          }
        }
      }
    }
    if (j1 != kNone) a.r1[e] = r1;
    a.r2[e] = r2;
    a.cc[e] = (uint32_t)c | (closed ? kClosed : 0u);
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
// The step runs in three phases (see the engine): A groups the batch
// (k_hist .. k_dir), B is k_est, C is Step 3 (k_pcnt .. k_pjoin) and may run
// on another stream, overlapping the next step's phase A.  ev: optional
// 2 * kNumKernels events; kernel k is bracketed by ev[2k] and ev[2k+1]
// when those are non-null (untimed kernels get no event).
// the grouping sort of one step with D-bit digits: launch 0 k_hist, 1 the
// fold (and Step 1), 2 k_cscan<0>, 3 k_scat<0>; pass P >= 1 is launches
// 4 + 4 (P - 1) + {k_cnt, k_csum, k_cscan, k_scat}.  Passes above the
// declared vertex bound are not launched (k_hist reports an id above it),
// nor is k_cscan when every segment is a single chunk (8-bit digits).
template <int D, class Run>
void launch_sort(const StepArgs& a, hipStream_t st, Run& run) {
  constexpr uint32_t kPer = Rdx<D>::kPer;
  const dim3 blk(kBlock), tiles(a.ntiles);
  const dim3 chunks(a.nchunk * kPer), segs(a.nseg * (Rdx<D>::kBins / 64));
  run(0, [&] { hipLaunchKernelGGL(k_hist<D>, dim3(a.nhblk), blk, 0, st, a); });
  run(1, [&] {
    const dim3 g(a.nchunk * kPer + a.nstep1);
    if (a.nseg == 1) hipLaunchKernelGGL((k_fold_step1<D, true>), g, blk, 0, st, a);
    else hipLaunchKernelGGL((k_fold_step1<D, false>), g, blk, 0, st, a);
  });
  if (!a.single_chunk)
    run(2, [&] { hipLaunchKernelGGL((k_cscan<0, D>), segs, blk, 0, st, a); });
  run(3, [&] { hipLaunchKernelGGL((k_scat<0, D>), tiles, blk, 0, st, a); });
  auto pass = [&](int P, auto cntk, auto csumk, auto cscank, auto scatk) {
    const int k = 4 + 4 * (P - 1);
    run(k, [&] { hipLaunchKernelGGL(cntk, tiles, blk, 0, st, a); });
    run(k + 1, [&] { hipLaunchKernelGGL(csumk, chunks, blk, 0, st, a); });
    if (!a.single_chunk) run(k + 2, [&] { hipLaunchKernelGGL(cscank, segs, blk, 0, st, a); });
    run(k + 3, [&] { hipLaunchKernelGGL(scatk, tiles, blk, 0, st, a); });
  };
  if constexpr (D == 8) {
    if (a.npass > 1) pass(1, k_cnt<1, 8>, k_csum<1, 8>, k_cscan<1, 8>, k_scat4<1, 8>);
    if (a.npass > 2) pass(2, k_cnt<2, 8>, k_csum<2, 8>, k_cscan<2, 8>, k_scat4<2, 8>);
    if (a.npass > 3) pass(3, k_cnt<3, 8>, k_csum<3, 8>, k_cscan<3, 8>, k_scat<3, 8>);
  } else {
    if (a.npass > 1) pass(1, k_cnt<1, D>, k_csum<1, D>, k_cscan<1, D>, k_scat4<1, D>);
  }
}

hipError_t launch_phase(int phase, const StepArgs& a, hipStream_t st,
                        hipEvent_t* ev) {
  const dim3 blk(kBlock);
  const dim3 tiles(a.ntiles);
  const dim3 ests((uint32_t)((a.nest + kBlock - 1) / kBlock));
  auto run = [&](int k, auto&& launch) {
    const bool t = ev && ev[2 * k];
    if (t) (void)hipEventRecord(ev[2 * k], st);
    launch();
    if (t) (void)hipEventRecord(ev[2 * k + 1], st);
  };
  if (phase == 0) {
    if (a.dbits == (uint32_t)kWideBits) {
      static_assert(kWidePasses == 2, "wide digits take two passes");
      launch_sort<kWideBits>(a, st, run);
    } else {
      launch_sort<8>(a, st, run);
    }
    run(kSmallKernel - 6, [&] { hipLaunchKernelGGL(k_dir, tiles, blk, 0, st, a); });
  } else if (phase == 1) {
    run(kSmallKernel - 5, [&] {
      if (a.nseg == 1) hipLaunchKernelGGL(k_est<true>, ests, blk, 0, st, a);
      else hipLaunchKernelGGL(k_est<false>, ests, blk, 0, st, a);
    });
  } else {
    const dim3 pblk(kPThreads), jblk(kJoinThreads);
    run(kSmallKernel - 4, [&] { hipLaunchKernelGGL(k_pcnt, dim3(a.nptile), pblk, 0, st, a); });
    run(kSmallKernel - 3, [&] { hipLaunchKernelGGL(k_pscan, dim3(a.npscan), pblk, 0, st, a); });
    run(kSmallKernel - 2, [&] { hipLaunchKernelGGL(k_pscat, dim3(a.nptile), pblk, 0, st, a); });
    run(kSmallKernel - 1, [&] { hipLaunchKernelGGL(k_pjoin, dim3(a.njblk), jblk, 0, st, a); });
  }
  return hipGetLastError();
}

hipError_t launch_small(const SmallArgs& a, hipStream_t st, hipEvent_t* ev) {
  const bool t = ev && ev[2 * kSmallKernel];
  if (t) (void)hipEventRecord(ev[2 * kSmallKernel], st);
  hipLaunchKernelGGL(k_small, dim3(a.nblk), dim3(kSmallThreads), 0, st, a);
  if (t) (void)hipEventRecord(ev[2 * kSmallKernel + 1], st);
  return hipGetLastError();
}

hipError_t launch_gsum(const uint32_t* cc, uint64_t e0, uint64_t n,
                       const uint64_t* bank_off, uint32_t nbanks, uint32_t g,
                       unsigned long long* sums, hipStream_t st) {
  const uint32_t ngroups = bank_off ? nbanks : g;
  hipLaunchKernelGGL(k_fill64, dim3(1), dim3(kBlock), 0, st,
                     reinterpret_cast<uint64_t*>(sums), (uint64_t)ngroups, 0ull);
  if (n == 0) return hipGetLastError();
  const uint64_t nb = (n + kGsumChunk - 1) / kGsumChunk;
  hipLaunchKernelGGL(k_gsum, dim3((uint32_t)nb), dim3(kBlock), 0, st, cc, e0, n,
                     bank_off, nbanks, g, sums);
  return hipGetLastError();
}

hipError_t launch_fill64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = std::min<uint64_t>((n + kBlock - 1) / kBlock, 65536);
  hipLaunchKernelGGL(k_fill64, dim3((uint32_t)nb), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = std::min<uint64_t>((n + kBlock - 1) / kBlock, 65536);
  hipLaunchKernelGGL(k_fill32, dim3((uint32_t)nb), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace tc
