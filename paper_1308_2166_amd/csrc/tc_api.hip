// Host side of libtc: bank storage, per-step scratch, the C-ABI.
//
// A tc_multi owns the estimator state of all its banks (structure of arrays
// in HBM) and the scratch of one step; a tc_state is a tc_multi with one
// bank.  Scratch grows to the largest step seen and is then reused, so a
// steady stream of equal-sized batches allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/tc.h"
#include "tc_internal.h"

// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid it) run a step entirely in this
// array (tc_process_batch_noalloc): every buffer of the step is carved from
// it.  Each device holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static constexpr uint64_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace tc {
hipError_t launch_phase(int phase, const StepArgs& a, hipStream_t st, hipEvent_t* ev);
hipError_t launch_gsum(const uint32_t* cc, uint64_t e0, uint64_t n,
                       const uint64_t* bank_off, uint32_t nbanks, uint32_t g,
                       unsigned long long* sums, hipStream_t st);
hipError_t launch_fill64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
hipError_t launch_naive(const NaiveArgs& a, hipStream_t st);
hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
hipError_t launch_small(const SmallArgs& a, hipStream_t st, hipEvent_t* ev);
}  // namespace tc

namespace {

using namespace tc;

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t log2_ceil(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// directory slots for a chunk of w edges: at most 2w distinct vertices,
// load <= 1/2 when hashed
uint32_t dir_log2_for(uint32_t w) {
  return std::max<uint32_t>(10, log2_ceil(4ull * w));
}
// Launch shapes a caller may tune (tc_set_tuning); none changes a result.
struct Tuning {
  uint32_t digits8 = 0;           // 1: 8-bit radix digits whatever the bound
  uint32_t chunk_log2 = 5;        // radix tiles per chunk of the scans: 8..kChunk
  uint32_t part_q = kPartQ;       // Step-3 estimators per partition aimed at
  uint32_t join_edges = kJoinEdges;  // Step-3 batch edges per join slice aimed at
  uint32_t fused_edges = kSmallW;    // chunks of at most this many edges take the
                                     // fused single-launch step (0: none)
};
constexpr uint32_t kMinChunkLog2 = 3;
constexpr uint32_t kMinPartQ = 512;

// Step-3 join of a bank of r estimators: partitions of about part_q
// waiting estimators each (at most 2^kMaxPartLog2), tiles of kPTile
// elements, and join slices of about join_edges batch edges
uint32_t part_log2_for(uint32_t r, uint32_t part_q = kPartQ) {
  return std::min<uint32_t>(kMaxPartLog2, log2_ceil((r + part_q - 1) / part_q));
}
// partition tiles of a chunk in a step of nseg chunks: about 32 per side
// over the step (at least 2^kMinPTileLog2 elements each, at most kPTile), so
// that a small step still spreads over the GPU; and tiles of n elements at
// that size
uint32_t ptile_log2_for(uint32_t r, uint32_t w, uint32_t nseg = 1) {
  const uint64_t n = (uint64_t)std::max(r, w) * nseg / 32;
  const uint32_t l = n ? 63u - (uint32_t)__builtin_clzll(n) : 0u;
  return std::min<uint32_t>(log2_ceil(kPTile), std::max(kMinPTileLog2, l));
}
uint32_t ptiles_for(uint64_t n, uint32_t ptl) { return (uint32_t)((n + (1ull << ptl) - 1) >> ptl); }
// join slices of a partition: about join_edges batch edges each, and for a
// small step enough of them for about 64 join blocks over the step (of at
// least 256 edges each)
uint32_t jslices_for(uint32_t w, uint32_t pbits, uint32_t join_edges = kJoinEdges,
                     uint32_t nseg = 1) {
  const uint64_t per = (uint64_t)join_edges << pbits;
  const uint64_t by_size = (w + per - 1) / per;
  const uint64_t spread = std::min<uint64_t>(((64u / std::max(1u, nseg)) >> pbits) + 1,
                                             (w + (256ull << pbits) - 1) >> (8 + pbits));
  return (uint32_t)std::max<uint64_t>(1, std::max(by_size, spread));
}

// Scratch a step needs for one more chunk of w > 0 edges of a bank of r
// estimators (the per-segment regions plan() hands out, in the same order).
struct Sizes;
void add_chunk(Sizes& z, uint32_t r, uint32_t w, uint32_t part_q = kPartQ, uint32_t nseg = 1);

template <class T>
hipError_t dalloc(T** p, uint64_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// kernels (bit k = launch k of a step) that the chain of a step with npass
// radix passes launches: the four kernels of each pass at or above npass are
// skipped, and every pass's k_cscan when the step's segments are single
// chunks (k_small, the fused step, is not part of the chain)
uint32_t launched_kernels(uint32_t npass, bool single_chunk) {
  static_assert(kSmallKernel == kNumKernels - 1, "the chain's kernels come first");
  uint32_t m = (1u << kSmallKernel) - 1u;
  for (uint32_t p = npass < 1 ? 1 : npass; p < (uint32_t)kPasses; ++p)
    m &= ~(15u << (4 + 4 * (p - 1)));
  if (single_chunk)
    for (uint32_t p = 0; p < (uint32_t)kPasses; ++p) m &= ~(1u << (2 + 4 * p));
  return m;
}


// Per-parity scratch: the Step-3 phase of step s (on the engine's second
// stream) overlaps the grouping phase of step s+1, so everything both
// phases touch exists twice and step s uses copy s & 1.
struct ParityScratch {
  SegWork* work = nullptr;    // per-segment histograms, counters, modes
  SegDesc* segs = nullptr;    // device copy of the step's descriptors
};

// Sizes a step's scratch must hold.
struct Sizes {
  uint64_t arcs = 0;   // arc slots (2 w summed over segments)
  uint64_t tiles = 0;  // radix tiles
  uint64_t dir = 0;    // directory slots
  uint64_t doff = 0;   // dense-directory words
  uint64_t prow = 0;   // Step-3 partition-count row words
  uint64_t parts = 0;  // Step-3 partitions
  uint64_t need = 0;   // need bytes
  uint64_t nest = 0;   // estimators (per-estimator step words)
  uint32_t segs = 0;   // segments
  bool fits(const Sizes& z) const {
    return z.arcs <= arcs && z.tiles <= tiles && z.dir <= dir && z.doff <= doff &&
           z.prow <= prow && z.parts <= parts &&
           z.need <= need && z.nest <= nest && z.segs <= segs;
  }
  void grow(const Sizes& z) {
    arcs = std::max(arcs, z.arcs), tiles = std::max(tiles, z.tiles);
    dir = std::max(dir, z.dir), need = std::max(need, z.need);
    prow = std::max(prow, z.prow), parts = std::max(parts, z.parts);
    doff = std::max(doff, z.doff);
    nest = std::max(nest, z.nest), segs = std::max(segs, z.segs);
  }
};

void add_chunk(Sizes& z, uint32_t r, uint32_t w, uint32_t part_q, uint32_t nseg) {
  const uint32_t dl = dir_log2_for(w);
  z.need += (w + 15) / 16 * 16;
  z.arcs += 2ull * w;
  z.tiles += (2ull * w + kTile - 1) / kTile;
  z.dir += 1ull << dl;
  z.doff += (1ull << dl) + kDoffPad;
  const uint32_t pb = part_log2_for(r, part_q), ptl = ptile_log2_for(r, w, nseg);
  z.prow += (uint64_t)(ptiles_for(w, ptl) + ptiles_for(r, ptl)) << pb;
  z.parts += 1ull << pb;
  z.nest += r;
  z.segs += 1;
}

// Sizes that hold every step of at most n chunks (banks of at most r_max
// estimators) with at most E edges in all, under any tuning: per field, the
// largest total add_chunk can reach (2^ceil(log2 x) < 2x bounds the rounded
// regions; the most partitions come with the fewest estimators per one).
Sizes step_bound(uint32_t n, uint32_t r_max, uint64_t E) {
  Sizes z;
  if (n == 0 || E == 0) return z;
  z.arcs = 2 * E;
  z.tiles = 2 * E / kTile + n;
  z.dir = 8 * E + 1024ull * n;
  z.doff = z.dir + (uint64_t)kDoffPad * n;
  const uint32_t pb = part_log2_for(r_max, kMinPartQ);  // grows with r
  z.prow = ((E >> kMinPTileLog2) + n + (uint64_t)n * ptiles_for(r_max, kMinPTileLog2)) << pb;
  z.parts = (uint64_t)n << pb;
  z.need = E + 16ull * n;
  z.nest = (uint64_t)n * r_max;
  z.segs = n;
  return z;
}

// Device bytes a bank of r estimators holds for its life: f1, f2 and the
// packed chi/closed word (20 B), and the per-estimator step words j1, qq
// and qthr (16 B).
constexpr uint64_t kBankBytesPerEst = 8 + 8 + 4 + 4 + 8 + 4;

// The per-step scratch buffers, carved from one block of device memory.
struct Scratch {
  uint64_t* arcs[2] = {nullptr, nullptr};
  uint32_t* csum = nullptr;   // radix chunk sums / prefixes
  DirSlot* dir = nullptr;
  uint32_t* doff = nullptr;  // dense directories (rewritten every step)
  uint8_t* need = nullptr;
  uint32_t* inv = nullptr;
  uint32_t* prow = nullptr;   // Step-3 join: partition-count rows,
  uint32_t* ptot = nullptr;   // partition totals and starts (two sides),
  uint32_t* pstart = nullptr;
  uint64_t* erec = nullptr;   // and the partitioned records
  uint64_t* qrec = nullptr;
  uint32_t* hpart = nullptr;  // k_hist partial counts (one row per tile)
  uint32_t* mpart = nullptr;  // k_hist partial max ids
  ParityScratch par[2];
  // per-estimator step words and the directory tag: carved only for the
  // static scratch of tc_process_batch_noalloc (an engine's own live with
  // its banks)
  uint32_t* j1 = nullptr;
  uint64_t* qq = nullptr;
  uint32_t* qthr = nullptr;
  uint32_t* tagp = nullptr;
};

// Directory slots the static scratch holds (batches of up to 2^18 edges).
// It sits at a fixed offset, with the tag word and the work area: their
// contents carry over from one call to the next, while every other buffer
// is rewritten before it is read, so it may move with the step's sizes.
constexpr uint64_t kStaticDirSlots = 1ull << 20;

// Lay out the buffers of a step of sizes z from `base` (nullptr: only
// count), each 256-byte aligned, with `nparity` copies of the per-parity
// part.  stat: the static-scratch layout (one parity, one segment): the
// tag word, the work area and a directory of kStaticDirSlots slots first,
// then the per-estimator words.  Returns the bytes the layout takes.
uint64_t carve(uint8_t* base, const Sizes& z, int nparity, bool stat, Scratch* out) {
  uint64_t off = 0;
  auto take = [&](auto*& p, uint64_t n) {
    using T = std::remove_reference_t<decltype(*p)>;
    off = (off + 255) & ~255ull;
    p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<uint64_t>(n, 1) * sizeof(T);
  };
  Scratch s;
  if (stat) {
    nparity = 1;
    take(s.tagp, 64);
    take(s.par[0].work, 1);
    take(s.dir, kStaticDirSlots);
    take(s.j1, z.nest), take(s.qq, z.nest), take(s.qthr, z.nest);
  }
  take(s.arcs[0], z.arcs), take(s.arcs[1], z.arcs);
  // (chunks of at least 2^kMinChunkLog2 tiles, plus one ragged per segment)
  take(s.csum, ((z.tiles >> kMinChunkLog2) + z.segs) * kRowWords);
  if (!stat) take(s.dir, z.dir);
  take(s.doff, z.doff);
  take(s.need, z.need), take(s.inv, z.arcs);
  take(s.hpart, z.tiles * kRowWords), take(s.mpart, z.tiles);
  // (one copy: the join runs only while no other step's join does)
  take(s.prow, z.prow), take(s.ptot, 2 * z.parts), take(s.pstart, 2 * z.parts);
  take(s.erec, z.arcs / 2), take(s.qrec, z.nest);
  for (int p = 0; p < nparity; ++p) {
    ParityScratch& P = s.par[p];
    if (!stat) take(P.work, z.segs);
    if (!stat) take(P.segs, z.segs);
  }
  if (nparity == 1) s.par[1] = s.par[0];
  if (out) *out = s;
  return (off + 255) & ~255ull;
}

// ---- the static scratch of tc_process_batch_noalloc ------------------------
struct StaticScratch {
  bool looked_up = false;
  hipError_t status = hipSuccess;
  uint8_t* ptr = nullptr;    // the device address of `scratch`
  uint64_t steps = 0;        // steps run in it (directory tag wrap guard)
  bool dirty = false;        // a step's launches failed part-way: the work
                             // area and directory are cleared before the next
};
std::mutex g_static_mu;
StaticScratch g_static[64];  // per device ordinal

// Look up the device address of `scratch` on `device` (current) once.
StaticScratch* static_scratch(int device) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticScratch& s = g_static[device];
  if (!s.looked_up) {
    void* p = nullptr;
    s.status = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.ptr = s.status == hipSuccess ? static_cast<uint8_t*>(p) : nullptr;
    s.looked_up = true;
  }
  return &s;
}

struct Engine {
  int device = 0;
  uint32_t nbanks = 0;
  std::vector<uint32_t> r;
  std::vector<uint64_t> seed, key0, m, batch, est_off;  // est_off: nbanks+1
  uint64_t total = 0;

  // bank state (all banks, contiguous) and per-estimator step scratch
  uint64_t* R1 = nullptr;
  uint64_t* R2 = nullptr;
  uint32_t* CC = nullptr;
  uint32_t* J1 = nullptr;  // Step-1 replacement per estimator
  uint64_t* QQ = nullptr;  // closing edge each estimator waits for
  uint32_t* QT = nullptr;  // its first closing batch position
  uint64_t* bank_off = nullptr;  // device copy of est_off
  SmallDesc* sdesc = nullptr;    // device copy of a fused step's descriptors
  unsigned long long* sums = nullptr;
  unsigned long long* gsums = nullptr;  // median-of-means group sums
  uint64_t* h_gsums = nullptr;          // pinned
  uint32_t cap_groups = 0;
  uint32_t* err = nullptr;
  uint32_t* tagp = nullptr;  // directory tag (advanced by every step)
  unsigned long long* h_sums = nullptr;  // pinned
  uint32_t* h_err = nullptr;             // pinned

  // step scratch (one device block, carved), its capacity, and blocks
  // retired by a growth after some step was captured into a HIP graph
  // (a captured graph keeps their addresses; they are freed by
  // tc_multi_graph_reserve or destroy)
  Sizes cap;
  uint8_t* block = nullptr;
  Scratch S;
  bool captured = false;
  std::vector<uint8_t*> retired;
  uint64_t retired_bytes = 0;
  StaticScratch* stat = nullptr;  // the device's static scratch

  // host ingest (tc_process_host_stream): two device staging buffers of
  // hbuf_w edges, filled on the copy stream stc while the previous batch is
  // processed; h_ready[b] marks buffer b copied, h_free[b] its last reader
  // done (h_used[b]: h_free[b] has been recorded)
  hipStream_t stc = nullptr;
  uint32_t* hbuf[2] = {nullptr, nullptr};
  uint64_t hbuf_w = 0;
  hipEvent_t h_ready[2] = {nullptr, nullptr}, h_free[2] = {nullptr, nullptr};
  bool h_used[2] = {false, false};

  // the Step-3 phase runs on st2; evB orders it after k_est, evC orders
  // the next k_est (and any state access) after it
  hipStream_t st2 = nullptr;
  hipEvent_t evB = nullptr, evC = nullptr;
  bool c_pending = false;

  // pinned staging ring for multi-segment descriptors
  static constexpr int kRing = 4;
  SegDesc* stage[kRing] = {};
  hipEvent_t stage_ev[kRing] = {};
  bool stage_used[kRing] = {};
  uint32_t stage_cap = 0;
  int ring = 0;

  uint64_t steps = 0;  // steps enqueued (parity, tag wrap guard)
  hipStream_t last = nullptr;
  // descriptor staging for steps captured into a HIP graph: one pinned
  // buffer per captured step, kept unchanged so every replay reads it
  std::vector<SegDesc*> graph_stage;
  size_t graph_next = 0;
  int sticky = TC_OK;
  Tuning tune;
  uint32_t id_limit = 0xFFFFFFFFu;  // declared vertex bound - 1
  uint32_t npass = kPasses;
  uint32_t dbits = 8;  // radix digit width for that bound

  // optional per-kernel timing: a start/end event pair per timed kernel
  // and step (bit k of timing_mask times kernel k)
  bool timing = false;
  uint32_t timing_mask = 0;
  std::vector<hipEvent_t*> ev_pending, ev_free;
  std::vector<uint32_t> ev_launched;  // per pending step: kernels it launched
  double kernel_ms[kNumKernels] = {};
  uint64_t timed_steps = 0;

  ~Engine() { release(); }

  void wait_all() {
    if (last) (void)hipStreamSynchronize(last);
    if (st2) (void)hipStreamSynchronize(st2);
  }

  // make `st` wait for a Step-3 phase left on st2 by an overlapped step
  int join(hipStream_t st) {
    if (!c_pending) return TC_OK;
    c_pending = false;
    if (hipStreamWaitEvent(st, evC, 0) != hipSuccess)
      return fail(TC_EHIP, "hipStreamWaitEvent failed");
    return TC_OK;
  }

  void release() {
    wait_all();
    (void)hipDeviceSynchronize();
    ev_launched.clear();
    for (auto* v : {&ev_pending, &ev_free})
      for (hipEvent_t* e : *v) {
        for (int k = 0; k < 2 * kNumKernels; ++k)
          if (e[k]) (void)hipEventDestroy(e[k]);
        delete[] e;
      }
    ev_pending.clear();
    ev_free.clear();
    dfree(R1), dfree(R2), dfree(CC), dfree(J1), dfree(QQ), dfree(QT), dfree(bank_off);
    dfree(sdesc);
    dfree(sums), dfree(err), dfree(tagp), dfree(gsums);
    if (stc) (void)hipStreamSynchronize(stc);
    for (int b = 0; b < 2; ++b) {
      dfree(hbuf[b]);
      if (h_ready[b]) (void)hipEventDestroy(h_ready[b]);
      if (h_free[b]) (void)hipEventDestroy(h_free[b]);
      h_ready[b] = h_free[b] = nullptr;
      h_used[b] = false;
    }
    hbuf_w = 0;
    if (stc) (void)hipStreamDestroy(stc);
    stc = nullptr;
    if (h_gsums) (void)hipHostFree(h_gsums);
    h_gsums = nullptr;
    cap_groups = 0;
    for (SegDesc* g : graph_stage) (void)hipHostFree(g);
    graph_stage.clear();
    if (h_sums) (void)hipHostFree(h_sums);
    if (h_err) (void)hipHostFree(h_err);
    h_sums = nullptr, h_err = nullptr;
    free_scratch();
    free_retired();
    for (int i = 0; i < kRing; ++i) {
      if (stage[i]) (void)hipHostFree(stage[i]);
      if (stage_ev[i]) (void)hipEventDestroy(stage_ev[i]);
      stage[i] = nullptr, stage_ev[i] = nullptr;
    }
    if (evB) (void)hipEventDestroy(evB);
    if (evC) (void)hipEventDestroy(evC);
    if (st2) (void)hipStreamDestroy(st2);
    evB = evC = nullptr;
    st2 = nullptr;
  }

  void free_scratch() {
    if (block) (void)hipFree(block);
    block = nullptr;
    S = Scratch{};
    cap = Sizes{};
  }

  // free the blocks that captured graphs may still have referred to
  void free_retired() {
    for (uint8_t* b : retired) (void)hipFree(b);
    retired.clear();
    retired_bytes = 0;
  }

  int init(uint32_t n, const uint32_t* rr, const uint64_t* seeds) {
    if (hipGetDevice(&device) != hipSuccess) return fail(TC_EHIP, "hipGetDevice failed");
    stat = static_scratch(device);
    nbanks = n;
    r.assign(rr, rr + n);
    seed.assign(seeds, seeds + n);
    key0.resize(n);
    m.assign(n, 0);
    batch.assign(n, 0);
    est_off.resize(n + 1);
    est_off[0] = 0;
    for (uint32_t b = 0; b < n; ++b) {
      if (r[b] == 0) return fail(TC_EINVAL, "every bank needs r >= 1");
      key0[b] = host_mix64(seed[b] ^ kGolden);
      est_off[b + 1] = est_off[b] + r[b];
    }
    total = est_off[n];
    if (total >= 0x7FFFFFFFull)
      return fail(TC_EINVAL, "too many estimators in one object (max 2^31-2)");
    // default priority (same as the caller's streams)
    if (hipStreamCreateWithFlags(&st2, hipStreamNonBlocking) ||
        hipEventCreateWithFlags(&evB, hipEventDisableTiming) ||
        hipEventCreateWithFlags(&evC, hipEventDisableTiming))
      return fail(TC_EHIP, "stream or event creation failed");
    if (dalloc(&R1, total) || dalloc(&R2, total) || dalloc(&CC, total) ||
        dalloc(&J1, total) || dalloc(&QQ, total) || dalloc(&QT, total) ||
        dalloc(&bank_off, n + 1) || dalloc(&sdesc, n) ||
        dalloc(&sums, n) || dalloc(&err, 1) || dalloc(&tagp, 1))
      return fail(TC_ENOMEM, "device allocation of the estimator banks failed");
    if (hipHostMalloc(reinterpret_cast<void**>(&h_sums), sizeof(uint64_t) * n) ||
        hipHostMalloc(reinterpret_cast<void**>(&h_err), sizeof(uint32_t)))
      return fail(TC_ENOMEM, "pinned host allocation failed");
    if (launch_fill64(R1, total, kEmpty, nullptr) ||
        launch_fill64(R2, total, kEmpty, nullptr) ||
        launch_fill32(CC, total, 0, nullptr) ||
        launch_fill32(err, 1, 0, nullptr) ||
        launch_fill32(tagp, 1, 1, nullptr) ||
        hipMemcpy(bank_off, est_off.data(), sizeof(uint64_t) * (n + 1),
                  hipMemcpyHostToDevice) ||
        hipDeviceSynchronize())
      return fail(TC_EHIP, "initialising the estimator banks failed");
    return TC_OK;
  }

  // Grow the step scratch to hold z (no-op when it does).  After a step
  // was captured into a HIP graph the old block is retired, not freed: the
  // graph's kernels keep its addresses.
  int ensure_scratch(const Sizes& z, hipStream_t st) {
    if (cap.fits(z)) return TC_OK;
    wait_all();
    if (st) (void)hipStreamSynchronize(st);
    Sizes want = cap;
    want.grow(z);
    if (captured && block) {
      retired.push_back(block);
      retired_bytes += carve(nullptr, cap, 2, false, nullptr);
      block = nullptr;
    }
    free_scratch();
    const uint64_t bytes = carve(nullptr, want, 2, false, nullptr);
    if (hipMalloc(reinterpret_cast<void**>(&block), bytes) != hipSuccess) {
      block = nullptr;
      return fail(TC_ENOMEM, "device allocation of step scratch failed");
    }
    carve(block, want, 2, false, &S);
    cap = want;
    // zero = "no tag" for the directory, cleared work areas
    bool bad = hipMemsetAsync(S.dir, 0, sizeof(DirSlot) * cap.dir, st) ||
               hipMemsetAsync(S.need, 0, cap.need, st);
    for (ParityScratch& p : S.par)
      bad = bad || hipMemsetAsync(p.work, 0, sizeof(SegWork) * cap.segs, st);
    if (bad || hipStreamSynchronize(st))
      return fail(TC_EHIP, "clearing step scratch failed");
    return TC_OK;
  }

  int stage_descs(const std::vector<SegDesc>& segs, SegDesc* dst,
                  hipStream_t st, bool capturing) {
    return stage_bytes(segs.data(), (uint32_t)segs.size(), sizeof(SegDesc), dst, st, capturing);
  }

  // n items of `item` bytes (at most sizeof(SegDesc) each) to the device
  // buffer dst on st, through a pinned staging ring (or, under capture, the
  // captured step's own pinned buffer)
  int stage_bytes(const void* src, uint32_t n, size_t item, void* dst, hipStream_t st,
                  bool capturing) {
    if (capturing) {
      if (graph_next >= graph_stage.size())
        return fail(TC_EINVAL, "more captured steps than tc_multi_graph_reserve allowed");
      if (n > nbanks) return fail(TC_EINVAL, "too many chunks");
      SegDesc* buf = graph_stage[graph_next++];
      std::memcpy(buf, src, item * n);
      if (hipMemcpyAsync(dst, buf, item * n, hipMemcpyHostToDevice, st))
        return fail(TC_EHIP, "descriptor upload failed");
      return TC_OK;
    }
    if (n > stage_cap) {
      for (int i = 0; i < kRing; ++i) {
        if (stage_used[i]) (void)hipEventSynchronize(stage_ev[i]);
        if (stage[i]) (void)hipHostFree(stage[i]);
        stage[i] = nullptr;
        stage_used[i] = false;
        if (hipHostMalloc(reinterpret_cast<void**>(&stage[i]), sizeof(SegDesc) * n))
          return fail(TC_ENOMEM, "pinned descriptor staging failed");
        if (!stage_ev[i] && hipEventCreateWithFlags(&stage_ev[i], hipEventDisableTiming))
          return fail(TC_EHIP, "hipEventCreate failed");
      }
      stage_cap = n;
    }
    const int k = ring;
    ring = (ring + 1) % kRing;
    if (stage_used[k]) (void)hipEventSynchronize(stage_ev[k]);
    std::memcpy(stage[k], src, item * n);
    if (hipMemcpyAsync(dst, stage[k], item * n, hipMemcpyHostToDevice, st) ||
        hipEventRecord(stage_ev[k], st))
      return fail(TC_EHIP, "descriptor upload failed");
    stage_used[k] = true;
    return TC_OK;
  }

  // The segments of one step: a descriptor per chunk with w > 0 and the
  // scratch sizes they take.  Validates the chunk list.
  struct Plan {
    std::vector<SegDesc> segs;
    std::vector<uint32_t> bank;  // bank of each segment
    Sizes z;
    uint64_t hblks = 0, chunks = 0;
    uint64_t ptiles = 0, pscans = 0, jblks = 0;  // Step-3 grids
  };

  int plan(uint32_t nchunks, const uint32_t* ids, const uint32_t* const* edges,
           const uint32_t* w, bool reserve, Plan& pl) {
    pl.segs.reserve(nchunks);
    std::vector<char> seen(nbanks, 0);
    Sizes& z = pl.z;
    uint32_t nseg = 0;  // chunks with edges: the step's segments
    for (uint32_t k = 0; k < nchunks; ++k) nseg += w[k] != 0 && w[k] <= TC_MAX_BATCH;
    for (uint32_t k = 0; k < nchunks; ++k) {
      const uint32_t b = ids[k];
      if (b >= nbanks) return fail(TC_EINVAL, "bank id out of range");
      if (seen[b]) return fail(TC_EINVAL, "a bank appears twice in one step");
      seen[b] = 1;
      if (w[k] > TC_MAX_BATCH) return fail(TC_EINVAL, "batch larger than TC_MAX_BATCH");
      if (w[k] == 0) continue;
      if (!reserve && !edges[k]) return fail(TC_EINVAL, "null edge pointer with w > 0");
      if (!reserve && (reinterpret_cast<uintptr_t>(edges[k]) & 7u))
        return fail(TC_EINVAL, "edge buffer must be 8-byte aligned");
      SegDesc d{};
      d.edges = reserve ? nullptr : edges[k];
      d.m = m[b];
      d.batch = batch[b];
      d.key0 = key0[b];
      d.est_off = est_off[b];
      d.gest_off = z.nest;
      d.arc_off = z.arcs;
      d.dir_off = z.dir;
      d.doff_off = z.doff;
      d.w = w[k];
      d.r = r[b];
      d.tile_off = (uint32_t)z.tiles;
      d.ntiles = (uint32_t)((2ull * w[k] + kTile - 1) / kTile);
      d.hblk_off = (uint32_t)pl.hblks;
      d.nhblk = (d.ntiles + kHistTiles - 1) / kHistTiles;
      pl.hblks += d.nhblk;
      d.chunk_off = (uint32_t)pl.chunks;
      d.nchunks = (d.ntiles + (1u << tune.chunk_log2) - 1) >> tune.chunk_log2;
      pl.chunks += d.nchunks;
      d.dir_log2 = dir_log2_for(w[k]);
      d.need_off = (uint32_t)z.need;
      d.prow_off = z.prow;
      d.pbits = part_log2_for(r[b], tune.part_q);
      d.ptile_off = (uint32_t)pl.ptiles;
      d.ptile_log2 = ptile_log2_for(r[b], w[k], nseg);
      d.netile = ptiles_for(w[k], d.ptile_log2);
      d.nqtile = ptiles_for(r[b], d.ptile_log2);
      pl.ptiles += d.netile + d.nqtile;
      d.part_off = (uint32_t)(z.parts);
      d.pscan_off = (uint32_t)pl.pscans;
      pl.pscans += 2ull * (((1ull << d.pbits) + 63) / 64);
      d.jslices = jslices_for(w[k], d.pbits, tune.join_edges, nseg);
      d.jblk_off = (uint32_t)pl.jblks;
      pl.jblks += (uint64_t)d.jslices << d.pbits;
      add_chunk(z, r[b], w[k], tune.part_q, nseg);
      pl.segs.push_back(d);
      pl.bank.push_back(b);
    }
    z.segs = (uint32_t)pl.segs.size();
    if (z.tiles >= 0x7FFFFFFFull || z.need >= 0xFFFFFFFFull || pl.ptiles >= 0x7FFFFFFFull ||
        pl.jblks >= 0x7FFFFFFFull || z.parts >= 0x7FFFFFFFull)
      return fail(TC_EINVAL, "step too large");
    return TC_OK;
  }

  // kernel arguments of a planned step on scratch X (parity copy P)
  StepArgs make_args(const Plan& pl, const Scratch& X, const ParityScratch& P) const {
    const Sizes& z = pl.z;
    StepArgs a{};
    a.nseg = (uint32_t)pl.segs.size();
    a.segs = P.segs;
    a.seg0 = pl.segs[0];
    a.ntiles = (uint32_t)z.tiles;
    a.nhblk = (uint32_t)pl.hblks;
    a.nstep1 = (uint32_t)((z.nest + kBlock - 1) / kBlock);
    a.hpart = X.hpart;
    a.mpart = X.mpart;
    a.nest = z.nest;
    a.tagp = tagp;
    a.r1 = R1, a.r2 = R2, a.cc = CC;
    a.work = P.work;
    a.arcs[0] = X.arcs[0], a.arcs[1] = X.arcs[1];
    a.csum = X.csum;
    a.nchunk = (uint32_t)pl.chunks;
    a.dir = X.dir;
    a.doff = X.doff;
    a.prow = X.prow, a.ptot = X.ptot, a.pstart = X.pstart;
    a.erec = X.erec, a.qrec = X.qrec;
    a.nptile = (uint32_t)pl.ptiles;
    a.npscan = (uint32_t)pl.pscans;
    a.njblk = (uint32_t)pl.jblks;
    a.j1 = J1;
    a.qq = QQ;
    a.qthr = QT;
    a.need = X.need;
    a.need_bytes = z.need;
    a.inv = X.inv;
    a.err = err;
    a.id_limit = id_limit;
    a.npass = npass;
    a.dbits = dbits;
    a.chunk_log2 = tune.chunk_log2;
    a.single_chunk = dbits == 8 && pl.chunks == pl.segs.size() ? 1u : 0u;
    return a;
  }

  // Enqueue phases A, B and C of one step (C on st2 when it may overlap
  // the next step's A), then advance the banks' counters.
  int launch(const Plan& pl, const StepArgs& a, hipStream_t st, hipEvent_t* ev,
             bool overlap) {
    // A: group the batch; B: Steps 1-2, after the previous step's Step 3;
    // C: Step 3, on st2 when it may overlap the next step's A
    if (launch_phase(0, a, st, ev) != hipSuccess)
      return fail(TC_EHIP, "kernel launch failed");
    int rc = join(st);
    if (rc != TC_OK) return rc;
    if (launch_phase(1, a, st, ev) != hipSuccess)
      return fail(TC_EHIP, "kernel launch failed");
    if (overlap) {
      if (hipEventRecord(evB, st) != hipSuccess ||
          hipStreamWaitEvent(st2, evB, 0) != hipSuccess ||
          launch_phase(2, a, st2, ev) != hipSuccess ||
          hipEventRecord(evC, st2) != hipSuccess)
        return fail(TC_EHIP, "kernel launch failed");
      c_pending = true;
    } else if (launch_phase(2, a, st, ev) != hipSuccess) {
      return fail(TC_EHIP, "kernel launch failed");
    }
    for (size_t k = 0; k < pl.segs.size(); ++k) {
      m[pl.bank[k]] += pl.segs[k].w;
      batch[pl.bank[k]] += 1;
    }
    last = st;
    return TC_OK;
  }

  // reserve == true: size the scratch for this step without launching it
  // overlap == true: Step 3 runs on st2 and the next step (of the same API
  // call) waits for it before its Steps 1-2; the call's last step must not
  // overlap, so every call returns with all its work ordered on st
  int step(uint32_t nchunks, const uint32_t* ids, const uint32_t* const* edges,
           const uint32_t* w, hipStream_t st, bool reserve = false,
           bool overlap = false) {
    if (sticky != TC_OK) return fail(sticky, "an earlier batch failed on the device");
    Plan all;  // every chunk, validated
    int rc = plan(nchunks, ids, edges, w, reserve, all);
    if (rc || all.segs.empty()) return rc;
    if (reserve) return ensure_scratch(all.z, st);
    // the capture status decides before anything may synchronize, allocate
    // or free: growing the scratch under capture would do all three
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess)
      return fail(TC_EHIP, "hipStreamIsCapturing failed");
    const bool capturing = cs == hipStreamCaptureStatusActive;
    if (capturing && timing) return fail(TC_EINVAL, "kernel timing is on while capturing");
    // a step whose chunks all have at most fused_edges edges takes the
    // fused step (one launch, no scratch); any other step the chain of
    // kernels, for all its chunks (a fused launch after the chain would
    // only add to the step's time).  Under capture every step takes the
    // chain, whose descriptors have per-capture buffers.
    bool fuse = !capturing;
    for (const SegDesc& d : all.segs) fuse = fuse && d.w <= tune.fused_edges;
    std::vector<SmallDesc> small;
    std::vector<uint32_t> sbank, lid, lw;
    std::vector<const uint32_t*> led;
    uint32_t sblk = 0;
    for (size_t k = 0; k < all.segs.size(); ++k) {
      const SegDesc& d = all.segs[k];
      if (fuse) {
        small.push_back(SmallDesc{d.edges, d.m, d.batch, d.key0, d.est_off, d.w, d.r, sblk, 0});
        sbank.push_back(all.bank[k]);
        sblk += (d.r + kSmallR - 1) / kSmallR;
      } else {
        lid.push_back(all.bank[k]), led.push_back(d.edges), lw.push_back(d.w);
      }
    }
    Plan pl;
    if (!lid.empty()) {
      rc = plan((uint32_t)lid.size(), lid.data(), led.data(), lw.data(), false, pl);
      if (rc) return rc;
    }
    const bool chain = !pl.segs.empty();
    if (capturing && chain && !cap.fits(pl.z))
      return fail(TC_EINVAL, "a step being captured needs more scratch than reserved "
                             "(call tc_reserve / tc_multi_reserve before capturing)");
    StepArgs a{};
    if (chain) {
      rc = ensure_scratch(pl.z, st);
      if (rc) return rc;
      if (++steps % 0xFFFF0000ull == 0 && !capturing) {
        // directory tags are about to wrap: forget every entry (fill, not memset)
        if (join(st) || launch_fill32(reinterpret_cast<uint32_t*>(S.dir), cap.dir * 4, 0, st))
          return fail(TC_EHIP, "table reset failed");
      }
      const ParityScratch& P = S.par[steps & 1];
      a = make_args(pl, S, P);
      if (a.nseg > 1) {
        rc = stage_descs(pl.segs, P.segs, st, capturing);
        if (rc) return rc;
      }
      if (capturing) captured = true;
    }
    hipEvent_t* ev = nullptr;
    if (timing) {
      if (!ev_free.empty()) {
        ev = ev_free.back();
        ev_free.pop_back();
      } else {
        ev = new hipEvent_t[2 * kNumKernels]();
        for (int k = 0; k < kNumKernels; ++k)
          if (timing_mask >> k & 1u)
            if (hipEventCreate(&ev[2 * k]) || hipEventCreate(&ev[2 * k + 1]))
              return fail(TC_EHIP, "hipEventCreate failed");
      }
      ev_pending.push_back(ev);
      ev_launched.push_back((chain ? launched_kernels(npass, a.single_chunk != 0) : 0u) |
                            (small.empty() ? 0u : 1u << kSmallKernel));
    }
    if (chain) {
      rc = launch(pl, a, st, ev, overlap);
      if (rc) return rc;
    }
    if (!small.empty()) return launch_fused(small, sbank, sblk, st, ev, !chain);
    return TC_OK;
  }

  // The fused step of the small chunks: after the previous step's Step 3
  // (join_first: when no chain of this step has already waited for it),
  // one launch of k_small.
  int launch_fused(const std::vector<SmallDesc>& small, const std::vector<uint32_t>& sbank,
                   uint32_t nblk, hipStream_t st, hipEvent_t* ev, bool join_first) {
    if (join_first) {
      int rc = join(st);
      if (rc) return rc;
    }
    SmallArgs a{};
    a.nseg = (uint32_t)small.size();
    a.d0 = small[0];
    a.nblk = nblk;
    a.descs = sdesc;
    if (a.nseg > 1) {
      int rc = stage_bytes(small.data(), a.nseg, sizeof(SmallDesc), sdesc, st, false);
      if (rc) return rc;
    }
    a.r1 = R1, a.r2 = R2, a.cc = CC, a.err = err, a.id_limit = id_limit;
    if (launch_small(a, st, ev) != hipSuccess) return fail(TC_EHIP, "kernel launch failed");
    for (size_t k = 0; k < small.size(); ++k) {
      m[sbank[k]] += small[k].w;
      batch[sbank[k]] += 1;
    }
    last = st;
    return TC_OK;
  }

  // One batch for bank 0 with every per-step buffer carved from the
  // device's static scratch: no allocation, no free, no synchronisation.
  // Calls on one device share that scratch, so calls that overlap in time
  // on one device race (they must be ordered, e.g. on one stream).
  int step_noalloc(const uint32_t* edges, uint32_t w, hipStream_t st) {
    if (sticky != TC_OK) return fail(sticky, "an earlier batch failed on the device");
    if (nbanks != 1) return fail(TC_EINVAL, "the no-allocation step serves one bank");
    if (timing) return fail(TC_EINVAL, "kernel timing is on (its events are allocated)");
    const uint32_t id = 0;
    Plan pl;
    int rc = plan(1, &id, &edges, &w, false, pl);
    if (rc || pl.segs.empty()) return rc;
    if (!stat || !stat->ptr)
      return fail(TC_EHIP, "the static scratch of this device could not be located");
    const uint64_t bytes = carve(nullptr, pl.z, 1, true, nullptr);
    if (pl.z.dir > kStaticDirSlots || bytes > kStaticScratchBytes)
      return fail(TC_EINVAL, "batch and bank too large for the no-allocation step: they need " +
                                 std::to_string(bytes) + " bytes of scratch and " +
                                 std::to_string(pl.z.dir) + " directory slots, it holds " +
                                 std::to_string(kStaticScratchBytes) + " and " +
                                 std::to_string(kStaticDirSlots) +
                                 " (every w <= 2^18 with r <= 2^18 fits)");
    Scratch X;
    carve(stat->ptr, pl.z, 1, true, &X);
    rc = join(st);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_static_mu);
    // the directory tag lives in the scratch and advances once per step on
    // this device; before it wraps, and after a step whose launches failed
    // part-way, the directory and the work area are cleared (fill kernels)
    const bool wrap = ++stat->steps % 0xFFFF0000ull == 0;
    if (wrap || stat->dirty) {
      if (launch_fill32(reinterpret_cast<uint32_t*>(X.dir), kStaticDirSlots * 4, 0, st) ||
          launch_fill32(reinterpret_cast<uint32_t*>(X.par[0].work), sizeof(SegWork) / 4, 0, st))
        return fail(TC_EHIP, "static scratch reset failed");
      stat->dirty = false;
    }
    StepArgs a = make_args(pl, X, X.par[0]);
    a.tagp = X.tagp;
    a.j1 = X.j1, a.qq = X.qq, a.qthr = X.qthr;
    rc = launch(pl, a, st, nullptr, false);
    if (rc) stat->dirty = true;
    return rc;
  }

  // device bytes this object holds now (as requested from hipMalloc)
  uint64_t device_bytes() const {
    uint64_t b = kBankBytesPerEst * total + 8ull * (nbanks + 1) + 8ull * nbanks + 8 +
                 8ull * cap_groups;
    if (block) b += carve(nullptr, cap, 2, false, nullptr);
    return b + retired_bytes + 16ull * hbuf_w;
  }

  // A stream in host memory: batch k is copied into staging buffer k & 1 on
  // the copy stream (after that buffer's previous batch is done with it)
  // while batch k - 1 is processed on st; each step waits for its copy.
  int host_stream(const uint32_t* host, uint64_t mm, uint32_t w, hipStream_t st) {
    if (sticky != TC_OK) return fail(sticky, "an earlier batch failed on the device");
    if (nbanks != 1) return fail(TC_EINVAL, "host ingest serves one bank");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess)
      return fail(TC_EHIP, "hipStreamIsCapturing failed");
    if (cs == hipStreamCaptureStatusActive)
      return fail(TC_EINVAL, "host ingest cannot be captured (it copies from host memory)");
    const uint64_t need_w = std::min<uint64_t>(w, mm);
    if (!stc && hipStreamCreateWithFlags(&stc, hipStreamNonBlocking) != hipSuccess)
      return fail(TC_EHIP, "copy stream creation failed");
    for (int b = 0; b < 2; ++b)
      if ((!h_ready[b] && hipEventCreateWithFlags(&h_ready[b], hipEventDisableTiming)) ||
          (!h_free[b] && hipEventCreateWithFlags(&h_free[b], hipEventDisableTiming)))
        return fail(TC_EHIP, "hipEventCreate failed");
    if (need_w > hbuf_w) {
      // the old buffers may still be read by enqueued steps
      wait_all();
      if (st) (void)hipStreamSynchronize(st);
      (void)hipStreamSynchronize(stc);
      for (int b = 0; b < 2; ++b) {
        dfree(hbuf[b]);
        h_used[b] = false;
      }
      hbuf_w = 0;
      if (dalloc(&hbuf[0], 2 * need_w) || dalloc(&hbuf[1], 2 * need_w)) {
        dfree(hbuf[0]), dfree(hbuf[1]);
        return fail(TC_ENOMEM, "device staging buffers for host ingest");
      }
      hbuf_w = need_w;
    }
    const uint32_t id = 0;
    uint64_t k = 0;
    for (uint64_t j = 0; j < mm; j += w, ++k) {
      const int b = (int)(k & 1);
      const uint32_t wk = (uint32_t)std::min<uint64_t>(w, mm - j);
      if ((h_used[b] && hipStreamWaitEvent(stc, h_free[b], 0) != hipSuccess) ||
          hipMemcpyAsync(hbuf[b], host + 2 * j, 8ull * wk, hipMemcpyHostToDevice, stc) !=
              hipSuccess ||
          hipEventRecord(h_ready[b], stc) != hipSuccess ||
          hipStreamWaitEvent(st, h_ready[b], 0) != hipSuccess) {
        (void)join(st);
        return fail(TC_EHIP, "host-to-device copy of a batch failed");
      }
      // Step 3 of a batch may overlap the next batch's grouping (as in
      // tc_process_stream); its last reader of the buffer is then on st2
      const bool more = j + w < mm;
      const uint32_t* ek = hbuf[b];
      int rc = step(1, &id, &ek, &wk, st, false, more);
      if (rc) {
        (void)join(st);
        return rc;
      }
      if (hipEventRecord(h_free[b], c_pending ? st2 : st) != hipSuccess) {
        (void)join(st);
        return fail(TC_EHIP, "hipEventRecord failed");
      }
      h_used[b] = true;
    }
    return TC_OK;
  }

  // one batch for bank b by the per-estimator kernel (same state, same draws)
  int step_naive(uint32_t b, const uint32_t* edges, uint32_t w, hipStream_t st) {
    if (sticky != TC_OK) return fail(sticky, "an earlier batch failed on the device");
    if (w > TC_MAX_BATCH) return fail(TC_EINVAL, "batch larger than TC_MAX_BATCH");
    if (w == 0) return TC_OK;
    if (!edges) return fail(TC_EINVAL, "null edge pointer with w > 0");
    if (reinterpret_cast<uintptr_t>(edges) & 7u)
      return fail(TC_EINVAL, "edge buffer must be 8-byte aligned");
    NaiveArgs a{};
    a.edges = edges;
    a.w = w;
    a.r = r[b];
    a.m = m[b];
    a.batch = batch[b];
    a.key0 = key0[b];
    a.est_off = est_off[b];
    a.r1 = R1, a.r2 = R2, a.cc = CC, a.err = err;
    if (join(st) || launch_naive(a, st) != hipSuccess)
      return fail(TC_EHIP, "kernel launch failed");
    m[b] += w;
    batch[b] += 1;
    last = st;
    return TC_OK;
  }

  // every bank back to empty, |E| = 0, batch 0 (fill kernels only, so a
  // reset can be captured into a graph ahead of captured steps)
  int reset(hipStream_t st) {
    if (join(st) || launch_fill64(R1, total, kEmpty, st) ||
        launch_fill64(R2, total, kEmpty, st) || launch_fill32(CC, total, 0, st))
      return fail(TC_EHIP, "bank reset failed");
    std::fill(m.begin(), m.end(), 0);
    std::fill(batch.begin(), batch.end(), 0);
    last = st;
    return TC_OK;
  }

  // bank b starts over as an empty bank with a new seed (kernels only)
  int assign(uint32_t b, uint64_t new_seed, hipStream_t st) {
    const uint64_t off = est_off[b], n = r[b];
    if (join(st) || launch_fill64(R1 + off, n, kEmpty, st) ||
        launch_fill64(R2 + off, n, kEmpty, st) || launch_fill32(CC + off, n, 0, st))
      return fail(TC_EHIP, "bank reset failed");
    seed[b] = new_seed;
    key0[b] = host_mix64(new_seed ^ kGolden);
    m[b] = 0;
    batch[b] = 0;
    last = st;
    return TC_OK;
  }

  // every vertex id is below n (2 <= n <= 2^32): the radix passes above
  // the top digit of n - 1 are not launched.  Ids of 17 to 20 bits take
  // two passes of 10-bit digits instead of three of 8.
  int set_bound(uint64_t n) {
    if (n < 2 || n > (1ull << 32)) return fail(TC_EINVAL, "vertex bound must be in [2, 2^32]");
    id_limit = (uint32_t)(n - 1);
    digits();
    return TC_OK;
  }

  // digit width and passes for the declared bound (and the tuning)
  void digits() {
    const uint32_t bits = 32u - (uint32_t)__builtin_clz(id_limit | 1u);
    const bool wide = !tune.digits8 && bits > 16 && bits <= (uint32_t)(kWidePasses * kWideBits);
    dbits = wide ? (uint32_t)kWideBits : 8u;
    npass = (bits + dbits - 1) / dbits;
  }

  int set_tuning(const Tuning& t) {
    auto pow2 = [](uint32_t x) { return x && !(x & (x - 1)); };
    if (t.digits8 > 1 || t.chunk_log2 < kMinChunkLog2 || (1u << t.chunk_log2) > kChunk ||
        !pow2(t.part_q) || t.part_q < kMinPartQ || t.part_q > 8192 || !pow2(t.join_edges) ||
        t.join_edges < 1024 || t.join_edges > 65536 || t.fused_edges > kSmallW)
      return fail(TC_EINVAL, "tuning out of range");
    tune = t;
    digits();
    return TC_OK;
  }

  int graph_reserve(uint32_t nsteps) {
    // outstanding eager work is finished, so a capture starts from a state
    // that depends on no event recorded outside it
    wait_all();
    c_pending = false;
    // graphs captured before are void from here on: the scratch blocks
    // they referred to can go
    free_retired();
    captured = false;
    for (SegDesc* g : graph_stage) (void)hipHostFree(g);
    graph_stage.assign(nsteps, nullptr);
    graph_next = 0;
    for (uint32_t i = 0; i < nsteps; ++i)
      if (hipHostMalloc(reinterpret_cast<void**>(&graph_stage[i]),
                        sizeof(SegDesc) * nbanks))
        return fail(TC_ENOMEM, "pinned descriptor staging failed");
    return TC_OK;
  }

  int sync() {
    if (last && hipStreamSynchronize(last) != hipSuccess)
      return fail(TC_EHIP, "hipStreamSynchronize failed");
    if (st2 && hipStreamSynchronize(st2) != hipSuccess)
      return fail(TC_EHIP, "hipStreamSynchronize failed");
    if (hipMemcpy(h_err, err, 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(TC_EHIP, "reading the device error word failed");
    const uint32_t e = *h_err;
    if (e & kErrRange) sticky = TC_EINVAL;
    else if (e & kErrSelfLoop) sticky = TC_EBADEDGE;
    else if (e & kErrOverflow) sticky = TC_EOVERFLOW;
    else if (e & (kErrProbe | kErrIndex)) sticky = TC_EHIP;
    if (sticky == TC_EINVAL)
      return fail(sticky, "a batch contained a vertex id at or above the declared bound");
    if (sticky == TC_EBADEDGE) return fail(sticky, "a batch contained a self-loop");
    if (sticky == TC_EOVERFLOW) return fail(sticky, "an adjacency count reached 2^31");
    if (sticky != TC_OK) return fail(sticky, "a device table or wait ran past its bound");
    return TC_OK;
  }

  // accumulate the elapsed time of every pending timed step
  int collect_times() {
    for (size_t i = 0; i < ev_pending.size(); ++i) {
      hipEvent_t* e = ev_pending[i];
      for (int k = 0; k < kNumKernels; ++k) {
        if (!e[2 * k] || !(ev_launched[i] >> k & 1u)) continue;
        float ms = 0;
        if (hipEventSynchronize(e[2 * k + 1]) ||
            hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]))
          return fail(TC_EHIP, "event timing failed");
        kernel_ms[k] += ms;
      }
      ++timed_steps;
      ev_free.push_back(e);
    }
    ev_pending.clear();
    ev_launched.clear();
    return TC_OK;
  }

  int sums_all(uint64_t* S) {
    int rc = sync();
    if (rc) return rc;
    hipStream_t st = last;
    if (launch_gsum(CC, 0, total, bank_off, nbanks, 0, sums, st) != hipSuccess ||
        hipMemcpyAsync(h_sums, sums, sizeof(uint64_t) * nbanks,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(TC_EHIP, "estimate reduction failed");
    for (uint32_t b = 0; b < nbanks; ++b) S[b] = h_sums[b];
    return TC_OK;
  }

  // median-of-means over g contiguous groups of bank b (group sums on the
  // device, the g means and their median on the host, in double)
  int mom(uint32_t b, uint32_t g, double* tau, uint64_t* group_sums) {
    if (g == 0 || g > r[b]) return fail(TC_EINVAL, "groups must be in [1, r]");
    int rc = sync();
    if (rc) return rc;
    if (g > cap_groups) {
      dfree(gsums);
      if (h_gsums) (void)hipHostFree(h_gsums);
      h_gsums = nullptr;
      cap_groups = 0;
      if (dalloc(&gsums, g) ||
          hipHostMalloc(reinterpret_cast<void**>(&h_gsums), sizeof(uint64_t) * g))
        return fail(TC_ENOMEM, "group-sum buffers");
      cap_groups = g;
    }
    hipStream_t st = last;
    if (launch_gsum(CC, est_off[b], r[b], nullptr, 0, g, gsums, st) != hipSuccess ||
        hipMemcpyAsync(h_gsums, gsums, sizeof(uint64_t) * g, hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(TC_EHIP, "group-sum reduction failed");
    std::vector<double> mean(g);
    for (uint32_t k = 0; k < g; ++k) {
      const uint64_t lo = (uint64_t)k * r[b] / g, hi = (uint64_t)(k + 1) * r[b] / g;
      mean[k] = (double)h_gsums[k] * (double)m[b] / (double)(hi - lo);
      if (group_sums) group_sums[k] = h_gsums[k];
    }
    std::sort(mean.begin(), mean.end());
    if (tau) *tau = (g & 1u) ? mean[g / 2] : 0.5 * (mean[g / 2 - 1] + mean[g / 2]);
    return TC_OK;
  }

  int read_bank(uint32_t b, uint64_t* r1, uint64_t* r2, uint32_t* c,
                uint8_t* closed) {
    int rc = sync();
    if (rc) return rc;
    const uint64_t off = est_off[b], n = r[b];
    if (r1 && hipMemcpy(r1, R1 + off, n * 8, hipMemcpyDeviceToHost))
      return fail(TC_EHIP, "state copy failed");
    if (r2 && hipMemcpy(r2, R2 + off, n * 8, hipMemcpyDeviceToHost))
      return fail(TC_EHIP, "state copy failed");
    if (c || closed) {
      std::vector<uint32_t> cc(n);
      if (hipMemcpy(cc.data(), CC + off, n * 4, hipMemcpyDeviceToHost))
        return fail(TC_EHIP, "state copy failed");
      for (uint64_t i = 0; i < n; ++i) {
        if (c) c[i] = cc[i] & kChiMax;
        if (closed) closed[i] = (cc[i] & kClosed) ? 1 : 0;
      }
    }
    return TC_OK;
  }
};

}  // namespace

namespace tc {
// error text for the entry points defined in other files
int report(int code, const char* msg) { return fail(code, msg); }
}  // namespace tc

struct tc_multi {
  Engine e;
};
struct tc_state {
  Engine e;
};

extern "C" {

const char* tc_last_error(void) { return g_err.c_str(); }

// ---- single bank ----------------------------------------------------------
tc_state* tc_create(uint32_t r, uint64_t seed) {
  if (r == 0) {
    fail(TC_EINVAL, "r must be >= 1");
    return nullptr;
  }
  tc_state* s = new (std::nothrow) tc_state;
  if (!s) {
    fail(TC_ENOMEM, "host allocation failed");
    return nullptr;
  }
  if (s->e.init(1, &r, &seed) != TC_OK) {
    delete s;
    return nullptr;
  }
  return s;
}

int tc_process_batch(tc_state* s, const uint32_t* edges, uint32_t w,
                     void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  const uint32_t id = 0;
  return s->e.step(1, &id, &edges, &w, static_cast<hipStream_t>(stream));
}

int tc_process_batch_noalloc(tc_state* s, const uint32_t* edges, uint32_t w,
                             void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.step_noalloc(edges, w, static_cast<hipStream_t>(stream));
}

int tc_process_batch_naive(tc_state* s, const uint32_t* edges, uint32_t w,
                           void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.step_naive(0, edges, w, static_cast<hipStream_t>(stream));
}

int tc_process_stream(tc_state* s, const uint32_t* edges, uint64_t m,
                      uint32_t w, void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  if (w == 0 || w > TC_MAX_BATCH) return fail(TC_EINVAL, "w must be in [1, TC_MAX_BATCH]");
  if (m == 0) return TC_OK;
  if (!edges) return fail(TC_EINVAL, "null edge pointer with m > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t id = 0;
  for (uint64_t j = 0; j < m; j += w) {
    const uint32_t wk = (uint32_t)std::min<uint64_t>(w, m - j);
    const uint32_t* ek = edges + 2 * j;
    // Step 3 of a batch overlaps the grouping of the next (the join's
    // probes are bound by LDS latency, the grouping by HBM bandwidth)
    const bool more = j + w < m;
    int rc = s->e.step(1, &id, &ek, &wk, st, false, more);
    if (rc) {
      (void)s->e.join(st);
      return rc;
    }
  }
  return TC_OK;
}

int tc_process_host_stream(tc_state* s, const uint32_t* host_edges, uint64_t m,
                           uint32_t w, void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  if (w == 0 || w > TC_MAX_BATCH) return fail(TC_EINVAL, "w must be in [1, TC_MAX_BATCH]");
  if (m == 0) return TC_OK;
  if (!host_edges) return fail(TC_EINVAL, "null edge pointer with m > 0");
  return s->e.host_stream(host_edges, m, w, static_cast<hipStream_t>(stream));
}

uint64_t tc_step_bytes_max(uint32_t nchunks, uint32_t r_max, uint64_t total_w) {
  if (nchunks == 0 || total_w == 0 || r_max == 0) return 0;
  return carve(nullptr, step_bound(nchunks, r_max, total_w), 2, false, nullptr);
}

int tc_multi_reserve_max(tc_multi* s, uint32_t nchunks, uint64_t total_w) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (nchunks == 0 || total_w == 0) return TC_OK;
  if (nchunks > s->e.nbanks) return fail(TC_EINVAL, "more chunks than banks");
  const uint32_t r_max = *std::max_element(s->e.r.begin(), s->e.r.end());
  return s->e.ensure_scratch(step_bound(nchunks, r_max, total_w), nullptr);
}

uint64_t tc_bank_bytes(uint32_t r) {
  // one bank's share of the per-bank words (offset, sum) included
  return kBankBytesPerEst * r + 16;
}

uint64_t tc_step_bytes(uint32_t nchunks, const uint32_t* r, const uint32_t* w) {
  if (nchunks && (!r || !w)) return 0;
  Sizes z;
  uint32_t nseg = 0;
  for (uint32_t k = 0; k < nchunks; ++k) {
    if (w[k] > TC_MAX_BATCH || r[k] == 0) return 0;
    nseg += w[k] != 0;
  }
  for (uint32_t k = 0; k < nchunks; ++k)
    if (w[k]) add_chunk(z, r[k], w[k], kPartQ, nseg);
  return z.segs ? carve(nullptr, z, 2, false, nullptr) : 0;
}

int tc_device_bytes(const tc_state* s, uint64_t* bytes) {
  if (!s || !bytes) return fail(TC_EINVAL, "null argument");
  *bytes = s->e.device_bytes();
  return TC_OK;
}

int tc_multi_device_bytes(const tc_multi* s, uint64_t* bytes) {
  if (!s || !bytes) return fail(TC_EINVAL, "null argument");
  *bytes = s->e.device_bytes();
  return TC_OK;
}

static int set_tuning_from(Engine& e, const tc_tuning* t) {
  if (!t) return fail(TC_EINVAL, "null tuning");
  Tuning u;
  if (t->digit_bits != 0 && t->digit_bits != 8) return fail(TC_EINVAL, "digit_bits must be 0 or 8");
  u.digits8 = t->digit_bits == 8 ? 1u : 0u;
  u.chunk_log2 = t->chunk_tiles ? (uint32_t)__builtin_ctz(t->chunk_tiles) : 0u;
  if (t->chunk_tiles == 0 || (t->chunk_tiles & (t->chunk_tiles - 1)))
    return fail(TC_EINVAL, "chunk_tiles must be 8, 16 or 32");
  u.part_q = t->part_estimators;
  u.join_edges = t->join_edges;
  u.fused_edges = t->fused_edges;
  return e.set_tuning(u);
}

static void get_tuning_from(const Engine& e, tc_tuning* t) {
  t->digit_bits = e.tune.digits8 ? 8u : 0u;
  t->chunk_tiles = 1u << e.tune.chunk_log2;
  t->part_estimators = e.tune.part_q;
  t->join_edges = e.tune.join_edges;
  t->fused_edges = e.tune.fused_edges;
}

int tc_set_tuning(tc_state* s, const tc_tuning* t) {
  if (!s) return fail(TC_EINVAL, "null state");
  return set_tuning_from(s->e, t);
}

int tc_multi_set_tuning(tc_multi* s, const tc_tuning* t) {
  if (!s) return fail(TC_EINVAL, "null object");
  return set_tuning_from(s->e, t);
}

int tc_get_tuning(const tc_state* s, tc_tuning* t) {
  if (!s || !t) return fail(TC_EINVAL, "null argument");
  get_tuning_from(s->e, t);
  return TC_OK;
}

int tc_multi_get_tuning(const tc_multi* s, tc_tuning* t) {
  if (!s || !t) return fail(TC_EINVAL, "null argument");
  get_tuning_from(s->e, t);
  return TC_OK;
}

int tc_set_vertex_bound(tc_state* s, uint64_t n) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.set_bound(n);
}

int tc_estimate_mom(tc_state* s, uint32_t groups, double* tau, uint64_t* group_sums) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.mom(0, groups, tau, group_sums);
}

uint64_t tc_estimators_needed(double eps, double delta, uint64_t m, uint64_t maxdeg,
                              double tau) {
  if (!(eps > 0.0) || !(delta > 0.0 && delta < 1.0) || !(tau > 0.0)) return 0;
  const double r = 96.0 / (eps * eps) * (double)m * (double)maxdeg / tau * std::log(1.0 / delta);
  return (uint64_t)std::ceil(r);
}

int tc_reserve(tc_state* s, uint32_t max_w) {
  if (!s) return fail(TC_EINVAL, "null state");
  const uint32_t id = 0;
  const uint32_t* none = nullptr;
  return s->e.step(1, &id, &none, &max_w, nullptr, true);
}

int tc_reset(tc_state* s, void* stream) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.reset(static_cast<hipStream_t>(stream));
}

int tc_estimate_ex(tc_state* s, uint64_t* S, uint64_t* m, double* tau) {
  if (!s) return fail(TC_EINVAL, "null state");
  uint64_t sum = 0;
  int rc = s->e.sums_all(&sum);
  if (rc) return rc;
  if (S) *S = sum;
  if (m) *m = s->e.m[0];
  if (tau) *tau = (double)sum * (double)s->e.m[0] / (double)s->e.r[0];
  return TC_OK;
}

double tc_estimate(tc_state* s) {
  double tau = NAN;
  if (tc_estimate_ex(s, nullptr, nullptr, &tau) != TC_OK) return NAN;
  return tau;
}

int tc_read_state(tc_state* s, uint64_t* r1, uint64_t* r2, uint32_t* c,
                  uint8_t* closed) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.read_bank(0, r1, r2, c, closed);
}

int tc_sync(tc_state* s) {
  if (!s) return fail(TC_EINVAL, "null state");
  return s->e.sync();
}

static const char* const kKernelNames[kNumKernels] = {
    "k_hist", "k_fold_step1", "k_cscan<0>", "k_scat<0>",
    "k_cnt<1>", "k_csum<1>", "k_cscan<1>", "k_scat<1>",
    "k_cnt<2>", "k_csum<2>", "k_cscan<2>", "k_scat<2>",
    "k_cnt<3>", "k_csum<3>", "k_cscan<3>", "k_scat<3>",
    "k_dir", "k_est", "k_pcnt", "k_pscan", "k_pscat", "k_pjoin", "k_small"};

static int set_timing(Engine& e, uint32_t mask) {
  int rc = e.collect_times();
  if (rc) return rc;
  mask &= (1u << kNumKernels) - 1u;
  if (mask != e.timing_mask) {
    // event sets are made for one mask
    for (hipEvent_t* ev : e.ev_free) {
      for (int k = 0; k < 2 * kNumKernels; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
      delete[] ev;
    }
    e.ev_free.clear();
  }
  e.timing_mask = mask;
  e.timing = mask != 0;
  for (double& v : e.kernel_ms) v = 0;
  e.timed_steps = 0;
  return TC_OK;
}

static int read_times(Engine& e, double* ms, uint64_t* steps) {
  int rc = e.collect_times();
  if (rc) return rc;
  for (int k = 0; k < kNumKernels; ++k)
    if (ms) ms[k] = e.kernel_ms[k];
  if (steps) *steps = e.timed_steps;
  return TC_OK;
}

int tc_set_kernel_timing(tc_state* s, uint32_t mask) {
  if (!s) return fail(TC_EINVAL, "null state");
  return set_timing(s->e, mask);
}

int tc_kernel_times(tc_state* s, double* ms, uint64_t* steps) {
  if (!s) return fail(TC_EINVAL, "null state");
  return read_times(s->e, ms, steps);
}

int tc_multi_set_kernel_timing(tc_multi* s, uint32_t mask) {
  if (!s) return fail(TC_EINVAL, "null object");
  return set_timing(s->e, mask);
}

int tc_multi_kernel_times(tc_multi* s, double* ms, uint64_t* steps) {
  if (!s) return fail(TC_EINVAL, "null object");
  return read_times(s->e, ms, steps);
}

int tc_num_kernels(void) { return kNumKernels; }

const char* tc_kernel_name(int k) {
  return (k >= 0 && k < kNumKernels) ? kKernelNames[k] : "";
}

uint32_t tc_num_estimators(const tc_state* s) { return s ? s->e.r[0] : 0; }
uint64_t tc_edges_seen(const tc_state* s) { return s ? s->e.m[0] : 0; }
uint64_t tc_batches_seen(const tc_state* s) { return s ? s->e.batch[0] : 0; }

void tc_destroy(tc_state* s) { delete s; }

// ---- many banks -----------------------------------------------------------
tc_multi* tc_multi_create(uint32_t nbanks, const uint32_t* r,
                          const uint64_t* seeds) {
  if (nbanks == 0 || !r || !seeds) {
    fail(TC_EINVAL, "need nbanks >= 1 and non-null r, seeds");
    return nullptr;
  }
  tc_multi* s = new (std::nothrow) tc_multi;
  if (!s) {
    fail(TC_ENOMEM, "host allocation failed");
    return nullptr;
  }
  if (s->e.init(nbanks, r, seeds) != TC_OK) {
    delete s;
    return nullptr;
  }
  return s;
}

int tc_multi_process(tc_multi* s, uint32_t nchunks, const uint32_t* bank_ids,
                     const uint32_t* const* edges, const uint32_t* w,
                     void* stream) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (nchunks == 0) return TC_OK;
  if (!bank_ids || !edges || !w) return fail(TC_EINVAL, "null chunk arrays");
  return s->e.step(nchunks, bank_ids, edges, w, static_cast<hipStream_t>(stream));
}

int tc_multi_reserve(tc_multi* s, uint32_t nchunks, const uint32_t* bank_ids,
                     const uint32_t* w) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (nchunks == 0) return TC_OK;
  if (!bank_ids || !w) return fail(TC_EINVAL, "null chunk arrays");
  std::vector<const uint32_t*> none(nchunks, nullptr);
  return s->e.step(nchunks, bank_ids, none.data(), w, nullptr, true);
}

int tc_multi_reset(tc_multi* s, void* stream) {
  if (!s) return fail(TC_EINVAL, "null object");
  return s->e.reset(static_cast<hipStream_t>(stream));
}

int tc_multi_assign(tc_multi* s, uint32_t bank, uint64_t seed, void* stream) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (bank >= s->e.nbanks) return fail(TC_EINVAL, "bank id out of range");
  return s->e.assign(bank, seed, static_cast<hipStream_t>(stream));
}

int tc_multi_estimate_mom(tc_multi* s, uint32_t bank, uint32_t groups, double* tau,
                          uint64_t* group_sums) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (bank >= s->e.nbanks) return fail(TC_EINVAL, "bank id out of range");
  return s->e.mom(bank, groups, tau, group_sums);
}

int tc_multi_set_vertex_bound(tc_multi* s, uint64_t n) {
  if (!s) return fail(TC_EINVAL, "null object");
  return s->e.set_bound(n);
}

int tc_multi_graph_reserve(tc_multi* s, uint32_t nsteps) {
  if (!s) return fail(TC_EINVAL, "null object");
  return s->e.graph_reserve(nsteps);
}

int tc_multi_estimate(tc_multi* s, uint64_t* S, uint64_t* m, double* tau) {
  if (!s) return fail(TC_EINVAL, "null object");
  std::vector<uint64_t> sums(s->e.nbanks);
  int rc = s->e.sums_all(sums.data());
  if (rc) return rc;
  for (uint32_t b = 0; b < s->e.nbanks; ++b) {
    if (S) S[b] = sums[b];
    if (m) m[b] = s->e.m[b];
    if (tau) tau[b] = (double)sums[b] * (double)s->e.m[b] / (double)s->e.r[b];
  }
  return TC_OK;
}

int tc_multi_read_state(tc_multi* s, uint32_t bank, uint64_t* r1, uint64_t* r2,
                        uint32_t* c, uint8_t* closed) {
  if (!s) return fail(TC_EINVAL, "null object");
  if (bank >= s->e.nbanks) return fail(TC_EINVAL, "bank id out of range");
  return s->e.read_bank(bank, r1, r2, c, closed);
}

int tc_multi_sync(tc_multi* s) {
  if (!s) return fail(TC_EINVAL, "null object");
  return s->e.sync();
}

uint32_t tc_multi_num_banks(const tc_multi* s) { return s ? s->e.nbanks : 0; }

void tc_multi_destroy(tc_multi* s) { delete s; }

}  // extern "C"
