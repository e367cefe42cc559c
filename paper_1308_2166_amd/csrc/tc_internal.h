// Internal layout shared by the kernels and the host side of libtc.
//
// One "step" advances one or more banks by one batch each.  Every chunk of a
// step is a segment; all per-step scratch is carved into per-segment regions
// so one set of launches serves the plain (one segment) and the batched
// (many segments) forms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr uint64_t kEmpty = ~0ull;      // empty edge code
constexpr uint32_t kNone = 0xFFFFFFFFu;  // no index
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// radix sort of the 2w arcs by vertex id, in passes of D-bit digits: D = 8
// (up to four passes), or D = 10 when a declared vertex bound above 2^16
// leaves at most 20 bits (two passes instead of three)
constexpr int kBlock = 256;              // threads per block
constexpr int kWaves = kBlock / 64;      // wave64
constexpr int kItems = 16;               // arcs per thread per tile
constexpr int kTile = kBlock * kItems;   // 4096 arcs per tile
constexpr int kPasses = 4;               // passes of 8-bit digits
constexpr int kWideBits = 10;            // the wide digit
constexpr int kWidePasses = 2;           // passes of wide digits
// words of one tile's (or chunk's, or segment's) digit counts over all
// passes: pass P's counts start at word P << D
constexpr int kRowWords = kWidePasses << kWideBits;
static_assert(kRowWords >= kPasses << 8, "a row holds every 8-bit pass");
constexpr int kNumKernels = 23;  // kernels of a step (k_hist .. k_pjoin, k_small)
constexpr int kSmallKernel = 22; // k_small's index (the fused step of small chunks)
constexpr int kHistTiles = 1;   // tiles per k_hist block (one: its counts are
                                // the per-tile counts of the first radix pass)
constexpr uint32_t kChunk = 32;  // most tiles per chunk of the radix scans (and
                                 // k_hist rows summed per k_fold block); a
                                 // step uses 2^chunk_log2 <= kChunk of them

// j1[] word: kNone, or the replacement position with kSideV set when the
// smaller endpoint u of W[j1] is its second vertex
constexpr uint32_t kSideV = 0x40000000u;
constexpr uint32_t kPosMask = 0x3FFFFFFFu;

// low word of a sorted arc: arc id (2 pos + side) and, in bit 31, a flag
// marking arcs of positions Step 1 takes an f1 from (ids stay below 2^29)
constexpr uint32_t kNeedFlag = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

// packed estimator word: chi in bits 0..30, closed flag in bit 31
constexpr uint32_t kClosed = 0x80000000u;
constexpr uint32_t kChiMax = 0x7FFFFFFFu;

// tagged directory: a slot is live only if its tag equals the step's tag

// sticky device error bits
constexpr uint32_t kErrSelfLoop = 1u;
constexpr uint32_t kErrOverflow = 2u;
constexpr uint32_t kErrProbe = 4u;  // a table probe ran past its bound
constexpr uint32_t kErrIndex = 8u;  // an index that no valid step produces
                                    // (guards against corrupt scratch)
constexpr uint32_t kErrRange = 16u;  // a vertex id above the declared bound
// errors after which the rest of a step must not trust its scratch
constexpr uint32_t kErrFatal = kErrSelfLoop | kErrIndex | kErrRange;

// one chunk of a step (device view)
struct SegDesc {
  const uint32_t* edges;  // W: uint32[2w], device
  uint64_t m;             // bank's |E| before this batch
  uint64_t batch;         // bank's batch index (random key)
  uint64_t key0;          // mix64(seed ^ golden), precomputed on the host
  uint64_t est_off;       // bank's first estimator in the state arrays
  uint64_t gest_off;      // first flat estimator thread of this segment
  uint64_t arc_off;       // first arc slot in the arc buffers (2 * sum w)
  uint64_t dir_off;       // first directory slot (hashed directory)
  uint64_t doff_off;      // first word of the dense offsets (dense directory)
  uint32_t w;             // edges in the chunk
  uint32_t r;             // estimators in the bank
  uint32_t tile_off;      // first global tile of the segment
  uint32_t ntiles;        // ceil(2w / kTile)
  uint32_t hblk_off;      // first k_hist block of the segment
  uint32_t nhblk;         // ceil(ntiles / kHistTiles)
  uint32_t chunk_off;     // first global radix chunk of the segment
  uint32_t nchunks;       // ceil(ntiles / 2^chunk_log2)
  uint32_t dir_log2;      // log2 of the directory region (slots)
  uint32_t need_off;      // first byte of the "position needed" bytes (w bytes)
  // Step 3 (partitioned join): the segment's edges and waiting estimators
  // go to 2^pbits partitions; k_pcnt / k_pscat blocks take partition tiles
  // (netile of edges, then nqtile of estimators), k_pscan blocks 64
  // partitions of one side, k_pjoin blocks one slice of one partition
  uint64_t prow_off;      // first word of the segment's partition-count rows
  uint32_t pbits;         // log2 of the partitions
  uint32_t ptile_off;     // first partition tile (global)
  uint32_t ptile_log2;    // log2 of the elements per partition tile
  uint32_t netile;        // edge tiles: ceil(w / 2^ptile_log2)
  uint32_t nqtile;        // estimator tiles: ceil(r / 2^ptile_log2)
  uint32_t part_off;      // first partition (global)
  uint32_t pscan_off;     // first k_pscan block (global)
  uint32_t jslices;       // k_pjoin blocks per partition
  uint32_t jblk_off;      // first k_pjoin block (global)
};

// per-segment values produced during a step (device)
struct SegWork {
  uint32_t hist[kRowWords];         // digit histograms of the 2w arcs
                                    // (pass P at word P << D)
  uint32_t maxid;                   // largest vertex id in the chunk
  uint32_t final_buf;               // arc buffer holding the sorted arcs
  uint32_t dense;                   // directory indexed by vertex id
  uint32_t pad;
};

// Vertex directory.  Dense (the segment's largest id below 2^dir_log2):
// CSR offsets, word x = the first sorted arc of a vertex >= x, for every x
// up to max id + 1, all rewritten every step, so vertex x's arcs are
// [off[x], off[x + 1]).  Hashed (any 32-bit ids): DirSlot, segment
// [start, end) of vertex `key` in the sorted arcs, live iff tag == step tag.
// Words of a dense region: its slot count plus room for the end word.
constexpr uint32_t kDoffPad = 64;
struct DirSlot {
  uint32_t key;
  uint32_t tag;
  uint32_t start;
  uint32_t end;
};

// Step 3 (Sec. 4.4) as a partitioned hash join.  Every waiting
// estimator's closing edge q and every batch edge are sent by the top
// pbits bits of h = mix64(q) (a bijection) to one of 2^pbits partitions,
// as 8-byte records (top 32 bits of h) << 32 | (batch position, or the
// estimator's state index), grouped by partition by a count / scan /
// scatter over tiles of up to kPTile elements.  One join block per slice of a
// partition loads the partition's waiting estimators into an LDS hash
// table (rounds of kJoinQ) and streams the slice's edges through it; equal
// high words are checked against the edge itself and the estimator's
// closing edge and position limit.
constexpr uint32_t kPTile = 16384;     // most elements per partition tile (the
                                       // scatter stages a tile in LDS)
constexpr uint32_t kMinPTileLog2 = 10; // fewest: small steps get more tiles
constexpr uint32_t kPartQ = 2048;      // estimators per partition aimed at
constexpr uint32_t kMaxPartLog2 = 11;  // at most 2048 partitions per segment
constexpr uint32_t kJoinQ = 4096;      // query records per join round (LDS)
constexpr uint32_t kJoinSlots = 8192;  // LDS hash slots (load <= 1/2)
constexpr uint32_t kJoinEdges = 8192;  // edges per join slice aimed at

struct StepArgs {
  const SegDesc* segs;    // device copy of all segment descriptors
  SegDesc seg0;           // inline copy when nseg == 1
  uint32_t nseg;
  uint32_t ntiles;        // total tiles over segments
  uint32_t nhblk;         // total k_hist blocks over segments
  uint32_t nstep1;        // k_step1 blocks (run in the k_fold launch)
  uint32_t* hpart;        // per tile: kRowWords digit counts (pass P at P << D)
  uint32_t* mpart;        // per k_hist block: largest vertex id
  uint64_t nest;          // total estimator threads over segments
  uint32_t* tagp;         // device word: this step's directory tag (never 0);
                          // advanced by the step's last kernel
  // estimator state (all banks)
  uint64_t* r1;
  uint64_t* r2;
  uint32_t* cc;
  // scratch
  SegWork* work;          // [nseg]
  uint64_t* arcs[2];      // ping-pong arc buffers
  uint32_t* csum;         // per radix chunk: kRowWords digit sums
  uint32_t nchunk;        // total radix chunks over segments
  DirSlot* dir;
  uint32_t* doff;         // dense directories (CSR offsets)
  // Step-3 join: per partition tile a row of 2^pbits counts (then in-side
  // prefixes); per global partition g and side s (0 edges, 1 estimators)
  // the total ptot[2g + s] and the start pstart[2g + s] of its records
  uint32_t* prow;
  uint32_t* ptot;
  uint32_t* pstart;
  uint64_t* erec;         // edge records, a segment's at arc_off / 2
  uint64_t* qrec;         // estimator records, a segment's at gest_off
  uint32_t nptile;        // partition tiles over segments
  uint32_t npscan;        // k_pscan blocks over segments
  uint32_t njblk;         // k_pjoin blocks over segments
  uint32_t* j1;           // per estimator: Step-1 replacement (see kSideV)
  uint64_t* qq;           // per estimator: closing edge it waits for, or kEmpty
  uint32_t* qthr;         // per estimator: first batch position that closes it
  uint8_t* need;          // per segment, one byte per batch position: 1 if
                          // some estimator takes its f1 from it this step
  uint64_t need_bytes;    // over all segments (a multiple of 16)
  uint32_t* inv;          // per arc slot: its index in the sorted arcs (only
                          // for arcs of needed positions)
  uint32_t* err;          // sticky error bits
  uint32_t id_limit;      // largest vertex id allowed (declared bound - 1)
  uint32_t npass;         // radix passes launched: the number of D-bit
                          // digits of the bound (1..kPasses)
  uint32_t dbits;         // digit width D: 8 or kWideBits
  uint32_t chunk_log2;    // log2 of the tiles per radix chunk (<= kChunk)
  uint32_t single_chunk;  // 1: every segment is one radix chunk and D = 8;
                          // the count sums then write each chunk's bin
                          // starts as its bases and no k_cscan runs
};

// arguments of the per-estimator (naive) step: one bank, one batch
struct NaiveArgs {
  const uint32_t* edges;  // W: uint32[2w], device
  uint32_t w;
  uint32_t r;
  uint64_t m;             // |E| before the batch
  uint64_t batch;
  uint64_t key0;
  uint64_t est_off;
  uint64_t* r1;
  uint64_t* r2;
  uint32_t* cc;
  uint32_t* err;
};

// The fused step of small chunks (k_small): every chunk of at most
// kSmallW edges runs Steps 1-3 in one launch, in LDS, with no scratch; a
// block takes one bank's slice of kSmallR estimators and rebuilds the
// chunk's sorted arcs and edge table itself.
constexpr uint32_t kSmallW = 2048;     // edges of a fused chunk at most
constexpr uint32_t kSmallR = 1024;     // estimators per block (one per
                                       // thread: small banks spread over CUs)
constexpr int kSmallThreads = 1024;

struct SmallDesc {
  const uint32_t* edges;  // W: uint32[2w], device
  uint64_t m;             // bank's |E| before this batch
  uint64_t batch;         // bank's batch index
  uint64_t key0;          // mix64(seed ^ golden)
  uint64_t est_off;       // bank's first estimator
  uint32_t w;             // edges (1..kSmallW)
  uint32_t r;             // estimators in the bank
  uint32_t blk_off;       // first k_small block of the chunk
  uint32_t pad;
};

struct SmallArgs {
  const SmallDesc* descs;  // device copy of the descriptors
  SmallDesc d0;            // inline copy when nseg == 1
  uint32_t nseg;
  uint32_t nblk;           // blocks over all chunks
  uint64_t* r1;
  uint64_t* r2;
  uint32_t* cc;
  uint32_t* err;
  uint32_t id_limit;       // largest vertex id allowed
};

}  // namespace tc
