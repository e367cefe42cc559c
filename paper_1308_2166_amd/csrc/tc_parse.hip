// On-device parsing of a text edge list (the input side of the stream: the
// paper reads its graphs as text edge lists and counts the reading time
// separately, Sec. 5, Table 2).
//
// Format: one edge per line, two unsigned decimal vertex ids separated by
// any run of non-digit bytes (spaces, tabs, commas); a line whose first
// byte is '#' or '%' is a comment; '\r\n' and a missing final newline are
// accepted.  Every token is a maximal run of digits on a non-comment line;
// tokens 2k and 2k+1 form edge k.
//
// Three launches: k_tok_count counts the tokens each thread's 128 bytes
// start (per thread and per block), k_tok_scan turns the per-block totals
// into exclusive prefixes (one block), and k_tok_write ranks each thread's
// tokens within the block, parses their values and writes every token to
// its place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "../../include/tc.h"

namespace {

constexpr int kPBlock = 256;
constexpr uint32_t kPBytes = 64;                   // bytes per thread (a slice)
constexpr uint64_t kPTile = (uint64_t)kPBlock * kPBytes;  // bytes per block
static_assert(kPTile % (16 * kPBlock) == 0, "a full tile is whole 16-byte loads per thread");
constexpr uint32_t kSliceWords = kPBytes / 4 + 1;  // a slice in LDS, plus a pad word
constexpr uint32_t kOutCap = 4096;  // ids a block stages in LDS before writing
constexpr uint32_t kMaxLine = 4096;  // a comment test looks back this far

// parse error bits (device word)
constexpr uint32_t kPErrOverflow = 1u;  // a token above 2^32 - 1
constexpr uint32_t kPErrLine = 2u;      // a line longer than kMaxLine
constexpr uint32_t kPErrRoom = 4u;      // more edges than the output holds

__device__ __forceinline__ bool is_digit(uint8_t c) { return c >= '0' && c <= '9'; }

// The block's tile of text staged in LDS; bytes outside it (a line start
// before the tile, a token running past its end) come from global memory.
// Slice k of the tile (the bytes thread k walks) starts at word
// k * kSliceWords: the pad word puts the 64 lanes of a wave, each reading
// word i of its own slice, on 64 different banks.
struct Tile {
  const uint8_t* t;   // whole text (global)
  const uint8_t* s;   // the tile in LDS
  uint64_t t0, t1;    // tile = [t0, t1)
  __device__ __forceinline__ static uint32_t lds_byte(uint32_t off) {
    return (off / kPBytes) * (4 * kSliceWords) + off % kPBytes;
  }
  __device__ __forceinline__ uint8_t operator[](uint64_t p) const {
    return (p >= t0 && p < t1) ? s[lds_byte((uint32_t)(p - t0))] : t[p];
  }
};

__device__ void stage_tile(const uint8_t* t, uint64_t n, uint8_t* s, uint64_t t0) {
  const uint64_t t1 = t0 + kPTile < n ? t0 + kPTile : n;
  const uint32_t len = (uint32_t)(t1 - t0);
  uint32_t* sw = reinterpret_cast<uint32_t*>(s);
  // the text base is 16-byte aligned when allocated by HIP and t0 is a
  // multiple of kPTile; a misaligned text falls back to byte loads.  Each
  // 16-byte load lands in one slice (kPBytes is a multiple of 16).
  constexpr uint32_t kLoads = (uint32_t)(kPTile / 16 / kPBlock);  // per thread
  if ((reinterpret_cast<uintptr_t>(t) & 15u) == 0 && len == kPTile) {
    // a full tile: every thread's loads in flight before the first store
    const uint4* g = reinterpret_cast<const uint4*>(t + t0);
    uint4 v[kLoads];
#pragma unroll
    for (uint32_t i = 0; i < kLoads; ++i) v[i] = g[threadIdx.x + i * kPBlock];
#pragma unroll
    for (uint32_t i = 0; i < kLoads; ++i) {
      uint32_t* d = sw + Tile::lds_byte(16 * (threadIdx.x + i * kPBlock)) / 4;
      d[0] = v[i].x;
      d[1] = v[i].y;
      d[2] = v[i].z;
      d[3] = v[i].w;
    }
  } else if ((reinterpret_cast<uintptr_t>(t) & 15u) == 0) {
    const uint4* g = reinterpret_cast<const uint4*>(t + t0);
    for (uint32_t k = threadIdx.x; k < len / 16; k += kPBlock) {
      const uint4 v = g[k];
      uint32_t* d = sw + Tile::lds_byte(16 * k) / 4;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
    for (uint32_t k = len / 16 * 16 + threadIdx.x; k < len; k += kPBlock)
      s[Tile::lds_byte(k)] = t[t0 + k];
  } else {
    for (uint32_t k = threadIdx.x; k < len; k += kPBlock) s[Tile::lds_byte(k)] = t[t0 + k];
  }
  __syncthreads();
}

// Is position p inside a comment line?  The line starts after the last
// '\n' before p (or at 0); the answer is its first byte.
__device__ bool in_comment(const Tile& t, uint64_t p, uint32_t* err) {
  uint64_t q = p;
  uint32_t back = 0;
  while (q > 0 && t[q - 1] != '\n') {
    --q;
    if (++back > kMaxLine) {
      atomicOr(err, kPErrLine);
      return false;
    }
  }
  return t[q] == '#' || t[q] == '%';
}

// Walk the bytes [b, e) of the thread's slice (inside the block's tile, read
// from LDS four at a time), calling f(p) at every token start outside a
// comment line; returns the number of token starts.
template <class F>
__device__ uint32_t walk_range(const Tile& t, uint64_t b, uint64_t e, uint32_t* err, F f) {
  if (b >= e) return 0;
  bool comment = in_comment(t, b, err);
  uint8_t prev = b > 0 ? t[b - 1] : (uint8_t)'\n';
  uint32_t k = 0;
  // slices start at multiples of kPBytes, so the slice's words are whole
  const uint32_t* sp =
      reinterpret_cast<const uint32_t*>(t.s) + Tile::lds_byte((uint32_t)(b - t.t0)) / 4;
  const uint32_t len = (uint32_t)(e - b);
  for (uint32_t i = 0; i < len; i += 4) {
    const uint32_t word = sp[i / 4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i + q >= len) break;
      const uint8_t c = (uint8_t)(word >> (8 * q));
      if (prev == '\n') comment = c == '#' || c == '%';
      if (!comment && is_digit(c) && !is_digit(prev)) {
        f(b + i + q);
        ++k;
      }
      prev = c;
    }
  }
  return k;
}

__device__ uint32_t count_range(const Tile& t, uint64_t n, uint64_t b, uint64_t e,
                                uint32_t* err) {
  return walk_range(t, b, e, err, [](uint64_t) {});
}

// acc = 10 acc + digit if that fits 32 bits (else false, acc unchanged)
__device__ __forceinline__ bool push_digit(uint32_t& acc, uint8_t c) {
  const uint32_t d = c - '0';
  if (acc > 429496729u || (acc == 429496729u && d > 5u)) return false;
  acc = acc * 10u + d;
  return true;
}

// The same walk, building each token's value as its digits go by (the work
// per byte is the same in every lane; a digit loop per token would run once
// per byte position at which any lane of the wave starts a token), and
// calling emit(value) when a token that started in [b, e) ends.  A token
// still open at e is finished from the bytes after it.
template <class F>
__device__ void walk_values(const Tile& t, uint64_t n, uint64_t b, uint64_t e, uint32_t* err,
                            F emit) {
  if (b >= e) return;
  bool comment = in_comment(t, b, err);
  uint8_t prev = b > 0 ? t[b - 1] : (uint8_t)'\n';
  bool open = false, over = false;
  uint32_t acc = 0;
  const uint32_t* sp =
      reinterpret_cast<const uint32_t*>(t.s) + Tile::lds_byte((uint32_t)(b - t.t0)) / 4;
  const uint32_t len = (uint32_t)(e - b);
  for (uint32_t i = 0; i < len; i += 4) {
    const uint32_t word = sp[i / 4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i + q >= len) break;
      const uint8_t c = (uint8_t)(word >> (8 * q));
      if (prev == '\n') comment = c == '#' || c == '%';
      const bool dig = !comment && is_digit(c);
      if (dig && !is_digit(prev)) {
        open = true;
        over = false;
        acc = 0;
      }
      if (dig && open) {
        over |= !push_digit(acc, c);
      } else if (open) {
        emit(over ? 0u : acc, over);
        open = false;
      }
      prev = c;
    }
  }
  if (open) {
    for (uint64_t q = e; q < n; ++q) {
      const uint8_t c = t[q];
      if (!is_digit(c)) break;
      over |= !push_digit(acc, c);
    }
    emit(over ? 0u : acc, over);
  }
}

constexpr uint32_t kTileLds = kPBlock * kSliceWords * 4;  // bytes of a staged tile

__global__ __launch_bounds__(kPBlock) void k_tok_count(const uint8_t* text, uint64_t n,
                                                       uint32_t* block_tok, uint32_t* thr_tok,
                                                       uint32_t* err) {
  __shared__ __align__(16) uint8_t s_tile[kTileLds];
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  const uint64_t t0 = (uint64_t)blockIdx.x * kPTile;
  stage_tile(text, n, s_tile, t0);
  const Tile t{text, s_tile, t0, t0 + kPTile < n ? t0 + kPTile : n};
  const uint64_t b = (uint64_t)blockIdx.x * kPTile + (uint64_t)threadIdx.x * kPBytes;
  const uint32_t k = count_range(t, n, std::min(b, n), std::min(b + kPBytes, n), err);
  thr_tok[(uint64_t)blockIdx.x * kPBlock + threadIdx.x] = k;
  if (k) atomicAdd(&s_sum, k);
  __syncthreads();
  if (threadIdx.x == 0) block_tok[blockIdx.x] = s_sum;
}

// exclusive prefix of the per-block token counts, in place (one block);
// *total receives the sum
__global__ __launch_bounds__(kPBlock) void k_tok_scan(uint32_t* block_tok, uint32_t nblk,
                                                      uint64_t* total) {
  __shared__ uint64_t s_part[kPBlock];
  const uint32_t per = (nblk + kPBlock - 1) / kPBlock;
  const uint32_t b0 = threadIdx.x * per, b1 = std::min(nblk, b0 + per);
  uint64_t sum = 0;
  for (uint32_t i = b0; i < b1; ++i) sum += block_tok[i];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (int i = 0; i < kPBlock; ++i) {
      const uint64_t v = s_part[i];
      s_part[i] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  uint64_t run = s_part[threadIdx.x];
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t v = block_tok[i];
    block_tok[i] = (uint32_t)run;  // token totals are checked to fit 32 bits
    run += v;
  }
}

// The ids a block parses go to LDS first and then out in one coalesced run
// (a block with more than kOutCap ids -- text denser than about four bytes
// per id -- stores them directly).
__global__ __launch_bounds__(kPBlock) void k_tok_write(const uint8_t* text, uint64_t n,
                                                       const uint32_t* block_tok,
                                                       const uint32_t* thr_tok,
                                                       uint32_t* out, uint64_t max_tok,
                                                       uint32_t* err) {
  __shared__ __align__(16) uint8_t s_tile[kTileLds];
  __shared__ uint32_t s_out[kOutCap];
  __shared__ uint32_t s_wave[kPBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t t0 = (uint64_t)blockIdx.x * kPTile;
  // the thread's token count (from k_tok_count), then its exclusive prefix
  // over the block: within the wave by shuffles, across waves in LDS
  const uint32_t k = thr_tok[(uint64_t)blockIdx.x * kPBlock + tid];
  uint32_t x = k;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  stage_tile(text, n, s_tile, t0);  // (ends with a barrier)
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kPBlock / 64; ++w) {
    before += w < wave ? s_wave[w] : 0u;
    total += s_wave[w];
  }
  const Tile t{text, s_tile, t0, t0 + kPTile < n ? t0 + kPTile : n};
  const uint64_t b = std::min((uint64_t)blockIdx.x * kPTile + (uint64_t)tid * kPBytes, n);
  const uint64_t e = std::min(b + kPBytes, n);
  const bool staged = total <= kOutCap;
  const uint64_t base = block_tok[blockIdx.x];
  uint32_t j = before + x - k;
  if (k) {
    walk_values(t, n, b, e, err, [&](uint32_t v, bool over) {
      if (over) atomicOr(err, kPErrOverflow);
      if (staged) {
        if (j < kOutCap) s_out[j] = v;  // (always: the counts match the walk)
      } else if (base + j < max_tok) {
        out[base + j] = v;
      } else {
        atomicOr(err, kPErrRoom);
      }
      ++j;
    });
  }
  if (!staged) return;
  __syncthreads();
  for (uint32_t i = tid; i < total; i += kPBlock) {
    if (base + i < max_tok) out[base + i] = s_out[i];
    else atomicOr(err, kPErrRoom);
  }
}

// Parser scratch, one block per device: grown to the largest text parsed so
// far and reused by later calls (held until the process ends).  The lock
// also keeps two host threads from parsing into one block at once.
struct ParseScratch {
  uint8_t* p = nullptr;
  uint64_t cap = 0;
};
std::mutex g_parse_mu;
ParseScratch g_parse[64];

}  // namespace

namespace tc {
int report(int code, const char* msg);  // sets the text of tc_last_error
}

extern "C" {

int tc_parse_edges(const char* text, uint64_t nbytes, uint32_t* edges, uint64_t max_edges,
                   uint64_t* nedges, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nedges) *nedges = 0;
  if (!nedges) return tc::report(TC_EINVAL, "null edge count pointer");
  if (nbytes == 0) return TC_OK;
  if (!text) return tc::report(TC_EINVAL, "null text pointer");
  if (!edges) max_edges = 0;  // nothing may be written
  const uint64_t nblk = (nbytes + kPTile - 1) / kPTile;
  if (nblk > 0xFFFFFFFFull / kPBlock) return tc::report(TC_EINVAL, "text too large");
  // scratch: [total u64][err u32][pad][block counts][thread counts]
  const uint64_t bytes = 16 + sizeof(uint32_t) * nblk * (1 + kPBlock);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return tc::report(TC_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_parse_mu);
  ParseScratch& ps = g_parse[dev];
  if (ps.cap < bytes) {
    if (ps.p) (void)hipFree(ps.p);
    ps.p = nullptr;
    ps.cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&ps.p), bytes) != hipSuccess) {
      ps.p = nullptr;
      return tc::report(TC_ENOMEM, "device allocation for parsing failed");
    }
    ps.cap = bytes;
  }
  uint8_t* scratch = ps.p;
  uint64_t* total = reinterpret_cast<uint64_t*>(scratch);
  uint32_t* err = reinterpret_cast<uint32_t*>(scratch + 8);
  uint32_t* block_tok = reinterpret_cast<uint32_t*>(scratch + 16);
  uint32_t* thr_tok = block_tok + nblk;
  const uint8_t* t = reinterpret_cast<const uint8_t*>(text);
  // every store of k_tok_write is bounded by the output's capacity, so the
  // three kernels run back to back and the total is checked afterwards
  // (on an error the output's contents are unspecified)
  uint64_t h[2] = {0, 0};  // total, error bits
  int rc = TC_OK;
  if (hipMemsetAsync(err, 0, sizeof(uint32_t), st) != hipSuccess) rc = TC_EHIP;
  if (rc == TC_OK) {
    hipLaunchKernelGGL(k_tok_count, dim3((uint32_t)nblk), dim3(kPBlock), 0, st, t, nbytes,
                       block_tok, thr_tok, err);
    hipLaunchKernelGGL(k_tok_scan, dim3(1), dim3(kPBlock), 0, st, block_tok, (uint32_t)nblk,
                       total);
    hipLaunchKernelGGL(k_tok_write, dim3((uint32_t)nblk), dim3(kPBlock), 0, st, t, nbytes,
                       block_tok, thr_tok, edges, 2 * max_edges, err);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, scratch, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = TC_EHIP;
  }
  const uint64_t tot = h[0];
  const uint32_t perr = (uint32_t)h[1];
  if (rc == TC_EHIP) return tc::report(rc, "a HIP call failed while parsing");
  if (perr || (tot & 1u) || tot >= 0xFFFFFFFFull || tot / 2 > max_edges)
    return tc::report(TC_EINVAL, "malformed edge list (odd id count, an id above "
                                 "2^32-1, a line over 4096 bytes) or too many edges");
  *nedges = tot / 2;
  return TC_OK;
}

}  // extern "C"
