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
// Three launches: k_tok_count counts the tokens each thread's 256 bytes
// start, k_tok_scan turns the per-block totals into exclusive prefixes (one
// block), and k_tok_write recounts, ranks within the block and writes every
// token to its place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/tc.h"

namespace {

constexpr int kPBlock = 256;
constexpr uint32_t kPBytes = 256;                  // bytes per thread
constexpr uint64_t kPTile = (uint64_t)kPBlock * kPBytes;  // bytes per block
constexpr uint32_t kMaxLine = 4096;  // a comment test looks back this far

// parse error bits (device word)
constexpr uint32_t kPErrOverflow = 1u;  // a token above 2^32 - 1
constexpr uint32_t kPErrLine = 2u;      // a line longer than kMaxLine
constexpr uint32_t kPErrRoom = 4u;      // more edges than the output holds

__device__ __forceinline__ bool is_digit(uint8_t c) { return c >= '0' && c <= '9'; }

// The block's tile of text staged in LDS (16-byte coalesced loads); bytes
// outside it (a line start before the tile, a token running past its end)
// come from global memory.
struct Tile {
  const uint8_t* t;   // whole text (global)
  const uint8_t* s;   // the tile in LDS
  uint64_t t0, t1;    // tile = [t0, t1)
  __device__ __forceinline__ uint8_t operator[](uint64_t p) const {
    return (p >= t0 && p < t1) ? s[p - t0] : t[p];
  }
};

__device__ void stage_tile(const uint8_t* t, uint64_t n, uint8_t* s, uint64_t t0) {
  const uint64_t t1 = t0 + kPTile < n ? t0 + kPTile : n;
  const uint64_t len = t1 - t0;
  // the text base is 16-byte aligned when allocated by HIP and t0 is a
  // multiple of kPTile; a misaligned text falls back to byte loads
  if ((reinterpret_cast<uintptr_t>(t) & 15u) == 0) {
    const uint4* g = reinterpret_cast<const uint4*>(t + t0);
    uint4* l = reinterpret_cast<uint4*>(s);
    for (uint64_t k = threadIdx.x; k < len / 16; k += kPBlock) l[k] = g[k];
    for (uint64_t k = len / 16 * 16 + threadIdx.x; k < len; k += kPBlock) s[k] = t[t0 + k];
  } else {
    for (uint64_t k = threadIdx.x; k < len; k += kPBlock) s[k] = t[t0 + k];
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
  const uint8_t* sp = t.s + (b - t.t0);  // 4-byte aligned: slices start at
  const uint32_t len = (uint32_t)(e - b);  // multiples of kPBytes
  for (uint32_t i = 0; i < len; i += 4) {
    const uint32_t word = *reinterpret_cast<const uint32_t*>(sp + i);
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

__global__ __launch_bounds__(kPBlock) void k_tok_count(const uint8_t* text, uint64_t n,
                                                       uint32_t* block_tok, uint32_t* err) {
  __shared__ __align__(16) uint8_t s_tile[kPTile];
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  const uint64_t t0 = (uint64_t)blockIdx.x * kPTile;
  stage_tile(text, n, s_tile, t0);
  const Tile t{text, s_tile, t0, t0 + kPTile < n ? t0 + kPTile : n};
  const uint64_t b = (uint64_t)blockIdx.x * kPTile + (uint64_t)threadIdx.x * kPBytes;
  const uint32_t k = count_range(t, n, std::min(b, n), std::min(b + kPBytes, n), err);
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

__global__ __launch_bounds__(kPBlock) void k_tok_write(const uint8_t* text, uint64_t n,
                                                       const uint32_t* block_tok,
                                                       uint32_t* out, uint64_t max_tok,
                                                       uint32_t* err) {
  __shared__ __align__(16) uint8_t s_tile[kPTile];
  __shared__ uint32_t s_cnt[kPBlock];
  const int tid = threadIdx.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * kPTile;
  stage_tile(text, n, s_tile, t0);
  const Tile t{text, s_tile, t0, t0 + kPTile < n ? t0 + kPTile : n};
  const uint64_t b = std::min((uint64_t)blockIdx.x * kPTile + (uint64_t)tid * kPBytes, n);
  const uint64_t e = std::min(b + kPBytes, n);
  const uint32_t k = count_range(t, n, b, e, err);
  s_cnt[tid] = k;
  __syncthreads();
  // exclusive prefix over the block's threads (a small serial scan by
  // thread 0 is plenty next to the byte loops)
  if (tid == 0) {
    uint32_t run = 0;
    for (int i = 0; i < kPBlock; ++i) {
      const uint32_t v = s_cnt[i];
      s_cnt[i] = run;
      run += v;
    }
  }
  __syncthreads();
  if (k == 0) return;
  uint64_t idx = (uint64_t)block_tok[blockIdx.x] + s_cnt[tid];
  walk_range(t, b, e, err, [&](uint64_t p) {
    uint64_t v = 0;
    for (uint64_t q = p; q < n && is_digit(t[q]); ++q) {
      v = v * 10 + (t[q] - '0');
      if (v > 0xFFFFFFFFull) {
        atomicOr(err, kPErrOverflow);
        v = 0;
        break;
      }
    }
    if (idx < max_tok) out[idx] = (uint32_t)v;
    else atomicOr(err, kPErrRoom);
    ++idx;
  });
}

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
  const uint64_t nblk = (nbytes + kPTile - 1) / kPTile;
  if (nblk > 0xFFFFFFFFull) return tc::report(TC_EINVAL, "text too large");
  uint32_t* block_tok = nullptr;
  uint32_t* err = nullptr;
  uint64_t* total = nullptr;
  int rc = TC_OK;
  if (hipMalloc(reinterpret_cast<void**>(&block_tok), sizeof(uint32_t) * nblk) ||
      hipMalloc(reinterpret_cast<void**>(&err), sizeof(uint32_t)) ||
      hipMalloc(reinterpret_cast<void**>(&total), sizeof(uint64_t))) {
    rc = TC_ENOMEM;
  } else {
    uint32_t h_err = 0;
    uint64_t h_total = 0;
    const uint8_t* t = reinterpret_cast<const uint8_t*>(text);
    if (hipMemsetAsync(err, 0, sizeof(uint32_t), st) != hipSuccess) rc = TC_EHIP;
    if (rc == TC_OK) {
      hipLaunchKernelGGL(k_tok_count, dim3((uint32_t)nblk), dim3(kPBlock), 0, st, t, nbytes,
                         block_tok, err);
      hipLaunchKernelGGL(k_tok_scan, dim3(1), dim3(kPBlock), 0, st, block_tok,
                         (uint32_t)nblk, total);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(&h_total, total, sizeof(uint64_t), hipMemcpyDeviceToHost, st) ||
          hipStreamSynchronize(st))
        rc = TC_EHIP;
    }
    if (rc == TC_OK && (h_total & 1u)) rc = TC_EINVAL;          // a dangling id
    if (rc == TC_OK && h_total >= 0xFFFFFFFFull) rc = TC_EINVAL;  // 32-bit token index
    if (rc == TC_OK && h_total / 2 > max_edges) rc = TC_EINVAL;
    if (rc == TC_OK && h_total && !edges) rc = TC_EINVAL;
    if (rc == TC_OK && h_total) {
      hipLaunchKernelGGL(k_tok_write, dim3((uint32_t)nblk), dim3(kPBlock), 0, st, t, nbytes,
                         block_tok, edges, 2 * max_edges, err);
      if (hipGetLastError() != hipSuccess) rc = TC_EHIP;
    }
    if (rc == TC_OK &&
        (hipMemcpyAsync(&h_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st) ||
         hipStreamSynchronize(st)))
      rc = TC_EHIP;
    if (rc == TC_OK && h_err) rc = TC_EINVAL;
    if (rc == TC_OK) *nedges = h_total / 2;
  }
  if (block_tok) (void)hipFree(block_tok);
  if (err) (void)hipFree(err);
  if (total) (void)hipFree(total);
  if (rc == TC_ENOMEM) return tc::report(rc, "device allocation for parsing failed");
  if (rc == TC_EHIP) return tc::report(rc, "a HIP call failed while parsing");
  if (rc != TC_OK) return tc::report(rc, "malformed edge list (odd id count, an id above "
                                         "2^32-1, a line over 4096 bytes) or too many edges");
  return TC_OK;
}

}  // extern "C"
