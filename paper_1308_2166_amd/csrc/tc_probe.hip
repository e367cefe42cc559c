// Diagnostics: the random cache-line read rate of the device, the ceiling
// of a kernel whose time goes to independent random line reads (Step 2's
// directory, inverse-index, arc and edge lookups, Sec. 4.3).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tc.h"

namespace tcprobe {

constexpr int kThreads = 256;
constexpr uint32_t kLineWords = 32;  // 128-byte lines of 32-bit words

__device__ __forceinline__ uint64_t hash64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// thread i reads `per` words, each the first word of a line drawn by the
// hash of (i, k, salt); dependent: the word read feeds the next address
__global__ __launch_bounds__(kThreads) void k_lines(const uint32_t* t, uint64_t nlines,
                                                    uint32_t n, uint32_t per, uint32_t dep,
                                                    uint32_t salt, uint32_t* sink) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  uint64_t key = ((uint64_t)salt << 40) ^ ((uint64_t)i << 3);
  uint32_t acc = 0;
  if (dep) {
    for (uint32_t k = 0; k < per; ++k) {
      acc += t[(hash64(key + k + acc) % nlines) * kLineWords];
    }
  } else {
    uint32_t v[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k)
      v[k] = k < per ? t[(hash64(key + k) % nlines) * kLineWords] : 0u;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) acc += v[k];
  }
  sink[i] = acc;
}

}  // namespace tcprobe

namespace tc {
int report(int code, const char* msg);  // sets the text of tc_last_error
}

extern "C" int tc_probe_line_rate(const void* table, uint64_t table_bytes, uint32_t n,
                                  uint32_t per_thread, uint32_t dependent, uint32_t reps,
                                  uint32_t* sink, double* lines_per_s, void* stream) {
  using namespace tcprobe;
  if (!table || !sink || !lines_per_s || table_bytes < 128 || table_bytes % 128 ||
      n == 0 || per_thread < 1 || per_thread > 8 || reps == 0)
    return tc::report(TC_EINVAL, "tc_probe_line_rate: bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint64_t nlines = table_bytes / 128;
  const uint32_t grid = (uint32_t)((n + kThreads - 1) / kThreads);
  const uint32_t* t = static_cast<const uint32_t*>(table);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = TC_EHIP;
  float ms = 0.f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  hipLaunchKernelGGL(k_lines, dim3(grid), dim3(kThreads), 0, st, t, nlines, n, per_thread,
                     dependent, 0u, sink);
  if (hipEventRecord(e0, st) != hipSuccess) goto done;
  for (uint32_t r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_lines, dim3(grid), dim3(kThreads), 0, st, t, nlines, n, per_thread,
                       dependent, r + 1u, sink);
  if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      ms <= 0.f)
    goto done;
  *lines_per_s = (double)n * per_thread * reps / (ms * 1e-3);
  rc = TC_OK;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc == TC_OK ? rc : tc::report(rc, "tc_probe_line_rate: a HIP call failed");
}
