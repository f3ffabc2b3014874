// A measurement aid: the achievable HBM bandwidth of the device, from a plain
// copy (STREAM-style), to set the grid path's bandwidth against what the
// memory system sustains rather than against the nominal peak alone.
#include <cstdint>

#include <hip/hip_runtime.h>

#include "fstat.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Grid-stride copy of n 16-byte words with streaming (non-temporal) accesses:
// every word is read once and written once, nothing is reused.
__global__ void __launch_bounds__(256) k_copy16(const f4* __restrict__ src, f4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" fstat_status fstat_copy_probe(void* dst, const void* src, int64_t bytes, int32_t blocks, void* hip_stream) {
  if (!dst || !src || bytes <= 0 || (bytes & 15) != 0 || ((uintptr_t)dst & 15) != 0 || ((uintptr_t)src & 15) != 0 ||
      blocks < 0 || blocks > (1 << 20))
    return FSTAT_EINVAL;
  const char* d = (const char*)dst;
  const char* s = (const char*)src;
  if (d < s + bytes && s < d + bytes) return FSTAT_EINVAL;  // overlapping buffers
  const int64_t n = bytes / 16;
  const int64_t want = (n + 255) / 256;
  const int grid = (int)(blocks > 0 ? (want < blocks ? want : blocks) : (want < 8192 ? want : 8192));
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (const f4*)src, (f4*)dst, n);
  return hipGetLastError() == hipSuccess ? FSTAT_OK : FSTAT_EDEVICE;
}
