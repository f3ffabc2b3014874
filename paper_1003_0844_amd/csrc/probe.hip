// Measurement aids: the achievable HBM bandwidth of the device, from a plain
// copy (STREAM-style) and from the first FFT pass's store pattern alone, to
// set the grid path's bandwidth against what the memory system sustains
// rather than against the nominal peak alone.
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

// The store pattern of the first FFT pass alone (grid.hip, tiles.h): workgroup
// (r, node) writes the C elements of row r of its node's spill, thread t the
// elements k2 = t + q C/16 (q < 16) of the pass's last radix-16 stage, at
// Z[k2 / b2][r][k2 % b2] (blocked) or Z[r][k2] (b2 = 0), with 16-byte streaming
// stores: the pass's bytes without its transform, for the rate its write
// pattern can reach.  blockDim = C / 16.
__global__ void __launch_bounds__(256) k_spill_write(f4* __restrict__ dst, int R, int C, int lb2) {
  const int r = blockIdx.x;
  f4* __restrict__ node = dst + (int64_t)blockIdx.y * R * C;
  const int str = C / 16;
  const f4 v = {(float)r, (float)blockIdx.y, 0.0f, 1.0f};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k2 = (int)threadIdx.x + q * str;
    const int64_t at = lb2 > 0 ? ((int64_t)(k2 >> lb2) * R + r) * (1 << lb2) + (k2 & ((1 << lb2) - 1))
                               : (int64_t)r * C + k2;
    __builtin_nontemporal_store(v, node + at);
  }
}

}  // namespace

extern "C" fstat_status fstat_spill_write_probe(void* dst, int64_t nodes, int32_t R, int32_t C, int32_t b2,
                                                void* hip_stream) {
  if (!dst || ((uintptr_t)dst & 15) != 0 || nodes <= 0 || nodes > 65535 || R <= 0 || R > (1 << 20) ||
      (C != 1024 && C != 2048 && C != 4096) || b2 < 0 || b2 > C || (b2 > 0 && (b2 & (b2 - 1)) != 0))
    return FSTAT_EINVAL;
  const int lb2 = b2 > 0 ? __builtin_ctz((unsigned)b2) : 0;
  hipLaunchKernelGGL(k_spill_write, dim3((unsigned)R, (unsigned)nodes), dim3(C / 16), 0, (hipStream_t)hip_stream,
                     (f4*)dst, R, C, lb2);
  return hipGetLastError() == hipSuccess ? FSTAT_OK : FSTAT_EDEVICE;
}

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
