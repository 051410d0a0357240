// Internal helpers of libia355 (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ia355.h"

#define IA355_VERSION 100

namespace ia355 {

constexpr int kWave = 64;

// MFMA operand and accumulator vectors
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

inline int32_t launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? IA355_OK : IA355_ERR_HIP;
}

inline hipStream_t as_stream(ia355_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Grid size for a grid-stride kernel over n items: enough blocks to fill
// every CU several times (256 CUs on MI355X), never more than needed.
inline unsigned grid_for(int64_t n, int block, int64_t max_blocks = 256 * 16) {
  int64_t g = ceil_div(n, block);
  if (g > max_blocks) g = max_blocks;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Sample count of a call.  Without a device counter it is S; with one it is
// min(S, *S_dev), read on the device, and S is the capacity the caller sized
// the buffers and the launch for.  Kernels that take S_dev loop over their
// items (grid-stride), so a grid sized for the capacity stays bounded.
__device__ __forceinline__ int64_t count_of(int64_t S, const int64_t *S_dev) {
  if (!S_dev) return S;
  const int64_t d = *S_dev;
  return d < 0 ? 0 : (d < S ? d : S);
}

// Blocks for a grid-stride launch over `needed` blocks of work: all of them
// when the count is known on the host, at most `cap_blocks` when it is read
// on the device (the loop covers the rest).
inline unsigned stride_grid(int64_t needed, bool device_count, int64_t cap_blocks = 2048) {
  if (needed < 1) needed = 1;
  if (device_count && needed > cap_blocks) needed = cap_blocks;
  return (unsigned)needed;
}

// Packed occupancy bits: bricks of 8 x 8 x 16 cells (x, y, z), 1024 bits =
// one 128-byte cache line each, bricks in x-fastest order; inside a brick,
// cell (lx, ly, lz) is bit lx + 8 ly + 64 lz.
__host__ __device__ inline int64_t occ_words(int64_t G) {
  return ceil_div(G, 8) * ceil_div(G, 8) * ceil_div(G, 16) * 32;
}
__device__ __forceinline__ uint32_t occ_word(int x, int y, int z, int G) {
  const uint32_t nb = (uint32_t)(G + 7) >> 3;  // bricks along x and along y
  const uint32_t brick = ((uint32_t)x >> 3) + nb * (((uint32_t)y >> 3) + nb * ((uint32_t)z >> 4));
  return brick * 32u + (((uint32_t)y & 7u) >> 2) + 2u * ((uint32_t)z & 15u);
}
__device__ __forceinline__ uint32_t occ_bit(int x, int y) { return ((uint32_t)x & 7u) + 8u * ((uint32_t)y & 3u); }

// Workspace carving: 256-byte aligned slices.
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Wave-level reductions / scans with cross-lane shuffles (wave64).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ float wave_incl_scan_f(float v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    float t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// Multiresolution grid resolution of level l: floor(base * growth^l),
// computed on the host in double precision.
inline int32_t level_resolution(double base, double growth, int l) {
  return (int32_t)floor(base * pow(growth, (double)l));
}

}  // namespace ia355
