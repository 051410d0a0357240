// Library-wide entry points: version, status strings, zero fill, occupancy
// packing and the photometric L2 loss.
#include "common.h"

using namespace ia355;

extern "C" int32_t ia355_version(void) { return IA355_VERSION; }

extern "C" const char *ia355_error_string(int32_t s) {
  switch (s) {
    case IA355_OK: return "ok";
    case IA355_ERR_INVALID_ARG: return "invalid argument (null pointer, size, dtype or shape)";
    case IA355_ERR_WORKSPACE: return "workspace too small";
    case IA355_ERR_UNSUPPORTED: return "unsupported combination of arguments";
    case IA355_ERR_HIP: return "HIP launch error";
    case IA355_ERR_SCRATCH: return "problem larger than the fixed scratch of the allocation-free entry point";
    case IA355_ERR_CAPACITY: return "sample buffer too small (n_required holds the count needed)";
    default: return "unknown status";
  }
}

__global__ void zero_kernel(uint4 *p16, int64_t n16, uint8_t *tail, int64_t ntail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p16[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0)
    for (int64_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

extern "C" int32_t ia355_zero(void *p, size_t bytes, ia355_stream_t stream) {
  if (bytes == 0) return IA355_OK;
  if (!p) return IA355_ERR_INVALID_ARG;
  uint8_t *b = (uint8_t *)p;
  // head bytes up to 16-byte alignment are folded into the tail pass
  size_t mis = (16 - ((uintptr_t)b & 15)) & 15;
  if (mis > bytes) mis = bytes;
  if (mis) {
    zero_kernel<<<1, 64, 0, as_stream(stream)>>>(nullptr, 0, b, (int64_t)mis);
    b += mis;
    bytes -= mis;
  }
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t nt = (int64_t)(bytes - 16 * (size_t)n16);
  if (n16 || nt)
    zero_kernel<<<grid_for(n16 ? n16 : 1, 256), 256, 0, as_stream(stream)>>>((uint4 *)b, n16, b + 16 * n16, nt);
  return launch_status();
}

// One thread per output word: 32 cells of one brick (8 along x, 4 along y).
__global__ void occ_pack_kernel(const uint8_t *occ, int G, uint32_t *bits, int64_t nword) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nword) return;
  const int64_t nb = (G + 7) / 8;
  const int64_t brick = w >> 5;
  const int q = (int)(w & 31);
  const int x0 = (int)(brick % nb) * 8, y0 = (int)((brick / nb) % nb) * 8 + (q & 1) * 4;
  const int z = (int)(brick / (nb * nb)) * 16 + (q >> 1);
  uint32_t v = 0;
  if (z < G) {
    for (int j = 0; j < 32; ++j) {
      const int x = x0 + (j & 7), y = y0 + (j >> 3);
      if (x < G && y < G && occ[(int64_t)x + (int64_t)G * ((int64_t)y + (int64_t)G * z)]) v |= 1u << j;
    }
  }
  bits[w] = v;
}

extern "C" size_t ia355_occ_words(int32_t G) { return G > 0 && G <= 2048 ? (size_t)occ_words(G) : 0; }

extern "C" int32_t ia355_occ_pack(const uint8_t *occ, int32_t G, uint32_t *bits, ia355_stream_t stream) {
  if (!occ || !bits || G <= 0 || G > 2048) return IA355_ERR_INVALID_ARG;
  const int64_t nword = occ_words(G);
  occ_pack_kernel<<<(unsigned)ceil_div(nword, 256), 256, 0, as_stream(stream)>>>(occ, G, bits, nword);
  return launch_status();
}

// One block: deterministic reduction order for any R.
__global__ void __launch_bounds__(1024) l2_loss_kernel(const float *c, const float *t, int64_t n, float inv,
                                                       float *loss, float *grad) {
  __shared__ float part[1024 / kWave];
  constexpr int kU = 8;  // elements per thread per round, loads issued together
  float acc = 0.0f;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kU * blockDim.x) {
    float cv[kU], tv[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int64_t i = i0 + (int64_t)k * blockDim.x;
      cv[k] = i < n ? c[i] : 0.0f;
      tv[k] = i < n ? t[i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int64_t i = i0 + (int64_t)k * blockDim.x;
      const float e = cv[k] - tv[k];
      acc += e * e;
      if (i < n) grad[i] = 2.0f * e * inv;
    }
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) part[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += part[i];
    loss[0] = s * inv;
  }
}

extern "C" int32_t ia355_l2_loss(const float *color, const float *target, int64_t R, float *loss, float *grad_color,
                                 ia355_stream_t stream) {
  if (R <= 0 || !color || !target || !loss || !grad_color) return IA355_ERR_INVALID_ARG;
  l2_loss_kernel<<<1, 1024, 0, as_stream(stream)>>>(color, target, 3 * R, 1.0f / (3.0f * (float)R), loss, grad_color);
  return launch_status();
}
