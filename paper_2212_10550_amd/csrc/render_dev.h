// Volume rendering along a ray (Sec. 3.2): alpha compositing of the samples
// of one ray by kSeg lanes, shared by the compositing kernels and the fused
// batch renderer so that both take the same early-termination decisions and
// round the same way (internal).
#pragma once
#include "common.h"

namespace ia355 {
namespace rnd {

constexpr int kSeg = 16;  // lanes per ray

// Inclusive scans over the kSeg lanes of a segment (lane j of the segment
// gets the product / sum over lanes 0..j).
__device__ __forceinline__ float seg_scan_mul(float v, int j) {
#pragma unroll
  for (int o = 1; o < kSeg; o <<= 1) {
    const float t = __shfl_up(v, o, kSeg);
    if (j >= o) v *= t;
  }
  return v;
}
__device__ __forceinline__ float seg_scan_add(float v, int j) {
#pragma unroll
  for (int o = 1; o < kSeg; o <<= 1) {
    const float t = __shfl_up(v, o, kSeg);
    if (j >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ float seg_sum(float v) {
#pragma unroll
  for (int o = kSeg / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kSeg);
  return v;
}

// Transmittance before each lane's sample: T_in times the product of the
// lower lanes' factors.  Also returns the product over all kSeg lanes.
__device__ __forceinline__ float seg_trans(float T_in, float ex, int j, float *chunk_prod) {
  const float incl = seg_scan_mul(ex, j);
  const float excl = __shfl_up(incl, 1, kSeg);
  *chunk_prod = __shfl(incl, kSeg - 1, kSeg);
  return j == 0 ? T_in : T_in * excl;
}

// Number of lanes of this segment whose predicate holds (a prefix).
__device__ __forceinline__ int seg_count(bool p) {
  const int seg = (threadIdx.x & (kWave - 1)) / kSeg;
  return __popcll((__ballot(p) >> (kSeg * seg)) & 0xffffull);
}

struct RayOut {
  float C[3], A, T;
  int used;
};

// Composites samples b..e-1 of one ray (lane j of its kSeg-lane segment);
// src(i, &sigma, rgb) reads sample i.  Every lane of the segment returns the
// ray's colour, opacity, final transmittance and number of samples used.
template <class Src>
__device__ __forceinline__ RayOut composite_ray(const Src &src, int64_t b, int64_t e, float dt, float T_thresh,
                                                int j) {
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, A = 0.0f;
  int used = 0;
  for (int64_t base = b; base < e; base += kSeg) {
    const int64_t i = base + j;
    const bool valid = i < e;
    float s = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
    if (valid) src(i, &s, c);
    const float x = valid ? s * dt : 0.0f;
    float prod;
    const float Ti = seg_trans(T, valid ? expf(-x) : 1.0f, j, &prod);
    const bool use = valid && Ti >= T_thresh;
    if (use) {
      const float w = Ti * -expm1f(-x);
      C0 += w * c[0];
      C1 += w * c[1];
      C2 += w * c[2];
      A += w;
    }
    const int n = seg_count(use);
    used += n;
    const int len = e - base < kSeg ? (int)(e - base) : kSeg;
    if (n < len) {  // terminated inside this chunk: T of the first unused sample
      T = __shfl(Ti, n, kSeg);
      break;
    }
    T *= prod;
  }
  RayOut q;
  q.C[0] = seg_sum(C0);
  q.C[1] = seg_sum(C1);
  q.C[2] = seg_sum(C2);
  q.A = seg_sum(A);
  q.T = T;
  q.used = used;
  return q;
}

// Reads sigma and the three colour channels of sample i from planar arrays
// (channel c of sample i at rgb[c * ld + i]).
struct PlanarSrc {
  const float *__restrict__ sigma;
  const float *__restrict__ rgb;
  int64_t ld;
  __device__ __forceinline__ void operator()(int64_t i, float *s, float c[3]) const {
    *s = sigma[i];
    c[0] = rgb[i];
    c[1] = rgb[ld + i];
    c[2] = rgb[2 * ld + i];
  }
};

}  // namespace rnd
}  // namespace ia355
