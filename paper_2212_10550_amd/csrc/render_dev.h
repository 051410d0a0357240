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

// Compositing state of one ray between its groups of kSeg samples: T and
// used are the same in every lane of the segment, C and A are per-lane
// partial sums (lane j holds samples j, j + kSeg, ...).
struct RayState {
  float T, C0, C1, C2, A;
  int used;
  bool done;
};

__device__ __forceinline__ RayState ray_start() { return RayState{1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0, false}; }

// One group: samples base .. base + kSeg - 1 of samples .. e - 1 (lane j
// takes sample base + j); src(i, &sigma, rgb) reads sample i.  Sets done at
// the first group with an unused sample (T is then the transmittance of
// that sample), as the termination test T_i >= T_thresh keeps a prefix.
template <class Src>
__device__ __forceinline__ void composite_group(const Src &src, int64_t base, int64_t e, float dt, float T_thresh,
                                                int j, RayState &st) {
  const int64_t i = base + j;
  const bool valid = i < e;
  float s = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
  if (valid) src(i, &s, c);
  const float x = valid ? s * dt : 0.0f;
  float prod;
  const float Ti = seg_trans(st.T, valid ? expf(-x) : 1.0f, j, &prod);
  const bool use = valid && Ti >= T_thresh;
  if (use) {
    const float w = Ti * -expm1f(-x);
    st.C0 += w * c[0];
    st.C1 += w * c[1];
    st.C2 += w * c[2];
    st.A += w;
  }
  const int n = seg_count(use);
  st.used += n;
  const int len = e - base < kSeg ? (int)(e - base) : kSeg;
  if (n < len) {  // terminated inside this group: T of the first unused sample
    st.T = __shfl(Ti, n, kSeg);
    st.done = true;
  } else {
    st.T *= prod;
  }
}

// Composites samples b..e-1 of one ray (lane j of its kSeg-lane segment);
// src(i, &sigma, rgb) reads sample i.  Every lane of the segment returns the
// ray's colour, opacity, final transmittance and number of samples used.
// Only the groups up to the one where the ray terminates are read.
template <class Src>
__device__ __forceinline__ RayOut composite_ray(const Src &src, int64_t b, int64_t e, float dt, float T_thresh,
                                                int j) {
  RayState st = ray_start();
  for (int64_t base = b; base < e && !st.done; base += kSeg) composite_group(src, base, e, dt, T_thresh, j, st);
  RayOut q;
  q.C[0] = seg_sum(st.C0);
  q.C[1] = seg_sum(st.C1);
  q.C[2] = seg_sum(st.C2);
  q.A = seg_sum(st.A);
  q.T = st.T;
  q.used = st.used;
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
