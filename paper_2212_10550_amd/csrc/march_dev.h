// Ray sampling with empty-space skipping (Sec. 3.2, Sec. 3.3), shared by the
// march kernels and the fused batch renderer so that both take the same
// keep/skip decisions and compute the same sample positions: every
// operation is an individually rounded IEEE single operation (internal).
#pragma once
#include <cmath>

#include "common.h"

namespace ia355 {
namespace mch {

struct Box {
  float lo[3], hi[3];
  float inv_ext[3];  // 1 / (hi - lo), used only when every extent is a power of two
};

struct RaySpan {
  float tn, tf, dt;
  bool hit;
};

__device__ __forceinline__ RaySpan ray_span(const float o[3], const float d[3], const Box &b, float dt_fixed,
                                            int n_per_ray) {
#pragma clang fp contract(off)
  float tmin = -INFINITY, tmax = INFINITY;
  RaySpan s{0.0f, 0.0f, 0.0f, false};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0f) {
      const float ta = (b.lo[a] - o[a]) / d[a];
      const float tb = (b.hi[a] - o[a]) / d[a];
      const float t0 = ta < tb ? ta : tb;
      const float t1 = ta < tb ? tb : ta;
      if (t0 > tmin) tmin = t0;
      if (t1 < tmax) tmax = t1;
    } else if (o[a] < b.lo[a] || o[a] > b.hi[a]) {
      return s;
    }
  }
  const float tn = tmin > 0.0f ? tmin : 0.0f;
  if (!(tmax > tn)) return s;
  s.tn = tn;
  s.tf = tmax;
  s.dt = n_per_ray > 0 ? (tmax - tn) / (float)n_per_ray : dt_fixed;
  s.hit = true;
  return s;
}

// Ray parameter of step k: the midpoint of the k-th interval.
__device__ __forceinline__ float step_t(const RaySpan &s, int k) {
#pragma clang fp contract(off)
  return s.tn + ((float)k + 0.5f) * s.dt;
}

// Sample k of a ray: position and whether its cell is occupied.
// kPow2Ext: every box extent is a power of two, so dividing by it and
// multiplying by its (exact) reciprocal round the same real number once and
// give the same float; the multiply saves the division sequence.
template <bool kPow2Ext>
__device__ __forceinline__ bool sample_at(const float o[3], const float d[3], const RaySpan &s, int k, const Box &b,
                                          const uint32_t *bits, int G, float *t_out, float x[3]) {
#pragma clang fp contract(off)
  const float t = step_t(s, k);
  *t_out = t;
  int cell[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a] = o[a] + t * d[a];
    const float rel = kPow2Ext ? (x[a] - b.lo[a]) * b.inv_ext[a] : (x[a] - b.lo[a]) / (b.hi[a] - b.lo[a]);
    const float u = rel * (float)G;
    int c = (int)floorf(u);
    cell[a] = c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
  }
  if (!bits) return true;
  const uint32_t word = occ_word(cell[0], cell[1], cell[2], G);
  return (bits[word] >> occ_bit(cell[0], cell[1])) & 1u;
}

__device__ __forceinline__ void load_ray(const float *ro, const float *rd, int64_t r, float o[3], float d[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = ro[3 * r + a];
    d[a] = rd[3 * r + a];
  }
}

// Position and ray parameter of step k (the expressions of sample_at).
__device__ __forceinline__ void sample_pos(const float o[3], const float d[3], float tn, float dt, int k, float *t_out,
                                           float x[3]) {
#pragma clang fp contract(off)
  const float t = tn + ((float)k + 0.5f) * dt;
  *t_out = t;
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
}

// Host side: the occupancy box, and whether every extent is a power of two
// (then sample_at may multiply by the exact reciprocal).  False for an empty
// or inverted box.
inline bool make_box(const float *aabb, Box *box, bool *pow2) {
  if (!aabb) return false;
  for (int a = 0; a < 3; ++a) {
    box->lo[a] = aabb[a];
    box->hi[a] = aabb[3 + a];
    if (!(box->hi[a] > box->lo[a])) return false;
  }
  bool p2 = true;
  for (int a = 0; a < 3; ++a) {
    const float ext = box->hi[a] - box->lo[a];
    int e;
    p2 = p2 && std::isfinite(ext) && std::frexp(ext, &e) == 0.5f && e > -100 && e < 100;
    box->inv_ext[a] = p2 ? 1.0f / ext : 0.0f;
  }
  *pow2 = p2;
  return true;
}

}  // namespace mch
}  // namespace ia355
