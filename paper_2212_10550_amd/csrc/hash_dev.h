// Per-point arithmetic of the multiresolution hash encoding (Sec. 3.1),
// shared by the encoding kernels and the fused batch renderer so that both
// compute the same floats: the level's cell and corner weights, the corner
// gathers and the trilinear interpolation (internal).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "common.h"

namespace ia355 {
namespace hsh {

constexpr int kMaxLevels = 32;
constexpr int kXcd = 8;

struct Levels {
  int res[kMaxLevels];
  int dense[kMaxLevels];
};

struct Box {
  float lo[3], inv[3];
};

struct Corners {
  uint32_t idx[8];
  float w[8];
  float dw[8][3];
};

// Cell of x on a level of resolution N: base vertex v0, fraction f and the
// scale dN x / dx (0 along a clamped axis).
struct CellPos {
  int v0[3];
  float f[3], sc[3];
};

__device__ __forceinline__ CellPos level_pos(const float x[3], const Box &box, int N) {
  // no contraction: (uh - i) must stay a separately rounded difference, or
  // the compiler folds the product back in and the remainder counts twice
#pragma clang fp contract(off)
  CellPos p;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float xn = (x[a] - box.lo[a]) * box.inv[a];
    p.sc[a] = (float)N * box.inv[a];
    if (!(xn >= 0.0f)) { xn = 0.0f; p.sc[a] = 0.0f; }  // also catches NaN
    if (xn > 1.0f) { xn = 1.0f; p.sc[a] = 0.0f; }
    const float uh = xn * (float)N;
    const float ul = fmaf(xn, (float)N, -uh);  // exact remainder of the product
    int i = (int)floorf(uh);
    float fr = (uh - (float)i) + ul;
    if (fr < 0.0f && i > 0) { i -= 1; fr += 1.0f; }
    if (i > N - 1) { fr += (float)(i - (N - 1)); i = N - 1; }
    if (i < 0) { i = 0; }
    p.v0[a] = i;
    p.f[a] = fr;
  }
  return p;
}

// Table index and trilinear weight of corner k (k = cx + 2 cy + 4 cz).
__device__ __forceinline__ uint32_t corner_index(const CellPos &p, int k, int N, bool dense, uint32_t Tmask) {
  const uint32_t vx = (uint32_t)(p.v0[0] + (k & 1));
  const uint32_t vy = (uint32_t)(p.v0[1] + ((k >> 1) & 1));
  const uint32_t vz = (uint32_t)(p.v0[2] + ((k >> 2) & 1));
  const uint32_t side = (uint32_t)N + 1u;
  return dense ? vx + side * (vy + side * vz) : ((vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u)) & Tmask;
}

__device__ __forceinline__ float corner_weight(const CellPos &p, int k) {
  const float wx = (k & 1) ? p.f[0] : 1.0f - p.f[0];
  const float wy = (k & 2) ? p.f[1] : 1.0f - p.f[1];
  const float wz = (k & 4) ? p.f[2] : 1.0f - p.f[2];
  return wx * wy * wz;
}

__device__ __forceinline__ void level_cell(const float x[3], const Box &box, int N, bool dense, uint32_t Tmask,
                                           Corners &c, bool want_grad) {
  const CellPos p = level_pos(x, box, N);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    c.idx[k] = corner_index(p, k, N, dense, Tmask);
    c.w[k] = corner_weight(p, k);
    if (want_grad) {
      const float wx = (k & 1) ? p.f[0] : 1.0f - p.f[0];
      const float wy = (k & 2) ? p.f[1] : 1.0f - p.f[1];
      const float wz = (k & 4) ? p.f[2] : 1.0f - p.f[2];
      c.dw[k][0] = ((k & 1) ? p.sc[0] : -p.sc[0]) * wy * wz;
      c.dw[k][1] = wx * ((k & 2) ? p.sc[1] : -p.sc[1]) * wz;
      c.dw[k][2] = wx * wy * ((k & 4) ? p.sc[2] : -p.sc[2]);
    }
  }
}

__device__ __forceinline__ float2 load_feat2(const float *t, uint32_t i) {
  return reinterpret_cast<const float2 *>(t)[i];
}
__device__ __forceinline__ float2 load_feat2(const __half *t, uint32_t i) {
  return __half22float2(reinterpret_cast<const __half2 *>(t)[i]);
}

// The two x-neighbouring corners (k, k + 1) of a cell are adjacent table
// entries on dense levels, and on hashed levels whenever x + 1 changes the
// index by one (x even: only bit 0 flips; otherwise the flipped low bits can
// still leave the two entries next to each other) -- about two pairs in
// three.  Such a pair is one load of two entries at the lower index (4-byte
// aligned for FP16 entries, 8-byte for FP32: the unaligned access mode of the
// HSA ABI, which the compiler itself assumes).  Any other pair loads the
// aligned two-entry block holding its first corner and the second corner on
// its own.  Every load stays inside the level's table (T is even), and the
// data path returns about 9.5 bytes per FP16 pair instead of a 16-byte block
// of which half was used.  Values are unchanged.
__device__ __forceinline__ float2 h2f(uint32_t a) { return __half22float2(__builtin_bit_cast(__half2, a)); }

// FP16 table (4-byte entries).  The second corner's own load (non-adjacent
// pairs only) sits alone in its branch and both corners are picked after it,
// so no branch waits for a load: the pairs' loads of a cell, and of the
// levels a lane holds, are in flight together.
__device__ __forceinline__ void gather_pair(const __half *t, uint32_t i0, uint32_t i1, float2 &v0, float2 &v1) {
  const uint32_t *t32 = reinterpret_cast<const uint32_t *>(t);
  const bool adj = i1 == i0 + 1u || i0 == i1 + 1u;
  const uint32_t lo = i0 < i1 ? i0 : i1;
  const uint32_t base = adj ? lo : (i0 & ~1u);
  uint2 q;
  __builtin_memcpy(&q, t32 + base, 8);
  uint32_t e1 = 0u;
  if (!adj) e1 = t32[i1];
  const bool first = adj ? i0 == lo : (i0 & 1u) == 0u;
  v0 = h2f(first ? q.x : q.y);
  v1 = h2f(adj ? (first ? q.y : q.x) : e1);
}

// FP32 table (8-byte entries), the same scheme.
__device__ __forceinline__ void gather_pair(const float *t, uint32_t i0, uint32_t i1, float2 &v0, float2 &v1) {
  const float2 *t2 = reinterpret_cast<const float2 *>(t);
  const bool adj = i1 == i0 + 1u || i0 == i1 + 1u;
  const uint32_t lo = i0 < i1 ? i0 : i1;
  const uint32_t base = adj ? lo : (i0 & ~1u);
  float4 q;
  __builtin_memcpy(&q, t2 + base, 16);
  float2 e1 = make_float2(0.0f, 0.0f);
  if (!adj) e1 = t2[i1];
  const bool first = adj ? i0 == lo : (i0 & 1u) == 0u;
  v0 = first ? make_float2(q.x, q.y) : make_float2(q.z, q.w);
  v1 = adj ? (first ? make_float2(q.z, q.w) : make_float2(q.x, q.y)) : e1;
}

// The eight corner values of a cell (table of one level, 16-byte aligned,
// T a multiple of 4).
template <typename TT>
__device__ __forceinline__ void gather8(const TT *tl, const Corners &c, float2 v[8]) {
#pragma unroll
  for (int k = 0; k < 8; k += 2) gather_pair(tl, c.idx[k], c.idx[k + 1], v[k], v[k + 1]);
}

__device__ __forceinline__ void store_feat2(float *f, int64_t i, float a, float b) {
  reinterpret_cast<float2 *>(f)[i] = make_float2(a, b);
}
__device__ __forceinline__ void store_feat2(__hip_bfloat16 *f, int64_t i, float a, float b) {
  __hip_bfloat162 v;
  v.x = __float2bfloat16(a);
  v.y = __float2bfloat16(b);
  reinterpret_cast<__hip_bfloat162 *>(f)[i] = v;
}

// Level l's two features of the point x: the trilinear interpolation of the
// eight corner entries (corners in order k = 0..7).
template <typename TT>
__device__ __forceinline__ void encode_level(const float x[3], const Box &box, int N, bool dense, uint32_t Tmask,
                                             const TT *tl, float *fa, float *fb) {
  Corners c;
  level_cell(x, box, N, dense, Tmask, c, false);
  float2 v[8];
  gather8(tl, c, v);
  float a = 0.0f, b = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a += c.w[k] * v[k].x;
    b += c.w[k] * v[k].y;
  }
  *fa = a;
  *fb = b;
}

// Host side: per-level resolutions and dense flags, and the encoding box.
inline int32_t make_levels(int L, int log2T, double base, double growth, Levels *lv) {
  const uint64_t T = 1ull << log2T;
  for (int l = 0; l < L; ++l) {
    const int N = level_resolution(base, growth, l);
    if (N < 1 || N > (1 << 22)) return IA355_ERR_INVALID_ARG;
    lv->res[l] = N;
    const uint64_t side = (uint64_t)N + 1;
    lv->dense[l] = side * side * side <= T;
  }
  return IA355_OK;
}

inline int32_t make_box(const float *aabb, Box *b) {
  if (!aabb) return IA355_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    if (!(aabb[3 + a] > aabb[a])) return IA355_ERR_INVALID_ARG;
    b->lo[a] = aabb[a];
    b->inv[a] = 1.0f / (aabb[3 + a] - aabb[a]);
  }
  return IA355_OK;
}

}  // namespace hsh
}  // namespace ia355
