// Per-sample arithmetic of the root finding (Sec. 3.1, Eq. 5-7), shared by
// the deform kernels and the fused batch renderer so that both compute the
// same floats: the blended transform grid A_v = sum_i W[v][i] B_i, the
// residual g(x) = sum_c tri_c (A_c x_h) - x' and its Jacobian on that grid,
// one Broyden solve and the multi-init search (internal).
#pragma once
#include "common.h"
#include "geometry.h"

namespace ia355 {
namespace dfm {

constexpr int kMaxBones = 64;

struct Grid {
  int D[3];       // Dx, Dy, Dz
  float lo[3];    // box low corner
  float scale[3]; // (D - 1) / (hi - lo)
  uint32_t dc[8]; // byte offset of corner k's transform (k = cx + 2 cy + 4 cz) from its cell's base vertex
};

struct Box {
  float lo[3], hi[3];
};

// A_v of one vertex from its skinning row w [nb] and the bone transforms
// sB [nb][12]: the weighted sum over bones in bone order.
__device__ __forceinline__ void blend_vertex(const float *w, const float *sB, int nb, float *Av) {
  float acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0f;
  for (int b = 0; b < nb; ++b) {
    const float wb = w[b];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += wb * sB[12 * b + k];
  }
  float4 *out = reinterpret_cast<float4 *>(Av);
  out[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
  out[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
  out[2] = make_float4(acc[8], acc[9], acc[10], acc[11]);
}

// Vertices blk * kBlendBlock ... of the blended grid A, one thread per
// vertex (a block of kBlendBlock threads).  The block's nb-float skinning
// rows are contiguous in W, so the block first copies them into LDS with
// coalesced 16-byte loads (a lane walking its own row would touch a
// different cache line per lane and weight), then each thread blends its row
// with the bone transforms.  sB [kMaxBones * 12] and
// sW [kBlendBlock * kBlendMaxBones] are the block's LDS.
constexpr int kBlendBlock = 256;
constexpr int kBlendMaxBones = 32;  // LDS rows: 256 x 32 floats = 32 KB
__device__ __forceinline__ void blend_block(const float *__restrict__ W, const float *__restrict__ B, int nb,
                                            int64_t nvert, float *__restrict__ A, int64_t blk, float *sB, float *sW) {
  for (int i = threadIdx.x; i < nb * 12; i += blockDim.x) sB[i] = B[i];
  const int64_t v0 = blk * kBlendBlock;
  const int64_t nv = nvert - v0 < kBlendBlock ? nvert - v0 : kBlendBlock;
  const bool staged = nb <= kBlendMaxBones;
  if (staged) {
    // the block's rows: nv * nb floats starting at W + v0 * nb
    const float *src = W + v0 * nb;
    const int64_t n = nv * nb;
    const int64_t head = (int64_t)((4 - (((uintptr_t)src >> 2) & 3)) & 3);  // floats before 16-byte alignment
    const int64_t h = head < n ? head : n;
    for (int64_t i = threadIdx.x; i < h; i += blockDim.x) sW[i] = src[i];
    const int64_t n4 = (n - h) >> 2;
    const float4 *src4 = reinterpret_cast<const float4 *>(src + h);
    for (int64_t i = threadIdx.x; i < n4; i += blockDim.x) {
      const float4 q = src4[i];
      sW[h + 4 * i] = q.x;
      sW[h + 4 * i + 1] = q.y;
      sW[h + 4 * i + 2] = q.z;
      sW[h + 4 * i + 3] = q.w;
    }
    for (int64_t i = h + 4 * n4 + threadIdx.x; i < n; i += blockDim.x) sW[i] = src[i];
  }
  __syncthreads();
  const int64_t v = v0 + threadIdx.x;
  if (threadIdx.x < nv) blend_vertex(staged ? sW + (int64_t)threadIdx.x * nb : W + v * nb, sB, nb, A + 12 * v);
}

// Cell lookup with align-corners vertices and clamping to the box: base
// vertex, fractional position and d(p)/dx (zero along a clamped axis).
struct Cell {
  int i0[3];
  float f[3];
  float dp[3];
};

__device__ __forceinline__ Cell locate(const Grid &g, const float x[3]) {
  Cell c;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float p = (x[a] - g.lo[a]) * g.scale[a];
    float s = g.scale[a];
    const float pmax = (float)(g.D[a] - 1);
    if (!(p >= 0.0f)) { p = 0.0f; s = 0.0f; }  // also catches NaN
    if (p > pmax) { p = pmax; s = 0.0f; }
    int i = (int)floorf(p);
    i = i > g.D[a] - 2 ? g.D[a] - 2 : i;
    i = i < 0 ? 0 : i;
    c.i0[a] = i;
    c.f[a] = p - (float)i;
    c.dp[a] = s;
  }
  return c;
}

// Base vertex of a cell.  The blended grid holds fewer than 2^32 / 48
// vertices (checked on the host), so vertex and byte offsets are 32-bit and
// every corner load is a uniform base plus one 32-bit lane offset.
// (byte offset of the base vertex's 12 floats)
__device__ __forceinline__ uint32_t cell_base(const Grid &g, const Cell &c) {
  return (((uint32_t)c.i0[2] * (uint32_t)g.D[1] + (uint32_t)c.i0[1]) * (uint32_t)g.D[0] + (uint32_t)c.i0[0]) * 48u;
}

__device__ __forceinline__ const float4 *corner_ptr(const float *A, const Grid &g, uint32_t base, int k) {
  return reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(A) + (base + g.dc[k]));
}

// Trilinear weights of the eight corners (k = cx + 2 cy + 4 cz).
__device__ __forceinline__ void tri_weights(const float f[3], float t[8]) {
  const float gx = 1.0f - f[0], gy = 1.0f - f[1], gz = 1.0f - f[2];
  const float a00 = gy * gz, a10 = f[1] * gz, a01 = gy * f[2], a11 = f[1] * f[2];
  t[0] = gx * a00;
  t[1] = f[0] * a00;
  t[2] = gx * a10;
  t[3] = f[0] * a10;
  t[4] = gx * a01;
  t[5] = f[0] * a01;
  t[6] = gx * a11;
  t[7] = f[0] * a11;
}

// g = (sum_c tri_c A_c) x_h - x': the 12 blended channels are interpolated
// first, then applied to x_h once.
__device__ __forceinline__ void residual(const float *__restrict__ A, const Grid &gr, const float x[3],
                                         const float xp[3], float g[3]) {
  const Cell c = locate(gr, x);
  const uint32_t base = cell_base(gr, c);
  float t[8];
  tri_weights(c.f, t);
  float4 m0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), m1 = m0, m2 = m0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 *p = corner_ptr(A, gr, base, k);
    const float4 r0 = p[0], r1 = p[1], r2 = p[2];
    m0.x += t[k] * r0.x; m0.y += t[k] * r0.y; m0.z += t[k] * r0.z; m0.w += t[k] * r0.w;
    m1.x += t[k] * r1.x; m1.y += t[k] * r1.y; m1.z += t[k] * r1.z; m1.w += t[k] * r1.w;
    m2.x += t[k] * r2.x; m2.y += t[k] * r2.y; m2.z += t[k] * r2.z; m2.w += t[k] * r2.w;
  }
  g[0] = (m0.x * x[0] + m0.y * x[1] + m0.z * x[2] + m0.w) - xp[0];
  g[1] = (m1.x * x[0] + m1.y * x[1] + m1.z * x[2] + m1.w) - xp[1];
  g[2] = (m2.x * x[0] + m2.y * x[1] + m2.z * x[2] + m2.w) - xp[2];
}

// Derivatives of a trilinear interpolant along its cell axes, from the
// eight corner values v[c] (c = cx + 2 cy + 4 cz) and the fractions f:
// differences of neighbouring corners are taken first, so the result does
// not cancel when the corner values are close (they are smooth fields).
__device__ __forceinline__ void tri_grad(const float v[8], const float f[3], float d[3]) {
  const float gx = 1.0f - f[0], gy = 1.0f - f[1], gz = 1.0f - f[2];
  d[0] = gy * gz * (v[1] - v[0]) + f[1] * gz * (v[3] - v[2]) + gy * f[2] * (v[5] - v[4]) + f[1] * f[2] * (v[7] - v[6]);
  d[1] = gx * gz * (v[2] - v[0]) + f[0] * gz * (v[3] - v[1]) + gx * f[2] * (v[6] - v[4]) + f[0] * f[2] * (v[7] - v[5]);
  d[2] = gx * gy * (v[4] - v[0]) + f[0] * gy * (v[5] - v[1]) + gx * f[1] * (v[6] - v[2]) + f[0] * f[1] * (v[7] - v[3]);
}

__device__ __forceinline__ float tri_weight(const float f[3], int k) {
  return ((k & 1) ? f[0] : 1.0f - f[0]) * ((k & 2) ? f[1] : 1.0f - f[1]) * ((k & 4) ? f[2] : 1.0f - f[2]);
}

// Residual and Jacobian: with y_c = A_c x_h, g = sum_c tri_c y_c - x' and
// J = sum_c tri_c M_c + (d/dx of the interpolant of y_c at fixed x_h).
__device__ __forceinline__ void residual_jac(const float *__restrict__ A, const Grid &gr, const float x[3],
                                             const float xp[3], float g[3], float J[3][3]) {
  const Cell c = locate(gr, x);
  const uint32_t base = cell_base(gr, c);
  float y[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) J[i][j] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 *p = corner_ptr(A, gr, base, k);
    const float4 r[3] = {p[0], p[1], p[2]};
    const float t = tri_weight(c.f, k);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      y[i][k] = r[i].x * x[0] + r[i].y * x[1] + r[i].z * x[2] + r[i].w;
      J[i][0] += t * r[i].x;
      J[i][1] += t * r[i].y;
      J[i][2] += t * r[i].z;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float d[3];
    tri_grad(y[i], c.f, d);
    g[i] = -xp[i];
#pragma unroll
    for (int k = 0; k < 8; ++k) g[i] += tri_weight(c.f, k) * y[i][k];
#pragma unroll
    for (int j = 0; j < 3; ++j) J[i][j] += c.dp[j] * d[j];
  }
}

__device__ __forceinline__ float norm3(const float v[3]) { return sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

constexpr int kSolveBlock = 256;
// kGroup lanes share one posed sample; lane j runs inits j, j + kGroup, ...
// (3 of the 24 bones each), then the group selects the lowest residual by
// shuffles.  Many more threads than samples keep the CUs busy at the
// training-step sample counts (tens of thousands).
constexpr int kGroup = 8;

struct InitResult {
  float x[3];
  float r;
  bool ok;
  int steps;
};

// One Broyden solve from the start point x (H0 = J(x)^{-1}).
__device__ __forceinline__ InitResult broyden_from(const float *__restrict__ A, const Grid &gr, float x[3], bool start_ok,
                                                  const float xp[3], int max_iter, float tol_stop) {
  InitResult res;
  const bool bone_ok = start_ok;
  float g[3], J[3][3], H[3][3];
  residual_jac(A, gr, x, xp, g, J);
  const float detJ = inv3(J, H);
  bool ok = bone_ok && fabsf(detJ) >= 1e-12f;
  int k = 0;
  const float tol2 = tol_stop * tol_stop;
  if (ok) {
    for (; k < max_iter; ++k) {
      if (g[0] * g[0] + g[1] * g[1] + g[2] * g[2] < tol2) break;
      float dx[3], xn[3], gn[3], dg[3], Hdg[3], dxH[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) dx[a] = -(H[a][0] * g[0] + H[a][1] * g[1] + H[a][2] * g[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) xn[a] = x[a] + dx[a];
      residual(A, gr, xn, xp, gn);
#pragma unroll
      for (int a = 0; a < 3; ++a) dg[a] = gn[a] - g[a];
#pragma unroll
      for (int a = 0; a < 3; ++a) Hdg[a] = H[a][0] * dg[0] + H[a][1] * dg[1] + H[a][2] * dg[2];
#pragma unroll
      for (int b = 0; b < 3; ++b) dxH[b] = dx[0] * H[0][b] + dx[1] * H[1][b] + dx[2] * H[2][b];
      const float den = dx[0] * Hdg[0] + dx[1] * Hdg[1] + dx[2] * Hdg[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[a] = xn[a];
        g[a] = gn[a];
      }
      if (fabsf(den) < 1e-30f) {
        ok = false;
        ++k;
        break;
      }
      const float iden = __builtin_amdgcn_rcpf(den);  // 1 ulp: H is an approximation of J^-1 anyway
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] += (dx[a] - Hdg[a]) * dxH[b] * iden;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) res.x[a] = x[a];
  res.r = norm3(g);
  res.ok = ok;
  res.steps = k;
  return res;
}

// One Broyden solve from bone init i: x0 = B_i^{-1} x'.
__device__ __forceinline__ InitResult broyden(const float *__restrict__ A, const Grid &gr, const float *Bi, bool bone_ok,
                                             const float xp[3], int max_iter, float tol_stop) {
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = Bi[4 * a] * xp[0] + Bi[4 * a + 1] * xp[1] + Bi[4 * a + 2] * xp[2] + Bi[4 * a + 3];
  return broyden_from(A, gr, x, bone_ok, xp, max_iter, tol_stop);
}

__device__ __forceinline__ bool in_hbox(const float x[3], const Box &b) {
  return x[0] >= b.lo[0] && x[0] <= b.hi[0] && x[1] >= b.lo[1] && x[1] <= b.hi[1] && x[2] >= b.lo[2] &&
         x[2] <= b.hi[2];
}

// Multi-init solve of one sample by a group of kGroup lanes (j = lane in
// group): lowest valid residual, ties to the lowest bone.  Every lane of the
// group returns the group's result; steps are summed over the inits.
struct Choice {
  float x[3], r, x0[3];
  int bone, steps;
};

template <int kG = kGroup>
__device__ __forceinline__ Choice multi_init(const float *__restrict__ A, const Grid &gr, const float *sBinv,
                                             const int *sBok, int nb, const float xp[3], bool act, int j, Box hbox,
                                             int max_iter, float tol_stop, float tol_valid) {
  float best_r = INFINITY, best_x[3] = {0.0f, 0.0f, 0.0f}, x0[3] = {0.0f, 0.0f, 0.0f};
  int best = 0x7fffffff, steps = 0;
  if (act) {
    for (int i = j; i < nb; i += kG) {
      const InitResult q = broyden(A, gr, sBinv + 12 * i, sBok[i], xp, max_iter, tol_stop);
      steps += q.steps;
      if (i == 0) {
        x0[0] = q.x[0];
        x0[1] = q.x[1];
        x0[2] = q.x[2];
      }
      if (q.ok && q.r < tol_valid && in_hbox(q.x, hbox) && q.r < best_r) {
        best_r = q.r;
        best = i;
        best_x[0] = q.x[0];
        best_x[1] = q.x[1];
        best_x[2] = q.x[2];
      }
    }
  }
#pragma unroll
  for (int o = kG / 2; o > 0; o >>= 1) {
    const float r2 = __shfl_xor(best_r, o, kG);
    const int b2 = __shfl_xor(best, o, kG);
    const float x20 = __shfl_xor(best_x[0], o, kG);
    const float x21 = __shfl_xor(best_x[1], o, kG);
    const float x22 = __shfl_xor(best_x[2], o, kG);
    steps += __shfl_xor(steps, o, kG);
    if (r2 < best_r || (r2 == best_r && b2 < best)) {
      best_r = r2;
      best = b2;
      best_x[0] = x20;
      best_x[1] = x21;
      best_x[2] = x22;
    }
  }
  Choice c;
  const bool valid = best != 0x7fffffff;
  // the group's first lane ran init 0: its final iterate stands for invalid samples
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c.x[a] = best_x[a];
    c.x0[a] = x0[a];
  }
  c.r = valid ? best_r : INFINITY;
  c.bone = valid ? best : -1;
  c.steps = steps;
  return c;
}

__device__ __forceinline__ void write_choice(const Choice &c, int64_t n, int64_t ld, int extra_steps, float *xc_soa,
                                             int16_t *bone_out, float *resid_out, int16_t *steps_out) {
  const bool valid = c.bone >= 0;
  xc_soa[n] = valid ? c.x[0] : c.x0[0];
  xc_soa[ld + n] = valid ? c.x[1] : c.x0[1];
  xc_soa[2 * ld + n] = valid ? c.x[2] : c.x0[2];
  bone_out[n] = (int16_t)c.bone;
  if (resid_out) resid_out[n] = c.r;
  if (steps_out) steps_out[n] = (int16_t)(c.steps + extra_steps);
}

inline Grid make_grid(int Dx, int Dy, int Dz, const float *aabb) {
  Grid g;
  g.D[0] = Dx;
  g.D[1] = Dy;
  g.D[2] = Dz;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = aabb[a];
    g.scale[a] = (float)(g.D[a] - 1) / (aabb[3 + a] - aabb[a]);
  }
  const uint32_t sx = 1, sy = (uint32_t)Dx, sz = (uint32_t)Dx * (uint32_t)Dy;
  for (int k = 0; k < 8; ++k) g.dc[k] = 48u * (((k & 1) ? sx : 0) + ((k & 2) ? sy : 0) + ((k & 4) ? sz : 0));
  return g;
}

inline bool grid_ok(int Dx, int Dy, int Dz, const float *aabb) {
  if (Dx < 2 || Dy < 2 || Dz < 2 || !aabb) return false;
  if ((int64_t)Dx * Dy * Dz * 48 >= ((int64_t)1 << 32)) return false;  // 32-bit byte offsets into the blended grid
  for (int a = 0; a < 3; ++a)
    if (!(aabb[3 + a] > aabb[a])) return false;
  return true;
}

}  // namespace dfm
}  // namespace ia355
