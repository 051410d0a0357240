// The learned root initialiser (an addition to the root finding of
// Sec. 3.1): (x', pose) -> nb bone logits and a canonical offset through
// (3 + 6 nb) -> 64 -> 64 -> (nb + 3), shared by the initialiser kernel and
// the fused batch renderer so that both compute the same floats (internal).
// Layer 1's pose part is folded into a per-neuron constant c1 once per pose;
// layers 2 and 3 run on MFMA with the decoder MLP's layouts.
#pragma once
#include <hip/hip_bf16.h>

#include "common.h"

namespace ia355 {
namespace rid {

constexpr int H = 64;        // hidden width
constexpr int kMaxOut = 32;  // nb + 3 outputs in two 16-row MFMA tiles

__device__ __forceinline__ float relu(float z) { return fmaxf(z, 0.0f); }

// Offsets of the flat parameter vector (per layer W [out][in], then b).
struct Layout {
  int nin, nout, offW1, offb1, offW2, offb2, offW3, offb3, total;
};
__host__ __device__ inline Layout layout(int nb) {
  Layout l;
  l.nin = 3 + 6 * nb;
  l.nout = nb + 3;
  l.offW1 = 0;
  l.offb1 = H * l.nin;
  l.offW2 = l.offb1 + H;
  l.offb2 = l.offW2 + H * H;
  l.offW3 = l.offb2 + H;
  l.offb3 = l.offW3 + l.nout * H;
  l.total = l.offb3 + l.nout;
  return l;
}

// n floats of P copied to sP by the block with coalesced 16-byte loads.
__device__ __forceinline__ void stage_copy(const float *__restrict__ P, int n, float *sP) {
  const int head = (int)((4 - (((uintptr_t)P >> 2) & 3)) & 3);  // floats before 16-byte alignment
  const int h = head < n ? head : n;
  for (int i = threadIdx.x; i < h; i += blockDim.x) sP[i] = P[i];
  const int n4 = (n - h) >> 2;
  const float4 *P4 = reinterpret_cast<const float4 *>(P + h);
  for (int i = threadIdx.x; i < n4; i += blockDim.x) {
    const float4 q = P4[i];
    sP[h + 4 * i] = q.x;
    sP[h + 4 * i + 1] = q.y;
    sP[h + 4 * i + 2] = q.z;
    sP[h + 4 * i + 3] = q.w;
  }
  for (int i = h + 4 * n4 + threadIdx.x; i < n; i += blockDim.x) sP[i] = P[i];
}

// c1[n] = W1[n, 3:] . pose + b1[n] by 256 threads (four per neuron, each a
// strided quarter of the pose terms in four independent partial sums,
// combined across the four lanes).  P may be in LDS or global memory.
__device__ __forceinline__ void fold_pose(const float *P, const Layout &l, const float *pose, int nb, float *c1) {
  const int n = (threadIdx.x >> 2) & (H - 1), q = threadIdx.x & 3;
  const float *wrow = P + l.offW1 + n * l.nin + 3;
  const int np = 6 * nb;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  int i = q;
  for (; i + 12 < np; i += 16) {
    a0 += wrow[i] * pose[i];
    a1 += wrow[i + 4] * pose[i + 4];
    a2 += wrow[i + 8] * pose[i + 8];
    a3 += wrow[i + 12] * pose[i + 12];
  }
  for (; i < np; i += 4) a0 += wrow[i] * pose[i];
  float acc = (a0 + a1) + (a2 + a3);
  acc += __shfl_xor(acc, 1, kWave);
  acc += __shfl_xor(acc, 2, kWave);
  if (q == 0 && threadIdx.x < 4 * H) c1[n] = acc + P[l.offb1 + n];
}

// Weight fragments of layers 2 and 3 of lane (r, g).
template <bool BF16>
struct Frag {
  float w2f[4][16], w3f[2][16];
  bf16x8 w2b[4][2], w3b[2][2];
  float b2[4][4], b3[2][4];
};

// Parameter index of lane (r, g)'s operand element: layer 2 (FP32 k = 4t + i,
// BF16 (c, j)) of output tile mt, layer 3 likewise (-1: a padded row, zero).
__host__ __device__ inline int w2f_at(const Layout &l, int mt, int k, int r, int g) {
  return l.offW2 + (16 * mt + r) * H + 16 * (k / 4) + 4 * g + (k % 4);
}
__host__ __device__ inline int w2b_at(const Layout &l, int mt, int c, int j, int r, int g) {
  return l.offW2 + (16 * mt + r) * H + 16 * (2 * c + j / 4) + 4 * g + (j % 4);
}
__host__ __device__ inline int w3f_at(const Layout &l, int mt, int k, int r, int g) {
  const int row = 16 * mt + r;
  return row < l.nout ? l.offW3 + row * H + 16 * (k / 4) + 4 * g + (k % 4) : -1;
}
__host__ __device__ inline int w3b_at(const Layout &l, int mt, int c, int j, int r, int g) {
  const int row = 16 * mt + r;
  return row < l.nout ? l.offW3 + row * H + 16 * (2 * c + j / 4) + 4 * g + (j % 4) : -1;
}

template <bool BF16>
__device__ __forceinline__ void load_frag(const float *sP, const Layout &l, int r, int g, Frag<BF16> &f) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) f.b2[mt][i] = sP[l.offb2 + 16 * mt + 4 * g + i];
    if (!BF16) {
#pragma unroll
      for (int k = 0; k < 16; ++k) f.w2f[mt][k] = sP[w2f_at(l, mt, k, r, g)];
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) f.w2b[mt][c][j] = (__bf16)sP[w2b_at(l, mt, c, j, r, g)];
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) f.b3[mt][i] = (16 * mt + 4 * g + i) < l.nout ? sP[l.offb3 + 16 * mt + 4 * g + i] : 0.0f;
    if (!BF16) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = w3f_at(l, mt, k, r, g);
        f.w3f[mt][k] = i >= 0 ? sP[i] : 0.0f;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int i = w3b_at(l, mt, c, j, r, g);
          f.w3b[mt][c][j] = (__bf16)(i >= 0 ? sP[i] : 0.0f);
        }
    }
  }
}

// BF16 fragment q (0-7: layer 2 (mt, c) = (q / 2, q % 2); 8-11: layer 3
// (mt, c) = ((q - 8) / 2, q % 2)) of lane (r, g), built alone (the same
// values as load_frag<true>).
__device__ __forceinline__ bf16x8 frag_bf(const float *P, const Layout &l, int q, int r, int g) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = q < 8 ? w2b_at(l, q / 2, q % 2, j, r, g) : w3b_at(l, (q - 8) / 2, q % 2, j, r, g);
    v[j] = (__bf16)(i >= 0 ? P[i] : 0.0f);
  }
  return v;
}

// Layers 2-3 and the argmax of one 16-sample tile from the layer-1
// activations h1 (lane r + 16 g holds neurons 16t + 4g + i of sample r),
// with the weight fragments from a source: w.w2f(mt, k) / w.w3f(mt, k)
// (FP32 16x16x4 operands), w.w2b(mt, c) / w.w3b(mt, c) (BF16 16x16x32
// operands), w.b2(mt) / w.b3(mt) (accumulator initialisers).  The bone
// (ties: the lowest) and the three offsets land in every lane of sample r.
template <bool BF16, class WSrc>
__device__ __forceinline__ void tile_tail(const float h1[4][4], const WSrc &w, int nb, int g, int *bone,
                                          float off_out[3]) {
  f32x4 z2[4], o[2];
  if (!BF16) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = w.b2(mt);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w2f(mt, 4 * t + i), h1[t][i], acc, 0, 0, 0);
      z2[mt] = acc;
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x4 acc = w.b3(mt);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w3f(mt, 4 * t + i), relu(z2[t][i]), acc, 0, 0, 0);
      o[mt] = acc;
    }
  } else {
    bf16x8 ha, hb;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ha[j] = (__bf16)h1[j / 4][j % 4];
      hb[j] = (__bf16)h1[2 + j / 4][j % 4];
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = w.b2(mt);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.w2b(mt, 0), ha, acc, 0, 0, 0);
      z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.w2b(mt, 1), hb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ha[j] = (__bf16)relu(z2[j / 4][j % 4]);
      hb[j] = (__bf16)relu(z2[2 + j / 4][j % 4]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x4 acc = w.b3(mt);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.w3b(mt, 0), ha, acc, 0, 0, 0);
      o[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.w3b(mt, 1), hb, acc, 0, 0, 0);
    }
  }
  // argmax over the bone logits (output index 16 mt + 4 g + i < nb), ties to
  // the lowest index; offsets are outputs nb, nb + 1, nb + 2
  float best = -INFINITY, off[3] = {0.0f, 0.0f, 0.0f};
  int bi = 0x7fffffff;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = 16 * mt + 4 * g + i;
      const float v = o[mt][i];
      if (idx < nb && (v > best || (v == best && idx < bi))) {
        best = v;
        bi = idx;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (idx == nb + a) off[a] = v;
    }
#pragma unroll
  for (int m = 16; m < 64; m <<= 1) {
    const float v2 = __shfl_xor(best, m, 64);
    const int i2 = __shfl_xor(bi, m, 64);
    if (v2 > best || (v2 == best && i2 < bi)) {
      best = v2;
      bi = i2;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) off[a] += __shfl_xor(off[a], m, 64);
  }
  *bone = bi;
  off_out[0] = off[0];
  off_out[1] = off[1];
  off_out[2] = off[2];
}

// Layer 1 on the VALU: lane r + 16 g holds neurons 16t + 4g + i of sample
// r (point x); c1 [64] and w1x [64][3] in LDS or global memory.
__device__ __forceinline__ void layer1(const float x[3], const float *c1, const float *w1x, int g, float h1[4][4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 16 * t + 4 * g + i;
      h1[t][i] = relu(c1[n] + w1x[3 * n] * x[0] + w1x[3 * n + 1] * x[1] + w1x[3 * n + 2] * x[2]);
    }
}

// Fragments held in registers (Frag).
template <bool BF16>
struct RegFrag {
  const Frag<BF16> &f;
  __device__ __forceinline__ float w2f(int mt, int k) const { return f.w2f[mt][k]; }
  __device__ __forceinline__ float w3f(int mt, int k) const { return f.w3f[mt][k]; }
  __device__ __forceinline__ bf16x8 w2b(int mt, int c) const { return f.w2b[mt][c]; }
  __device__ __forceinline__ bf16x8 w3b(int mt, int c) const { return f.w3b[mt][c]; }
  __device__ __forceinline__ f32x4 b2(int mt) const {
    return f32x4{f.b2[mt][0], f.b2[mt][1], f.b2[mt][2], f.b2[mt][3]};
  }
  __device__ __forceinline__ f32x4 b3(int mt) const {
    return f32x4{f.b3[mt][0], f.b3[mt][1], f.b3[mt][2], f.b3[mt][3]};
  }
};

// BF16 fragments of layers 2-3 read from LDS as each MFMA needs them:
// rw[q][lane] is fragment q of lane (lane % 16, lane / 16) (q as frag_bf:
// 0-7 layer 2, 8-11 layer 3), rb2 [64] and rb3 [kMaxOut] the biases
// (16-byte aligned, rb3 zero past nb + 3).
struct LdsFragW {
  const bf16x8 (*rw)[kWave];
  const float *rb2, *rb3;
  int lane, g;
  __device__ __forceinline__ float w2f(int, int) const { return 0.0f; }
  __device__ __forceinline__ float w3f(int, int) const { return 0.0f; }
  __device__ __forceinline__ bf16x8 w2b(int mt, int c) const { return rw[2 * mt + c][lane]; }
  __device__ __forceinline__ bf16x8 w3b(int mt, int c) const { return rw[8 + 2 * mt + c][lane]; }
  __device__ __forceinline__ f32x4 b2(int mt) const { return *reinterpret_cast<const f32x4 *>(rb2 + 16 * mt + 4 * g); }
  __device__ __forceinline__ f32x4 b3(int mt) const { return *reinterpret_cast<const f32x4 *>(rb3 + 16 * mt + 4 * g); }
};

// The block fills an LdsFragW's arrays from the parameters P (global
// memory), one fragment per thread at a time.
__device__ __forceinline__ void stage_frag_lds(const float *__restrict__ P, const Layout &l, bf16x8 (*rw)[kWave],
                                               float *rb2, float *rb3) {
  // a fragment's elements j = 0..3 and 4..7 are consecutive parameters at
  // 16-byte aligned offsets: two 16-byte loads when P is 16-byte aligned
  const bool al = ((uintptr_t)P & 15) == 0;
  for (int e = threadIdx.x; e < 12 * kWave; e += blockDim.x) {
    const int q = e / kWave, ln = e % kWave, r = ln & 15, g = ln >> 4;
    if (al) {
      bf16x8 v;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = q < 8 ? w2b_at(l, q / 2, q % 2, 4 * h, r, g) : w3b_at(l, (q - 8) / 2, q % 2, 4 * h, r, g);
        const float4 p4 = i >= 0 ? *reinterpret_cast<const float4 *>(P + i) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        v[4 * h] = (__bf16)p4.x;
        v[4 * h + 1] = (__bf16)p4.y;
        v[4 * h + 2] = (__bf16)p4.z;
        v[4 * h + 3] = (__bf16)p4.w;
      }
      rw[q][ln] = v;
    } else {
      rw[q][ln] = frag_bf(P, l, q, r, g);
    }
  }
  for (int i = threadIdx.x; i < H; i += blockDim.x) rb2[i] = P[l.offb2 + i];
  for (int i = threadIdx.x; i < kMaxOut; i += blockDim.x) rb3[i] = i < l.nout ? P[l.offb3 + i] : 0.0f;
}

// One 16-sample tile, called by all 64 lanes of a wave (lane r + 16 g holds
// sample r's point x): the argmax bone (ties: the lowest) and the three
// offsets, in every lane of sample r.  c1 [64] and w1x [64][3] in LDS.
template <bool BF16>
__device__ __forceinline__ void tile(const float x[3], const float *c1, const float *w1x, const Frag<BF16> &f, int nb,
                                     int g, int *bone, float off_out[3]) {
  float h1[4][4];
  layer1(x, c1, w1x, g, h1);
  tile_tail<BF16>(h1, RegFrag<BF16>{f}, nb, g, bone, off_out);
}

// Broyden start point x0 = B_k^{-1} x' + offset (Bi: [M^-1 | -M^-1 t] of
// bone k, row-major 3 x 4).
__device__ __forceinline__ void start_point(const float *Bi, const float x[3], const float off[3], float x0[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    x0[a] = Bi[4 * a] * x[0] + Bi[4 * a + 1] * x[1] + Bi[4 * a + 2] * x[2] + Bi[4 * a + 3] + off[a];
}

}  // namespace rid
}  // namespace ia355
