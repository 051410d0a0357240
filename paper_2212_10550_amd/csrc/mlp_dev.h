// The decoder MLP of Sec. 3.1, Eq. 1-2 (32 -> 64 -> 64 -> 4) in its BF16
// MFMA form, shared by the decoder kernels and the fused batch renderer so
// that both compute the same floats (internal).  Layouts: see mlp.hip.
#pragma once
#include <hip/hip_bf16.h>

#include "common.h"

namespace ia355 {
namespace mlpd {

constexpr int NIN = 32, NH = 64, NOUT = 4;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == 6532, "parameter count");


__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// max(z, 0) as a signed-integer max of the bits: one v_max_i32 (fmaxf
// first quiets its MFMA-produced input, a second instruction).  Every
// non-negative float keeps its bits, every negative one (and -0) gives +0;
// a NaN with the sign bit clear propagates.
__device__ __forceinline__ float relu(float z) {
  const int b = __builtin_bit_cast(int, z);
  return __builtin_bit_cast(float, b > 0 ? b : 0);
}

// Density exp(o0) (clamped at exp(80)) and colour sigmoid(o1..3); the
// sigmoid's reciprocal is the hardware one (1 ulp), not a division.
__device__ __forceinline__ void head(const float o[4], float *sig, float c[3]) {
  *sig = expf(fminf(o[0], 80.0f));
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = __builtin_amdgcn_rcpf(1.0f + expf(-o[1 + k]));
}

// The parameters (26 KB, 16-byte aligned) copied into LDS by the whole block
// with coalesced 16-byte loads; every wave then builds its MFMA fragments
// from LDS instead of gathering them from global memory one value at a time.
__device__ __forceinline__ void stage_params(const float *__restrict__ P, float *sP) {
  static_assert(NPARAM % 4 == 0, "parameter block in whole float4s");
  const float4 *P4 = reinterpret_cast<const float4 *>(P);
  float4 *s4 = reinterpret_cast<float4 *>(sP);
  for (int e = threadIdx.x; e < NPARAM / 4; e += blockDim.x) s4[e] = P4[e];
}

// --------------------------------------------------------------- BF16 fwd
__device__ __forceinline__ bf16x8 load_x_bf16(const __hip_bfloat16 *feat, int64_t fst, int64_t s, int g, bool ok) {
  bf16x8 x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t v = 0;
    if (ok) v = reinterpret_cast<const uint32_t *>(feat)[(int64_t)(4 * g + j) * fst + s];
    x[2 * j] = __builtin_bit_cast(__bf16, (uint16_t)(v & 0xffffu));
    x[2 * j + 1] = __builtin_bit_cast(__bf16, (uint16_t)(v >> 16));
  }
  return x;
}

struct FragBf {
  bf16x8 w1[4];     // [mt]: W1[16mt + r][8g + j]
  bf16x8 w2[4][2];  // [mt][c]: W2[16mt + r][16(2c + j/4) + 4g + j%4]
  bf16x8 w3[2];     // [c]: W3[r][...] (r < 4)
  float b1[4][4], b2[4][4], b3[4];
};

// Parameter index of element j of lane (r, g)'s fragments (-1: zero).
__host__ __device__ inline int w1_at(int mt, int r, int g, int j) { return OFF_W1 + (16 * mt + r) * NIN + 8 * g + j; }
__host__ __device__ inline int w2_at(int mt, int c, int r, int g, int j) {
  return OFF_W2 + (16 * mt + r) * NH + 16 * (2 * c + j / 4) + 4 * g + (j % 4);
}
__host__ __device__ inline int w3_at(int c, int r, int g, int j) {
  return r < NOUT ? OFF_W3 + r * NH + 16 * (2 * c + j / 4) + 4 * g + (j % 4) : -1;
}
__device__ __forceinline__ __bf16 frag_value(const float *P, int i) { return (__bf16)(i >= 0 ? P[i] : 0.0f); }

__device__ __forceinline__ void load_frag_bf(const float *P, int r, int g, FragBf &f) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int j = 0; j < 8; ++j) f.w1[mt][j] = frag_value(P, w1_at(mt, r, g, j));
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) f.w2[mt][c][j] = frag_value(P, w2_at(mt, c, r, g, j));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f.b1[mt][i] = P[OFF_B1 + 16 * mt + 4 * g + i];
      f.b2[mt][i] = P[OFF_B2 + 16 * mt + 4 * g + i];
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) f.w3[c][j] = frag_value(P, w3_at(c, r, g, j));
#pragma unroll
  for (int i = 0; i < 4; ++i) f.b3[i] = (4 * g + i) < NOUT ? P[OFF_B3 + 4 * g + i] : 0.0f;
}

// Fragment q (0-3: w1[q], 4-11: w2[(q-4)/2][(q-4)%2], 12-13: w3[q-12]) of
// lane (r, g), built alone (the same values as load_frag_bf).
__device__ __forceinline__ bf16x8 frag_bf(const float *P, int q, int r, int g) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = q < 4 ? w1_at(q, r, g, j) : (q < 12 ? w2_at((q - 4) / 2, (q - 4) % 2, r, g, j) : w3_at(q - 12, r, g, j));
    v[j] = frag_value(P, i);
  }
  return v;
}

// First parameter of half h (elements 4h .. 4h + 3, consecutive parameters)
// of fragment q of lane (r, g); -1: a zero half.
__host__ __device__ inline int frag_half_at(int q, int r, int g, int h) {
  return q < 4 ? w1_at(q, r, g, 4 * h) : (q < 12 ? w2_at((q - 4) / 2, (q - 4) % 2, r, g, 4 * h) : w3_at(q - 12, r, g, 4 * h));
}

// The BF16 decoder's fragments in LDS, one 16-byte slot per lane so that a
// wave reads a fragment with one conflict-free load: mw[q][lane] holds
// fragment q (0-3 layer 1, 4 + 2 mt + c layer 2, 12 + c layer 3) of lane
// (lane % 16, lane / 16); b1, b2, b3 the biases.
struct FragLds {
  bf16x8 mw[14][64];
  float b1[NH], b2[NH], b3[NOUT];
};
static_assert(offsetof(FragLds, b1) % 16 == 0 && offsetof(FragLds, b2) % 16 == 0 && offsetof(FragLds, b3) % 16 == 0,
              "16-byte bias vectors");

// A whole block fills the store from the parameters in global memory (16-byte
// aligned): each fragment is two 16-byte loads of consecutive parameters,
// converted as frag_value converts them.
__device__ __forceinline__ void stage_frag_lds(const float *__restrict__ P, FragLds &s) {
  for (int e = threadIdx.x; e < 14 * 64; e += blockDim.x) {
    const int q = e >> 6, l = e & 63;
    bf16x8 v;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = frag_half_at(q, l & 15, l >> 4, h);
      const float4 p = i >= 0 ? *reinterpret_cast<const float4 *>(P + i) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      v[4 * h] = (__bf16)p.x;
      v[4 * h + 1] = (__bf16)p.y;
      v[4 * h + 2] = (__bf16)p.z;
      v[4 * h + 3] = (__bf16)p.w;
    }
    s.mw[q][l] = v;
  }
  for (int i = threadIdx.x; i < NH; i += blockDim.x) {
    s.b1[i] = P[OFF_B1 + i];
    s.b2[i] = P[OFF_B2 + i];
  }
  if (threadIdx.x < NOUT) s.b3[threadIdx.x] = P[OFF_B3 + threadIdx.x];
}

// Weights fetched from a FragLds as each MFMA needs them.
struct LdsW {
  const FragLds &s;
  int lane, g;
  __device__ __forceinline__ bf16x8 w1(int mt) const { return s.mw[mt][lane]; }
  __device__ __forceinline__ bf16x8 w2(int mt, int c) const { return s.mw[4 + 2 * mt + c][lane]; }
  __device__ __forceinline__ bf16x8 w3(int c) const { return s.mw[12 + c][lane]; }
  __device__ __forceinline__ f32x4 b1(int mt) const { return *reinterpret_cast<const f32x4 *>(s.b1 + 16 * mt + 4 * g); }
  __device__ __forceinline__ f32x4 b2(int mt) const { return *reinterpret_cast<const f32x4 *>(s.b2 + 16 * mt + 4 * g); }
  __device__ __forceinline__ f32x4 b3() const {
    return g == 0 ? *reinterpret_cast<const f32x4 *>(s.b3) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
};

// A compiler-only barrier inside a loop: the LDS fragment reads after it
// cannot be hoisted out of the loop (which would hold every fragment in
// registers again).
__device__ __forceinline__ void pin_in_loop() { asm volatile("" ::: "memory"); }

// Pack the relu'd accumulators of tiles t = 2c, 2c+1 into one B operand.
__device__ __forceinline__ bf16x8 pack_act(const f32x4 z[4], int c) {
  bf16x8 b;
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = (__bf16)relu(z[2 * c + j / 4][j % 4]);
  return b;
}

// The BF16 forward of one 16-sample tile with the weights from a source:
// w.w1(mt), w.w2(mt, c), w.w3(c) give the A-operand fragments and
// w.b1(mt), w.b2(mt), w.b3() the accumulator initialisers (biases), so the
// fragments may live in registers or be fetched from LDS as they are used;
// the operations are the same either way.
template <class WSrc>
__device__ __forceinline__ void fwd_bf_src(const WSrc &w, const bf16x8 &X, f32x4 z1[4], f32x4 z2[4], f32x4 &o) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) z1[mt] = mfma32(w.w1(mt), X, w.b1(mt));
  const bf16x8 h1a = pack_act(z1, 0), h1b = pack_act(z1, 1);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = w.b2(mt);
    acc = mfma32(w.w2(mt, 0), h1a, acc);
    z2[mt] = mfma32(w.w2(mt, 1), h1b, acc);
  }
  const bf16x8 h2a = pack_act(z2, 0), h2b = pack_act(z2, 1);
  f32x4 acc = w.b3();
  acc = mfma32(w.w3(0), h2a, acc);
  o = mfma32(w.w3(1), h2b, acc);
}

// Weights held in registers (FragBf).
struct RegW {
  const FragBf &f;
  __device__ __forceinline__ bf16x8 w1(int mt) const { return f.w1[mt]; }
  __device__ __forceinline__ bf16x8 w2(int mt, int c) const { return f.w2[mt][c]; }
  __device__ __forceinline__ bf16x8 w3(int c) const { return f.w3[c]; }
  __device__ __forceinline__ f32x4 b1(int mt) const {
    return f32x4{f.b1[mt][0], f.b1[mt][1], f.b1[mt][2], f.b1[mt][3]};
  }
  __device__ __forceinline__ f32x4 b2(int mt) const {
    return f32x4{f.b2[mt][0], f.b2[mt][1], f.b2[mt][2], f.b2[mt][3]};
  }
  __device__ __forceinline__ f32x4 b3() const { return f32x4{f.b3[0], f.b3[1], f.b3[2], f.b3[3]}; }
};

__device__ __forceinline__ void fwd_bf(const FragBf &f, const bf16x8 &X, f32x4 z1[4], f32x4 z2[4], f32x4 &o) {
  fwd_bf_src(RegW{f}, X, z1, z2, o);
}

}  // namespace mlpd
}  // namespace ia355
