// Decoder MLP 32 -> 64 -> 64 -> 4 (Sec. 3.1, Eq. 1-2: the shallow MLP that
// turns concatenated hash features into density and colour) on MFMA.
//
// Layer products are out[m][n] = sum_k W[m][k] in[k][n] with m = neuron,
// n = sample (16 per tile), k = input.  One wave owns a 16-sample tile.
// MFMA operand layouts (lane l, r = l % 16, g = l / 16):
//   v_mfma_f32_16x16x4_f32   : A[r][g], B[g][r] (one value each), D[4g+i][r]
//   v_mfma_f32_16x16x32_bf16 : A[r][8g+j], B[8g+j][r] (8 bf16 each), D[4g+i][r]
// A lane therefore ends a layer holding neurons {16t + 4g + i} of sample r.
// The next layer consumes exactly those registers as its B operand by
// ordering its K dimension the same way (k-step (t, i), slot g = neuron
// 16t + 4g + i); its weight fragments are gathered in that order.  So the
// activations never leave registers between layers.  Features arrive
// level-major [L][S][2]: lane group g reads levels 4g..4g+3 of its sample,
// i.e. features 8g..8g+7, which fixes the K order of the first layer.
#include <hip/hip_bf16.h>

#include "common.h"
#include "mlp_dev.h"

using namespace ia355;
using namespace ia355::mlpd;

namespace {

// --------------------------------------------------------------- FP32 fwd
// Loads the 8 features of lane group g for sample s (levels 4g..4g+3).
__device__ __forceinline__ void load_x(const float *feat, int64_t fst, int64_t s, int g, bool ok, float X[8]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float2 v = make_float2(0.0f, 0.0f);
    if (ok) v = reinterpret_cast<const float2 *>(feat)[(int64_t)(4 * g + j) * fst + s];
    X[2 * j] = v.x;
    X[2 * j + 1] = v.y;
  }
}

struct Frag32 {
  float w1[4][8];   // [mt][c]  = W1[16mt + r][8g + c]
  float w2[4][16];  // [mt][4t+i] = W2[16mt + r][16t + 4g + i]
  float w3[16];     // [4t+i]   = W3[r][16t + 4g + i] (r < 4)
  float b1[4][4], b2[4][4], b3[4];  // [mt][i] = b[16mt + 4g + i]
};

__device__ __forceinline__ void load_frag32(const float *P, int r, int g, Frag32 &f) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int c = 0; c < 8; ++c) f.w1[mt][c] = P[OFF_W1 + (16 * mt + r) * NIN + 8 * g + c];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) f.w2[mt][4 * t + i] = P[OFF_W2 + (16 * mt + r) * NH + 16 * t + 4 * g + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f.b1[mt][i] = P[OFF_B1 + 16 * mt + 4 * g + i];
      f.b2[mt][i] = P[OFF_B2 + 16 * mt + 4 * g + i];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) f.w3[4 * t + i] = r < NOUT ? P[OFF_W3 + r * NH + 16 * t + 4 * g + i] : 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) f.b3[i] = (4 * g + i) < NOUT ? P[OFF_B3 + 4 * g + i] : 0.0f;
}

// Forward of one tile; z1/z2 are pre-activations, o the 4 outputs (valid in
// lanes g == 0).
__device__ __forceinline__ void fwd32(const Frag32 &f, const float X[8], f32x4 z1[4], f32x4 z2[4], f32x4 &o) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {f.b1[mt][0], f.b1[mt][1], f.b1[mt][2], f.b1[mt][3]};
#pragma unroll
    for (int c = 0; c < 8; ++c) acc = mfma4(f.w1[mt][c], X[c], acc);
    z1[mt] = acc;
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {f.b2[mt][0], f.b2[mt][1], f.b2[mt][2], f.b2[mt][3]};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = mfma4(f.w2[mt][4 * t + i], relu(z1[t][i]), acc);
    z2[mt] = acc;
  }
  f32x4 acc = {f.b3[0], f.b3[1], f.b3[2], f.b3[3]};
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc = mfma4(f.w3[4 * t + i], relu(z2[t][i]), acc);
  o = acc;
}

constexpr int kFwdBlock = 256;
constexpr int kFwdPre = 2;    // tiles whose features are in flight per wave (BF16)
constexpr int kFwdPre32 = 2;  // the same for FP32 features (eight registers a tile)

__global__ void __launch_bounds__(kFwdBlock) mlp_fwd_f32(const float *__restrict__ feat,
                                                         const int16_t *__restrict__ bone, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                         const float *__restrict__ P, float *__restrict__ sigma,
                                                         float *__restrict__ rgb) {
  __shared__ __attribute__((aligned(16))) float sP[NPARAM];
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  S = count_of(S, S_dev);
  const int64_t ntile = ceil_div(S, 16);
  const int64_t wstride = (int64_t)gridDim.x * (kFwdBlock / 64);
  if ((int64_t)blockIdx.x * (kFwdBlock / 64) >= ntile) return;  // the whole block (before the barrier)
  stage_params(P, sP);
  __syncthreads();
  // a wave without a tile skips the fragment loads (no barriers after this)
  if ((int64_t)blockIdx.x * (kFwdBlock / 64) + (threadIdx.x >> 6) >= ntile) return;
  Frag32 f;
  load_frag32(sP, r, g, f);
  // the features and bone of the next kFwdPre32 tiles of this wave are in
  // flight while a tile computes (a tile's MFMA chain is far shorter than
  // a load's latency)
  const int64_t tile0 = (int64_t)blockIdx.x * (kFwdBlock / 64) + (threadIdx.x >> 6);
  float Xq[kFwdPre32][8];
  int Bq[kFwdPre32];
#pragma unroll
  for (int u = 0; u < kFwdPre32; ++u) {
    const int64_t su = (tile0 + u * wstride) * 16 + r;
    const bool okn = tile0 + u * wstride < ntile && su < S;
    load_x(feat, ld, su, g, okn, Xq[u]);
    Bq[u] = okn && bone && g == 0 ? bone[su] : 0;
  }
  for (int64_t tile = tile0; tile < ntile; tile += kFwdPre32 * wstride) {
#pragma unroll
    for (int u = 0; u < kFwdPre32; ++u) {
      const int64_t tu = tile + u * wstride;
      if (tu >= ntile) break;
      const int64_t s = tu * 16 + r;
      const bool ok = s < S;
      float X[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) X[c] = Xq[u][c];
      const int bn = Bq[u];
      const int64_t tn = tu + kFwdPre32 * wstride, sn = tn * 16 + r;
      const bool okn = tn < ntile && sn < S;
      load_x(feat, ld, sn, g, okn, Xq[u]);
      Bq[u] = okn && bone && g == 0 ? bone[sn] : 0;
      f32x4 z1[4], z2[4], o;
      fwd32(f, X, z1, z2, o);
      if (g == 0 && ok) {
        float sg = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
        if (!bone || bn >= 0) {
          const float ov[4] = {o[0], o[1], o[2], o[3]};
          head(ov, &sg, c);
        }
        sigma[s] = sg;
        rgb[s] = c[0];
        rgb[ld + s] = c[1];
        rgb[2 * ld + s] = c[2];
      }
    }
  }
}

__global__ void __launch_bounds__(kFwdBlock, 4) mlp_fwd_bf16(const __hip_bfloat16 *__restrict__ feat,
                                                          const int16_t *__restrict__ bone, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                          const float *__restrict__ P, float *__restrict__ sigma,
                                                          float *__restrict__ rgb) {
  __shared__ __attribute__((aligned(16))) FragLds sF;
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  S = count_of(S, S_dev);
  const int64_t ntile = ceil_div(S, 16);
  const int64_t wstride = (int64_t)gridDim.x * (kFwdBlock / 64);
  if ((int64_t)blockIdx.x * (kFwdBlock / 64) >= ntile) return;  // the whole block (before the barrier)
  stage_frag_lds(P, sF);
  __syncthreads();
  if ((int64_t)blockIdx.x * (kFwdBlock / 64) + (threadIdx.x >> 6) >= ntile) return;
  // the fragments stay in LDS and are read as each MFMA needs them (held in
  // registers they cost 90 registers a lane, two waves per SIMD)
  // the features and bone of the next kFwdPre tiles of this wave are in
  // flight while a tile computes
  const int64_t tile0 = (int64_t)blockIdx.x * (kFwdBlock / 64) + (threadIdx.x >> 6);
  bf16x8 Xq[kFwdPre];
  int Bq[kFwdPre];
#pragma unroll
  for (int u = 0; u < kFwdPre; ++u) {
    const int64_t su = (tile0 + u * wstride) * 16 + r;
    const bool okn = tile0 + u * wstride < ntile && su < S;
    Xq[u] = load_x_bf16(feat, ld, su, g, okn);
    Bq[u] = okn && bone && g == 0 ? bone[su] : 0;
  }
  for (int64_t tile = tile0; tile < ntile; tile += kFwdPre * wstride) {
#pragma unroll
    for (int u = 0; u < kFwdPre; ++u) {
      const int64_t tu = tile + u * wstride;
      if (tu >= ntile) break;
      const int64_t s = tu * 16 + r;
      const bool ok = s < S;
      const bf16x8 X = Xq[u];
      const int bn = Bq[u];
      const int64_t tn = tu + kFwdPre * wstride, sn = tn * 16 + r;
      const bool okn = tn < ntile && sn < S;
      Xq[u] = load_x_bf16(feat, ld, sn, g, okn);
      Bq[u] = okn && bone && g == 0 ? bone[sn] : 0;
      f32x4 z1[4], z2[4], o;
      pin_in_loop();
      fwd_bf_src(LdsW{sF, lane, g}, X, z1, z2, o);
      if (g == 0 && ok) {
        float sg = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
        if (!bone || bn >= 0) {
          const float ov[4] = {o[0], o[1], o[2], o[3]};
          head(ov, &sg, c);
        }
        sigma[s] = sg;
        rgb[s] = c[0];
        rgb[ld + s] = c[1];
        rgb[2 * ld + s] = c[2];
      }
    }
  }
}

// --------------------------------------------------------------- FP32 bwd
// Per 16-sample tile (one wave): recompute the forward, then
//   d3 = dL/do (exp / sigmoid heads), gh2 = W3^T d3, d2 = gh2 * [z2 >= 0],
//   gh1 = W2^T d2, d1 = gh1 * [z1 >= 0], gfeat = W1^T d1,
//   dW3 += d3 h2^T, dW2 += d2 h1^T, dW1 += d1 x^T, db += sum d.
// The transposed products chain in registers like the forward; the weight
// gradients (K = samples) read tiles transposed through a per-wave LDS
// scratch.  Block partials are reduced in a fixed order.
constexpr int kBwdWaves = 2;
constexpr int kBwdBlock = 64 * kBwdWaves;
constexpr int LDP = 17;  // padded sample stride of the scratch tiles
constexpr int SCR_X = 0, SCR_H1 = SCR_X + 32 * LDP, SCR_H2 = SCR_H1 + 64 * LDP, SCR_D = SCR_H2 + 64 * LDP,
              SCR_D3 = SCR_D + 64 * LDP, SCR_SIZE = SCR_D3 + 4 * LDP;
// transposed-weight fragments in LDS, stored lane-contiguous: [mfma][lane]
constexpr int FT3 = 0;                 // 4 mfma   : W3[g][16mt + r]
constexpr int FT2 = FT3 + 4 * 64;      // 64 mfma  : W2[16t + 4g + i][16mt + r]   (mt, 4t+i)
constexpr int FT1 = FT2 + 64 * 64;     // 32 mfma  : W1[16t + 4g + i][16mt + r]   (mt in 0..1, 4t+i)
constexpr int FT_SIZE = FT1 + 32 * 64;
constexpr int LDS_FLOATS = FT_SIZE + kBwdWaves * SCR_SIZE;
static_assert(kBwdWaves * SCR_SIZE >= NPARAM, "parameters and block partial use the scratch region");
static_assert((FT_SIZE * 4) % 16 == 0, "16-byte aligned scratch region");
static_assert(LDS_FLOATS * 4 <= 65536, "one workgroup's LDS");

__global__ void __launch_bounds__(kBwdBlock) mlp_bwd_f32(const float *__restrict__ gsig, const float *__restrict__ grgb,
                                                         const float *__restrict__ feat,
                                                         const int16_t *__restrict__ bone, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                         const float *__restrict__ P, float *__restrict__ gfeat,
                                                         float *__restrict__ partial) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4, wid = threadIdx.x >> 6;
  float *ft = lds;
  float *scr = lds + FT_SIZE + wid * SCR_SIZE;
  // the parameters go to the scratch region, which the tiles use only after
  // the fragments are built
  float *sP = lds + FT_SIZE;
  stage_params(P, sP);
  __syncthreads();
  // transposed fragments, from the LDS copy
  for (int e = threadIdx.x; e < FT_SIZE; e += kBwdBlock) {
    const int L = e & 63, rr = L & 15, gg = L >> 4;
    float v;
    if (e < FT2) {
      const int mt = e >> 6;
      v = sP[OFF_W3 + gg * NH + 16 * mt + rr];
    } else if (e < FT1) {
      const int q = (e - FT2) >> 6, mt = q >> 4, ti = q & 15, t = ti >> 2, i = ti & 3;
      v = sP[OFF_W2 + (16 * t + 4 * gg + i) * NH + 16 * mt + rr];
    } else {
      const int q = (e - FT1) >> 6, mt = q >> 4, ti = q & 15, t = ti >> 2, i = ti & 3;
      v = sP[OFF_W1 + (16 * t + 4 * gg + i) * NIN + 16 * mt + rr];
    }
    ft[e] = v;
  }
  Frag32 f;
  load_frag32(sP, r, g, f);
  __syncthreads();  // every wave holds its fragments before the scratch is reused
  f32x4 aW1[4][2], aW2[4][4], aW3[4];
  float ab1[4][4], ab2[4][4], ab3[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    aW3[a] = f32x4{0, 0, 0, 0};
    ab3[a] = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      aW2[a][b] = f32x4{0, 0, 0, 0};
      ab1[a][b] = 0.0f;
      ab2[a][b] = 0.0f;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) aW1[a][b] = f32x4{0, 0, 0, 0};
  }
  S = count_of(S, S_dev);
  const int64_t ntile = ceil_div(S, 16);
  const int64_t wstride = (int64_t)gridDim.x * kBwdWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kBwdWaves + wid; tile < ntile; tile += wstride) {
    const int64_t s = tile * 16 + r;
    const bool ok = s < S;
    float X[8];
    load_x(feat, ld, s, g, ok, X);
    f32x4 z1[4], z2[4], o;
    fwd32(f, X, z1, z2, o);
    // output-head gradient (lanes g == 0 hold sample r's four outputs)
    float d3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (g == 0 && ok && (!bone || bone[s] >= 0)) {
      const float ov[4] = {o[0], o[1], o[2], o[3]};
      float sg, c[3];
      head(ov, &sg, c);
      d3[0] = ov[0] < 80.0f ? gsig[s] * sg : 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) d3[1 + k] = grgb[k * ld + s] * c[k] * (1.0f - c[k]);
    }
    // scratch: x, h1, h2, d3 tiles [feature/neuron][sample]
#pragma unroll
    for (int c = 0; c < 8; ++c) scr[SCR_X + (8 * g + c) * LDP + r] = X[c];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        scr[SCR_H1 + (16 * t + 4 * g + i) * LDP + r] = relu(z1[t][i]);
        scr[SCR_H2 + (16 * t + 4 * g + i) * LDP + r] = relu(z2[t][i]);
      }
    if (g == 0)
#pragma unroll
      for (int k = 0; k < 4; ++k) scr[SCR_D3 + k * LDP + r] = d3[k];
    // B operand of gh2 = W3^T d3: d3[output g][sample r]
    float b3 = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = __shfl(d3[k], r, 64);
      b3 = (g == k) ? t : b3;
    }
    f32x4 d2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = mfma4(ft[FT3 + mt * 64 + lane], b3, f32x4{0, 0, 0, 0});
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i] = z2[mt][i] < 0.0f ? 0.0f : acc[i];
        ab2[mt][i] += acc[i];
      }
      d2[mt] = acc;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) ab3[i] += (g == 0) ? d3[i] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) scr[SCR_D + (16 * t + 4 * g + i) * LDP + r] = d2[t][i];
    wave_sync();
    // dW3 += d3 h2^T ; dW2 += d2 h1^T   (K = 16 samples, 4 steps)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float a3 = r < NOUT ? scr[SCR_D3 + r * LDP + 4 * c + g] : 0.0f;
      float bh2[4], bh1[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        bh2[nt] = scr[SCR_H2 + (16 * nt + r) * LDP + 4 * c + g];
        bh1[nt] = scr[SCR_H1 + (16 * nt + r) * LDP + 4 * c + g];
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) aW3[nt] = mfma4(a3, bh2[nt], aW3[nt]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const float ad = scr[SCR_D + (16 * mt + r) * LDP + 4 * c + g];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) aW2[mt][nt] = mfma4(ad, bh1[nt], aW2[mt][nt]);
      }
    }
    wave_sync();
    // gh1 = W2^T d2 ; d1
    f32x4 d1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc = mfma4(ft[FT2 + (mt * 16 + 4 * t + i) * 64 + lane], d2[t][i], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i] = z1[mt][i] < 0.0f ? 0.0f : acc[i];
        ab1[mt][i] += acc[i];
      }
      d1[mt] = acc;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) scr[SCR_D + (16 * t + 4 * g + i) * LDP + r] = d1[t][i];
    // gfeat = W1^T d1 -> feature 16mt + 4g + i = level 8mt + 2g + i/2, f = i%2
    if (gfeat) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = mfma4(ft[FT1 + (mt * 16 + 4 * t + i) * 64 + lane], d1[t][i], acc);
        if (ok) {
          float2 *gf = reinterpret_cast<float2 *>(gfeat);
          gf[(int64_t)(8 * mt + 2 * g) * ld + s] = make_float2(acc[0], acc[1]);
          gf[(int64_t)(8 * mt + 2 * g + 1) * ld + s] = make_float2(acc[2], acc[3]);
        }
      }
    }
    wave_sync();
    // dW1 += d1 x^T
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float bx[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) bx[nt] = scr[SCR_X + (16 * nt + r) * LDP + 4 * c + g];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const float ad = scr[SCR_D + (16 * mt + r) * LDP + 4 * c + g];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) aW1[mt][nt] = mfma4(ad, bx[nt], aW1[mt][nt]);
      }
    }
    wave_sync();
  }
  // bias partials: sum over the 16 sample lanes r
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        ab1[a][b] += __shfl_xor(ab1[a][b], o, 16);
        ab2[a][b] += __shfl_xor(ab2[a][b], o, 16);
      }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) ab3[a] += __shfl_xor(ab3[a], o, 16);
  // block partial in the (now free) scratch region, waves added in order
  __syncthreads();
  float *bp = lds + FT_SIZE;
  for (int w = 0; w < kBwdWaves; ++w) {
    if (wid == w) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = 16 * mt + 4 * g + i;
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            const int e = OFF_W1 + m * NIN + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW1[mt][nt][i];
          }
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const int e = OFF_W2 + m * NH + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW2[mt][nt][i];
          }
          if (r == 0) {
            bp[OFF_B1 + m] = (w ? bp[OFF_B1 + m] : 0.0f) + ab1[mt][i];
            bp[OFF_B2 + m] = (w ? bp[OFF_B2 + m] : 0.0f) + ab2[mt][i];
          }
        }
      if (g == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const int e = OFF_W3 + i * NH + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW3[nt][i];
          }
          if (r == 0) bp[OFF_B3 + i] = (w ? bp[OFF_B3 + i] : 0.0f) + ab3[i];
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NPARAM; e += kBwdBlock) partial[(int64_t)blockIdx.x * NPARAM + e] = bp[e];
}

// --------------------------------------------------------------- BF16 bwd
// Same algebra as the FP32 backward, on BF16 MFMA 16x16x32 (FP32
// accumulate).  A wave owns a 32-sample tile: two 16-sample sub-tiles run
// the BF16 forward and the chained backward (gh1 = W2^T d2, gfeat = W1^T d1
// with transposed weight fragments; the 4-wide head gh2 = W3^T d3 on FP32
// MFMA), then the weight gradients take K = 32 samples per MFMA from
// [neuron][sample] BF16 tiles in LDS.
constexpr int LDB = 40;  // BF16 row stride of the sample tiles (32 + 8 pad)
constexpr int BR_X = 0, BR_H1 = 32, BR_H2 = 96, BR_D2 = 160, BR_D1 = 224, BR_D3 = 288, BR_ROWS = 292;
constexpr int SCRB_BYTES = BR_ROWS * LDB * 2;
constexpr int LDS_BF_BYTES = kBwdWaves * SCRB_BYTES;
static_assert(LDS_BF_BYTES >= NPARAM * 4, "block partial reuses the scratch region");
static_assert(LDS_BF_BYTES <= 65536, "one workgroup's LDS");

struct FragBfT {
  bf16x8 w2t[4][2];  // [mt][c]: W2[16(2c + j/4) + 4g + j%4][16mt + r]
  bf16x8 w1t[2][2];  // [mt][c]: W1[16(2c + j/4) + 4g + j%4][16mt + r]
  float w3t[4];      // [mt]: W3[g][16mt + r]
};

__device__ __forceinline__ void load_frag_bft(const float *P, int r, int g, FragBfT &f) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 16 * (2 * c + j / 4) + 4 * g + (j % 4);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) f.w2t[mt][c][j] = (__bf16)P[OFF_W2 + k * NH + 16 * mt + r];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) f.w1t[mt][c][j] = (__bf16)P[OFF_W1 + k * NIN + 16 * mt + r];
    }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) f.w3t[mt] = (float)(__bf16)P[OFF_W3 + g * NH + 16 * mt + r];
}

__device__ __forceinline__ bf16x8 pack_raw(const f32x4 z[4], int c) {
  bf16x8 b;
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = (__bf16)z[2 * c + j / 4][j % 4];
  return b;
}

__device__ __forceinline__ bf16x8 lds_row8(const __bf16 *scr, int row, int col) {
  return *reinterpret_cast<const bf16x8 *>(scr + row * LDB + col);
}

__global__ void __launch_bounds__(kBwdBlock) mlp_bwd_bf16(const float *__restrict__ gsig,
                                                          const float *__restrict__ grgb,
                                                          const __hip_bfloat16 *__restrict__ feat,
                                                          const int16_t *__restrict__ bone, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                          const float *__restrict__ P, float *__restrict__ gfeat,
                                                          float *__restrict__ partial) {
  extern __shared__ __attribute__((aligned(16))) unsigned char ldsb[];
  // the forward's fragments stay in LDS (read as each MFMA needs them); held
  // in registers beside the weight-gradient accumulators they spill
  __shared__ __attribute__((aligned(16))) FragLds sF;
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4, wid = threadIdx.x >> 6;
  __bf16 *scr = reinterpret_cast<__bf16 *>(ldsb + wid * SCRB_BYTES);
  stage_frag_lds(P, sF);
  // the parameters go to the scratch region until every wave holds its
  // transposed fragments
  float *sP = reinterpret_cast<float *>(ldsb);
  stage_params(P, sP);
  __syncthreads();
  FragBfT ft;
  load_frag_bft(sP, r, g, ft);
  __syncthreads();
  f32x4 aW1[4][2], aW2[4][4], aW3[4];
  float ab1[4][4], ab2[4][4], ab3[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    aW3[a] = f32x4{0, 0, 0, 0};
    ab3[a] = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      aW2[a][b] = f32x4{0, 0, 0, 0};
      ab1[a][b] = 0.0f;
      ab2[a][b] = 0.0f;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) aW1[a][b] = f32x4{0, 0, 0, 0};
  }
  S = count_of(S, S_dev);
  const int64_t ntile = ceil_div(S, 32);
  const int64_t wstride = (int64_t)gridDim.x * kBwdWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kBwdWaves + wid; tile < ntile; tile += wstride) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int col = 16 * half + r;
      const int64_t s = tile * 32 + col;
      const bool ok = s < S;
      const bf16x8 X = load_x_bf16(feat, ld, s, g, ok);
      f32x4 z1[4], z2[4], o;
      pin_in_loop();
      fwd_bf_src(LdsW{sF, lane, g}, X, z1, z2, o);
      float d3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (g == 0 && ok && (!bone || bone[s] >= 0)) {
        const float ov[4] = {o[0], o[1], o[2], o[3]};
        float sg, c[3];
        head(ov, &sg, c);
        d3[0] = ov[0] < 80.0f ? gsig[s] * sg : 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) d3[1 + k] = grgb[k * ld + s] * c[k] * (1.0f - c[k]);
      }
      // the 4-wide head runs on FP32 MFMA with BF16-valued operands (the
      // forward's W3, the output delta as stored for the weight gradient)
      float b3 = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float t = __shfl(d3[k], r, 64);
        b3 = (g == k) ? (float)(__bf16)t : b3;
      }
      f32x4 d2[4], d1[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = mfma4(ft.w3t[mt], b3, f32x4{0, 0, 0, 0});
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[i] = z2[mt][i] < 0.0f ? 0.0f : acc[i];
          ab2[mt][i] += acc[i];
        }
        d2[mt] = acc;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) ab3[i] += (g == 0) ? d3[i] : 0.0f;
      const bf16x8 d2a = pack_raw(d2, 0), d2b = pack_raw(d2, 1);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = mfma32(ft.w2t[mt][0], d2a, f32x4{0, 0, 0, 0});
        acc = mfma32(ft.w2t[mt][1], d2b, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[i] = z1[mt][i] < 0.0f ? 0.0f : acc[i];
          ab1[mt][i] += acc[i];
        }
        d1[mt] = acc;
      }
      if (gfeat) {
        const bf16x8 d1a = pack_raw(d1, 0), d1b = pack_raw(d1, 1);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          f32x4 acc = mfma32(ft.w1t[mt][0], d1a, f32x4{0, 0, 0, 0});
          acc = mfma32(ft.w1t[mt][1], d1b, acc);
          if (ok) {
            float2 *gf = reinterpret_cast<float2 *>(gfeat);
            gf[(int64_t)(8 * mt + 2 * g) * ld + s] = make_float2(acc[0], acc[1]);
            gf[(int64_t)(8 * mt + 2 * g + 1) * ld + s] = make_float2(acc[2], acc[3]);
          }
        }
      }
      // [neuron][sample] tiles for the weight gradients
#pragma unroll
      for (int j = 0; j < 8; ++j) scr[(BR_X + 8 * g + j) * LDB + col] = X[j];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int n = 16 * t + 4 * g + i;
          scr[(BR_H1 + n) * LDB + col] = (__bf16)relu(z1[t][i]);
          scr[(BR_H2 + n) * LDB + col] = (__bf16)relu(z2[t][i]);
          scr[(BR_D2 + n) * LDB + col] = (__bf16)d2[t][i];
          scr[(BR_D1 + n) * LDB + col] = (__bf16)d1[t][i];
        }
      if (g == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) scr[(BR_D3 + k) * LDB + col] = (__bf16)d3[k];
    }
    wave_sync();
    // weight gradients, K = the tile's 32 samples
    const bf16x8 zero8 = {};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 bh1 = lds_row8(scr, BR_H1 + 16 * nt + r, 8 * g);
      const bf16x8 bh2 = lds_row8(scr, BR_H2 + 16 * nt + r, 8 * g);
      const bf16x8 a3 = r < NOUT ? lds_row8(scr, BR_D3 + r, 8 * g) : zero8;
      aW3[nt] = mfma32(a3, bh2, aW3[nt]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) aW2[mt][nt] = mfma32(lds_row8(scr, BR_D2 + 16 * mt + r, 8 * g), bh1, aW2[mt][nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const bf16x8 bx = lds_row8(scr, BR_X + 16 * nt + r, 8 * g);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) aW1[mt][nt] = mfma32(lds_row8(scr, BR_D1 + 16 * mt + r, 8 * g), bx, aW1[mt][nt]);
    }
    wave_sync();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        ab1[a][b] += __shfl_xor(ab1[a][b], o, 16);
        ab2[a][b] += __shfl_xor(ab2[a][b], o, 16);
      }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) ab3[a] += __shfl_xor(ab3[a], o, 16);
  __syncthreads();
  float *bp = reinterpret_cast<float *>(ldsb);
  for (int w = 0; w < kBwdWaves; ++w) {
    if (wid == w) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = 16 * mt + 4 * g + i;
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            const int e = OFF_W1 + m * NIN + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW1[mt][nt][i];
          }
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const int e = OFF_W2 + m * NH + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW2[mt][nt][i];
          }
          if (r == 0) {
            bp[OFF_B1 + m] = (w ? bp[OFF_B1 + m] : 0.0f) + ab1[mt][i];
            bp[OFF_B2 + m] = (w ? bp[OFF_B2 + m] : 0.0f) + ab2[mt][i];
          }
        }
      if (g == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const int e = OFF_W3 + i * NH + 16 * nt + r;
            bp[e] = (w ? bp[e] : 0.0f) + aW3[nt][i];
          }
          if (r == 0) bp[OFF_B3 + i] = (w ? bp[OFF_B3 + i] : 0.0f) + ab3[i];
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NPARAM; e += kBwdBlock) partial[(int64_t)blockIdx.x * NPARAM + e] = bp[e];
}

// Sum of the block partials per parameter: 64 parameters x 16 partial groups
// per workgroup; each thread sums its group in double with four independent
// accumulators, then the 16 groups are combined in a fixed order (the
// result does not depend on scheduling).
constexpr int kRedP = 64, kRedG = 16;
__global__ void __launch_bounds__(kRedP *kRedG) reduce_partials(const float *__restrict__ partial, int nblk,
                                                                float *__restrict__ out, int overwrite) {
  __shared__ double part[kRedG][kRedP];
  const int pl = threadIdx.x % kRedP, grp = threadIdx.x / kRedP;
  const int e = blockIdx.x * kRedP + pl;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (e < NPARAM) {
    int b = grp;
    for (; b + 3 * kRedG < nblk; b += 4 * kRedG) {
      a0 += (double)partial[(int64_t)b * NPARAM + e];
      a1 += (double)partial[(int64_t)(b + kRedG) * NPARAM + e];
      a2 += (double)partial[(int64_t)(b + 2 * kRedG) * NPARAM + e];
      a3 += (double)partial[(int64_t)(b + 3 * kRedG) * NPARAM + e];
    }
    for (; b < nblk; b += kRedG) a0 += (double)partial[(int64_t)b * NPARAM + e];
  }
  part[grp][pl] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (grp == 0 && e < NPARAM) {
    double s = 0.0;
    for (int g = 0; g < kRedG; ++g) s += part[g][pl];
    out[e] = overwrite ? (float)s : out[e] + (float)s;
  }
}

constexpr int kMaxBwdBlocks = 512;

int bwd_blocks(int64_t S) {
  int64_t b = ceil_div(ceil_div(S, 16), kBwdWaves);
  if (b > kMaxBwdBlocks) b = kMaxBwdBlocks;
  return b < 1 ? 1 : (int)b;
}

// as many blocks as stay resident (2 waves per SIMD by registers): each
// wave then loops over its tiles with the next tile's loads in flight
// workgroups per CU the forward kernels keep resident: two for FP32 (256
// registers a lane), four for BF16 (fragments in LDS, 100 registers)
unsigned fwd_blocks(int64_t S, int per_cu) { return grid_for(ceil_div(S, 16) * 64, kFwdBlock, 256 * per_cu); }

}  // namespace

namespace {

// The one decoder shape the kernels implement (Eq. 1-2 with the widths of
// the Instant-NGP density/colour head): 32 -> 64 -> 64 -> 4.
int32_t widths_status(const int32_t *widths, int32_t n_layers) {
  if (!widths || n_layers < 1 || n_layers > 15) return IA355_ERR_INVALID_ARG;
  for (int l = 0; l <= n_layers; ++l)
    if (widths[l] <= 0) return IA355_ERR_INVALID_ARG;
  if (n_layers != 3 || widths[0] != NIN || widths[1] != NH || widths[2] != NH || widths[3] != NOUT)
    return IA355_ERR_UNSUPPORTED;
  return IA355_OK;
}

}  // namespace

extern "C" int32_t ia355_mlp_fwd(const void *feat, int32_t feat_dtype, const int16_t *bone, int64_t S,
                                 const int64_t *S_dev, int64_t ld, const float *params, const int32_t *widths,
                                 int32_t n_layers, int32_t dtype, float *sigma, float *rgb, ia355_stream_t stream) {
  const int32_t ws = widths_status(widths, n_layers);
  if (ws != IA355_OK) return ws;
  if (S < 0 || ld < S || !params || ((uintptr_t)params & 15)) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!feat || !sigma || !rgb)) return IA355_ERR_INVALID_ARG;
  if (dtype == IA355_F32 && feat_dtype != IA355_F32) return IA355_ERR_UNSUPPORTED;
  if (dtype == IA355_BF16 && feat_dtype != IA355_BF16) return IA355_ERR_UNSUPPORTED;
  if (dtype != IA355_F32 && dtype != IA355_BF16) return IA355_ERR_INVALID_ARG;
  if (S == 0) return IA355_OK;
  hipStream_t s = as_stream(stream);
  if (dtype == IA355_F32)
    mlp_fwd_f32<<<fwd_blocks(S, 2), kFwdBlock, 0, s>>>((const float *)feat, bone, S, S_dev, ld, params, sigma, rgb);
  else
    mlp_fwd_bf16<<<fwd_blocks(S, 4), kFwdBlock, 0, s>>>((const __hip_bfloat16 *)feat, bone, S, S_dev, ld, params, sigma,
                                                     rgb);
  return launch_status();
}

extern "C" size_t ia355_mlp_bwd_workspace_size(int64_t S) {
  return align256(sizeof(float) * (size_t)NPARAM * bwd_blocks(S));
}

extern "C" int32_t ia355_mlp_bwd(const float *grad_sigma, const float *grad_rgb, const void *feat, int32_t feat_dtype,
                                 const int16_t *bone, int64_t S, const int64_t *S_dev, int64_t ld,
                                 const float *params, const int32_t *widths, int32_t n_layers, int32_t dtype,
                                 float *grad_params, float *grad_feat, uint32_t flags, void *ws, size_t ws_bytes,
                                 ia355_stream_t stream) {
  const int32_t wst = widths_status(widths, n_layers);
  if (wst != IA355_OK) return wst;
  if (S < 0 || ld < S || !params || !grad_params || ((uintptr_t)params & 15)) return IA355_ERR_INVALID_ARG;
  if (flags & ~(uint32_t)IA355_OVERWRITE) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!grad_sigma || !grad_rgb || !feat)) return IA355_ERR_INVALID_ARG;
  if (!((dtype == IA355_F32 && feat_dtype == IA355_F32) || (dtype == IA355_BF16 && feat_dtype == IA355_BF16)))
    return IA355_ERR_UNSUPPORTED;
  if (S == 0) return (flags & IA355_OVERWRITE) ? ia355_zero(grad_params, sizeof(float) * NPARAM, stream) : IA355_OK;
  if (!ws || ws_bytes < ia355_mlp_bwd_workspace_size(S)) return IA355_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  const int nb = bwd_blocks(S);
  if (dtype == IA355_F32)
    mlp_bwd_f32<<<nb, kBwdBlock, LDS_FLOATS * sizeof(float), s>>>(grad_sigma, grad_rgb, (const float *)feat, bone, S,
                                                                  S_dev, ld, params, grad_feat, (float *)ws);
  else
    mlp_bwd_bf16<<<nb, kBwdBlock, LDS_BF_BYTES, s>>>(grad_sigma, grad_rgb, (const __hip_bfloat16 *)feat, bone, S,
                                                     S_dev, ld, params, grad_feat, (float *)ws);
  reduce_partials<<<(unsigned)ceil_div(NPARAM, kRedP), kRedP * kRedG, 0, s>>>((const float *)ws, nb, grad_params,
                                                                                     (flags & IA355_OVERWRITE) != 0);
  return launch_status();
}
