// Learned root initialiser for the canonical-correspondence search (an
// addition to the root finding of Sec. 3.1, not in the paper): a small MLP maps
// (posed point x', pose) to per-bone logits and a canonical offset; the
// start point handed to Broyden is x0 = B_k^{-1} x' + offset, k = argmax.
//
// Layer 1 takes (x', pose); the pose part W1[:, 3:] pose + b1 is the same
// for every sample of a pose, so each workgroup folds it into a per-neuron
// constant once and layer 1 costs 3 FMAs per neuron.  Layers 2 and 3 run on
// MFMA exactly like the decoder MLP (one wave per 16-sample tile, the
// hidden activations chained in registers through the K ordering), in FP32
// (16x16x4) or BF16 (16x16x32, FP32 accumulate).  The argmax over the bone
// logits is a cross-lane reduction.
#include "common.h"
#include "geometry.h"

using namespace ia355;

namespace {

constexpr int H = 64;           // hidden width
constexpr int kMaxOut = 32;     // nb + 3 outputs in two 16-row MFMA tiles
constexpr int kBlock = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// max(z, 0): one v_max_f32 (a compare-and-select keeps NaN semantics and costs two)
__device__ __forceinline__ float relu(float z) { return fmaxf(z, 0.0f); }

template <bool BF16>
__global__ void __launch_bounds__(kBlock) rootinit_kernel(const float *__restrict__ xp_soa, int64_t S,
                                                          const int64_t *__restrict__ S_dev, int64_t ld,
                                                          const float *__restrict__ pose, const float *__restrict__ P,
                                                          const float *__restrict__ B, int nb,
                                                          int16_t *__restrict__ bone_out, float *__restrict__ x0_soa) {
  const int nin = 3 + 6 * nb, nout = nb + 3;
  const int offW1 = 0, offb1 = H * nin, offW2 = offb1 + H, offb2 = offW2 + H * H, offW3 = offb2 + H,
            offb3 = offW3 + nout * H;
  // a block without a tile returns before any work (uniform, ahead of the
  // barriers): with a device-side count the grid is sized for the capacity
  const int64_t Sn = count_of(S, S_dev);
  if ((int64_t)blockIdx.x * (kBlock / 64) >= ceil_div(Sn, 16)) return;
  __shared__ float c1[H];        // W1[:, 3:] pose + b1
  __shared__ float w1x[H * 3];   // W1[:, :3]
  __shared__ float sBinv[64 * 12];
  __shared__ int sBok[64];
  // the parameters, copied into LDS once per block with coalesced 16-byte
  // loads (the pose fold walks W1 row by row; the MFMA fragments gather
  // single values): a lane reading them from global memory one value at a
  // time waits on a different cache line per value
  extern __shared__ __attribute__((aligned(16))) float sP[];
  const int np_all = offb3 + nout;
  {
    const int head = (int)((4 - (((uintptr_t)P >> 2) & 3)) & 3);  // floats before 16-byte alignment
    const int h = head < np_all ? head : np_all;
    for (int i = threadIdx.x; i < h; i += kBlock) sP[i] = P[i];
    const int n4 = (np_all - h) >> 2;
    const float4 *P4 = reinterpret_cast<const float4 *>(P + h);
    for (int i = threadIdx.x; i < n4; i += kBlock) {
      const float4 q = P4[i];
      sP[h + 4 * i] = q.x;
      sP[h + 4 * i + 1] = q.y;
      sP[h + 4 * i + 2] = q.z;
      sP[h + 4 * i + 3] = q.w;
    }
    for (int i = h + 4 * n4 + threadIdx.x; i < np_all; i += kBlock) sP[i] = P[i];
  }
  __syncthreads();
  {
    // four threads per neuron, each a strided quarter of the pose terms with
    // four independent partial sums, combined across the four lanes
    static_assert(kBlock == 4 * H, "four threads per hidden neuron");
    const int n = threadIdx.x >> 2, q = threadIdx.x & 3;
    const float *wrow = sP + offW1 + n * nin + 3;
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
    if (q == 0) c1[n] = acc + sP[offb1 + n];
  }
  for (int e = threadIdx.x; e < H * 3; e += kBlock) w1x[e] = sP[offW1 + (e / 3) * nin + (e % 3)];
  stage_bone_inverses(B, nb, sBinv, sBok);
  __syncthreads();

  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  // weight fragments (see the decoder MLP for the layouts)
  float w2f[4][16], w3f[2][16];
  bf16x8 w2b[4][2], w3b[2][2];
  float b2[4][4], b3[2][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) b2[mt][i] = sP[offb2 + 16 * mt + 4 * g + i];
    if (!BF16) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) w2f[mt][4 * t + i] = sP[offW2 + (16 * mt + r) * H + 16 * t + 4 * g + i];
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          w2b[mt][c][j] = (__bf16)sP[offW2 + (16 * mt + r) * H + 16 * (2 * c + j / 4) + 4 * g + (j % 4)];
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int row = 16 * mt + r;
#pragma unroll
    for (int i = 0; i < 4; ++i) b3[mt][i] = (16 * mt + 4 * g + i) < nout ? sP[offb3 + 16 * mt + 4 * g + i] : 0.0f;
    if (!BF16) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) w3f[mt][4 * t + i] = row < nout ? sP[offW3 + row * H + 16 * t + 4 * g + i] : 0.0f;
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          w3b[mt][c][j] = (__bf16)(row < nout ? sP[offW3 + row * H + 16 * (2 * c + j / 4) + 4 * g + (j % 4)] : 0.0f);
    }
  }

  S = Sn;
  const int64_t ntile = ceil_div(S, 16);
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); tile < ntile; tile += wstride) {
    const int64_t s = tile * 16 + r;
    const bool ok = s < S;
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (ok) {
      x[0] = xp_soa[s];
      x[1] = xp_soa[ld + s];
      x[2] = xp_soa[2 * ld + s];
    }
    // layer 1 on the VALU: lane holds neurons 16t + 4g + i of sample r
    float h1[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = 16 * t + 4 * g + i;
        h1[t][i] = relu(c1[n] + w1x[3 * n] * x[0] + w1x[3 * n + 1] * x[1] + w1x[3 * n + 2] * x[2]);
      }
    f32x4 z2[4], o[2];
    if (!BF16) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {b2[mt][0], b2[mt][1], b2[mt][2], b2[mt][3]};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w2f[mt][4 * t + i], h1[t][i], acc, 0, 0, 0);
        z2[mt] = acc;
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        f32x4 acc = {b3[mt][0], b3[mt][1], b3[mt][2], b3[mt][3]};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w3f[mt][4 * t + i], relu(z2[t][i]), acc, 0, 0, 0);
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
        f32x4 acc = {b2[mt][0], b2[mt][1], b2[mt][2], b2[mt][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2b[mt][0], ha, acc, 0, 0, 0);
        z2[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2b[mt][1], hb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        ha[j] = (__bf16)relu(z2[j / 4][j % 4]);
        hb[j] = (__bf16)relu(z2[2 + j / 4][j % 4]);
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        f32x4 acc = {b3[mt][0], b3[mt][1], b3[mt][2], b3[mt][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3b[mt][0], ha, acc, 0, 0, 0);
        o[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3b[mt][1], hb, acc, 0, 0, 0);
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
    if (g == 0 && ok) {
      const int k = bi < nb ? bi : 0;
      const float *Bi = sBinv + 12 * k;
      bone_out[s] = (int16_t)k;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        x0_soa[a * ld + s] = Bi[4 * a] * x[0] + Bi[4 * a + 1] * x[1] + Bi[4 * a + 2] * x[2] + Bi[4 * a + 3] + off[a];
    }
  }
}

}  // namespace

extern "C" int32_t ia355_rootinit_fwd(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld, const float *pose,
                                      const float *params,
                                      int32_t hidden, const float *B, int32_t nb, int32_t dtype, int16_t *init_bone,
                                      float *x0, ia355_stream_t stream) {
  if (S < 0 || ld < S || nb <= 0 || !pose || !params || !B) return IA355_ERR_INVALID_ARG;
  if (hidden != H || nb + 3 > kMaxOut) return IA355_ERR_UNSUPPORTED;
  if (dtype != IA355_F32 && dtype != IA355_BF16) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!xp || !init_bone || !x0)) return IA355_ERR_INVALID_ARG;
  if (S == 0) return IA355_OK;
  // at most two blocks per CU (the parameters take 61.5 KB of LDS each), each
  // wave looping over its tiles
  const unsigned grid = grid_for(ceil_div(S, 16) * 64, kBlock, 256 * 2);
  const size_t lds = sizeof(float) * (size_t)(H * (3 + 6 * nb) + H + H * H + H + (nb + 3) * H + (nb + 3));
  if (lds > 96 * 1024) return IA355_ERR_UNSUPPORTED;
  hipStream_t s = as_stream(stream);
  if (dtype == IA355_F32)
    rootinit_kernel<false><<<grid, kBlock, lds, s>>>(xp, S, S_dev, ld, pose, params, B, nb, init_bone, x0);
  else
    rootinit_kernel<true><<<grid, kBlock, lds, s>>>(xp, S, S_dev, ld, pose, params, B, nb, init_bone, x0);
  return launch_status();
}
