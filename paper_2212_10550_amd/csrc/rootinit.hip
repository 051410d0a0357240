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
#include "rootinit_dev.h"

using namespace ia355;

namespace {

constexpr int kBlock = 256;
using rid::H;
using rid::kMaxOut;

// BF16: the parameters are read from global memory once per block (the pose
// fold, layer 1's x weights, the layer 2-3 fragments into a 12 KB LDS store
// read as each MFMA needs them), so a block needs ~17 KB of LDS and ~100
// registers a lane: four waves per SIMD.  FP32: the whole parameter block
// is staged in LDS (61.5 KB) and the fragments held in registers.
template <bool BF16>
__global__ void __launch_bounds__(kBlock, BF16 ? 4 : 1) rootinit_kernel(
    const float *__restrict__ xp_soa, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
    const float *__restrict__ pose, const float *__restrict__ P, const float *__restrict__ B, int nb,
    int16_t *__restrict__ bone_out, float *__restrict__ x0_soa) {
  const rid::Layout l = rid::layout(nb);
  // a block without a tile returns before any work (uniform, ahead of the
  // barriers): with a device-side count the grid is sized for the capacity
  const int64_t Sn = count_of(S, S_dev);
  if ((int64_t)blockIdx.x * (kBlock / 64) >= ceil_div(Sn, 16)) return;
  __shared__ float c1[H];        // W1[:, 3:] pose + b1
  __shared__ float w1x[H * 3];   // W1[:, :3]
  __shared__ float sBinv[64 * 12];
  __shared__ int sBok[64];
  __shared__ __attribute__((aligned(16))) bf16x8 sRw[BF16 ? 12 : 1][kWave];
  __shared__ __attribute__((aligned(16))) float sRb2[BF16 ? H : 4], sRb3[BF16 ? kMaxOut : 4];
  // FP32: the parameters, copied into LDS once per block with coalesced
  // 16-byte loads (the pose fold walks W1 row by row; the MFMA fragments
  // gather single values)
  extern __shared__ __attribute__((aligned(16))) float sP[];
  static_assert(kBlock == 4 * H, "four threads per hidden neuron");
  const float *Pw;  // where the fold and layer 1 read the parameters
  if constexpr (BF16) {
    Pw = P;
    rid::stage_frag_lds(P, l, sRw, sRb2, sRb3);
  } else {
    rid::stage_copy(P, l.total, sP);
    __syncthreads();
    Pw = sP;
  }
  rid::fold_pose(Pw, l, pose, nb, c1);
  for (int e = threadIdx.x; e < H * 3; e += kBlock) w1x[e] = Pw[l.offW1 + (e / 3) * l.nin + (e % 3)];
  stage_bone_inverses(B, nb, sBinv, sBok);
  __syncthreads();

  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  rid::Frag<BF16> f;
  if constexpr (!BF16) rid::load_frag<BF16>(sP, l, r, g, f);
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
    int bi;
    float off[3];
    if constexpr (BF16) {
      float h1[4][4];
      rid::layer1(x, c1, w1x, g, h1);
      // the fragment reads stay in the loop (hoisted, they would hold every
      // fragment in registers)
      asm volatile("" ::: "memory");
      rid::tile_tail<true>(h1, rid::LdsFragW{sRw, sRb2, sRb3, lane, g}, nb, g, &bi, off);
    } else {
      rid::tile<BF16>(x, c1, w1x, f, nb, g, &bi, off);
    }
    if (g == 0 && ok) {
      const int k = bi < nb ? bi : 0;
      const float *Bi = sBinv + 12 * k;
      bone_out[s] = (int16_t)k;
      float x0[3];
      rid::start_point(Bi, x, off, x0);
#pragma unroll
      for (int a = 0; a < 3; ++a) x0_soa[a * ld + s] = x0[a];
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
  // FP32: at most two blocks per CU (the parameters take 61.5 KB of LDS
  // each); BF16: four; each wave loops over its tiles
  const size_t lds = sizeof(float) * (size_t)(H * (3 + 6 * nb) + H + H * H + H + (nb + 3) * H + (nb + 3));
  if (lds > 96 * 1024) return IA355_ERR_UNSUPPORTED;
  hipStream_t s = as_stream(stream);
  if (dtype == IA355_F32)
    rootinit_kernel<false><<<grid_for(ceil_div(S, 16) * 64, kBlock, 256 * 2), kBlock, lds, s>>>(
        xp, S, S_dev, ld, pose, params, B, nb, init_bone, x0);
  else
    rootinit_kernel<true><<<grid_for(ceil_div(S, 16) * 64, kBlock, 256 * 4), kBlock, 0, s>>>(
        xp, S, S_dev, ld, pose, params, B, nb, init_bone, x0);
  return launch_status();
}
