// Articulation (Sec. 3.1, Eq. 5-7): posed point x' -> canonical root x* of
// x' = sum_i w_i(x) B_i x, by multi-init Broyden root finding, and its
// backward by the implicit function theorem.
//
// Forward design (gfx950):
//  * blend kernel: because trilinear interpolation is linear in the vertex
//    values, sum_i w_i(x) B_i = sum_c tri_c(x) A_c with A_v = sum_i W[v][i] B_i
//    the per-pose blended transform of vertex v.  A is a 12-float-per-vertex
//    grid (3 x float4 per corner) built once per pose, which halves the
//    gathered bytes and removes the 24-bone blend from every residual.
//  * solve kernel: eight lanes per posed sample each run a third of the nb
//    Broyden solves in FP32 registers and pick the lowest residual with
//    shuffles; bone inverses are staged in LDS once per block; the blended
//    grid is read through the vector L1/L2 with float4 gathers.
#include <mutex>

#include "common.h"
#include "deform_dev.h"
#include "geometry.h"

using namespace ia355;
using namespace ia355::dfm;

namespace {

// qlen (nullable): a counter the next kernel on the stream needs at zero
// (the guided solve's fallback queue), cleared here instead of by a launch
// of its own.
__global__ void __launch_bounds__(kBlendBlock) blend_kernel(const float *__restrict__ W, const float *__restrict__ B,
                                                             int nb, int64_t nvert, float *__restrict__ A,
                                                             int32_t *__restrict__ qlen) {
  if (qlen && blockIdx.x == 0 && threadIdx.x == 0) *qlen = 0;
  __shared__ float sB[kMaxBones * 12];
  __shared__ __attribute__((aligned(16))) float sW[kBlendBlock * kBlendMaxBones];
  blend_block(W, B, nb, nvert, A, blockIdx.x, sB, sW);
}

__global__ void __launch_bounds__(kSolveBlock) solve_kernel(
    const float *__restrict__ xp_soa, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
    const float *__restrict__ B, int nb, const float *__restrict__ A, Grid gr, Box hbox, int max_iter, float tol_stop,
    float tol_valid, float *__restrict__ xc_soa, int16_t *__restrict__ bone_out, float *__restrict__ resid_out,
    int16_t *__restrict__ steps_out) {
  __shared__ float sBinv[kMaxBones * 12];
  __shared__ int sBok[kMaxBones];
  stage_bone_inverses(B, nb, sBinv, sBok);
  __syncthreads();
  const int64_t Sn = count_of(S, S_dev);
  const int j = threadIdx.x % kGroup;
  constexpr int kPerBlock = kSolveBlock / kGroup;
  // every lane of a block runs the same iterations, so the groups' shuffles
  // always see all eight lanes
  for (int64_t n0 = (int64_t)blockIdx.x * kPerBlock; n0 < Sn; n0 += (int64_t)gridDim.x * kPerBlock) {
    const int64_t n = n0 + threadIdx.x / kGroup;
    const bool act = n < Sn;
    float xp[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      xp[0] = xp_soa[n];
      xp[1] = xp_soa[ld + n];
      xp[2] = xp_soa[2 * ld + n];
    }
    const Choice c = multi_init(A, gr, sBinv, sBok, nb, xp, act, j, hbox, max_iter, tol_stop, tol_valid);
    if (act && j == 0) write_choice(c, n, ld, 0, xc_soa, bone_out, resid_out, steps_out);
  }
}

// Guided solve: one lane per sample starts Broyden at the given x0; an
// accepted root (residual < tol_valid, inside the canonical box) is final,
// otherwise the sample index is appended to the fallback queue.
// Every distinct valid root of each sample (multi-root aggregation, the
// alternative to keeping only the lowest-residual root): the kGroup lanes of
// a sample run its inits as in the multi-init solve and put each init's final
// iterate and residual (infinite when the init is not valid) in LDS; the
// group's first lane then takes up to K roots in order of increasing residual
// (ties: lower init), dropping every candidate within dup_tol of a root
// already taken.  With K = 1 this is the lowest-residual root.  Layout:
// roots [3][K][S] (slot k of sample n at (a K + k) S + n), root_bone [K][S]
// (-1 past the sample's count; the slot then holds init 0's final iterate).
constexpr int kRootSamples = kSolveBlock / kGroup;

__global__ void __launch_bounds__(kSolveBlock) roots_kernel(
    const float *__restrict__ xp_soa, int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
    const float *__restrict__ B, int nb, const float *__restrict__ A, Grid gr, Box hbox, int max_iter, float tol_stop,
    float tol_valid, int K, float dup_tol, float *__restrict__ roots, int16_t *__restrict__ rbone,
    int32_t *__restrict__ nroots) {
  __shared__ float sBinv[kMaxBones * 12];
  __shared__ int sBok[kMaxBones];
  __shared__ float cx[kRootSamples][kMaxBones][3];
  __shared__ float cr[kRootSamples][kMaxBones];
  stage_bone_inverses(B, nb, sBinv, sBok);
  __syncthreads();
  const int64_t Sn = count_of(S, S_dev);
  const int j = threadIdx.x % kGroup, sl = threadIdx.x / kGroup;
  const float tol2 = dup_tol * dup_tol;
  // every lane of a block runs the same iterations (the barriers below)
  for (int64_t n0 = (int64_t)blockIdx.x * kRootSamples; n0 < Sn; n0 += (int64_t)gridDim.x * kRootSamples) {
    const int64_t n = n0 + sl;
    const bool act = n < Sn;
    if (act) {
      const float xp[3] = {xp_soa[n], xp_soa[ld + n], xp_soa[2 * ld + n]};
      for (int i = j; i < nb; i += kGroup) {
        const InitResult q = broyden(A, gr, sBinv + 12 * i, sBok[i], xp, max_iter, tol_stop);
        const bool valid = q.ok && q.r < tol_valid && in_hbox(q.x, hbox);
        cx[sl][i][0] = q.x[0];
        cx[sl][i][1] = q.x[1];
        cx[sl][i][2] = q.x[2];
        cr[sl][i] = valid ? q.r : INFINITY;
      }
    }
    __syncthreads();
    if (act && j == 0) {
      int cnt = 0;
      for (int k = 0; k < K; ++k) {
        int best = -1;
        float br = INFINITY;
        for (int i = 0; i < nb; ++i)
          if (cr[sl][i] < br) {
            br = cr[sl][i];
            best = i;
          }
        if (best < 0) break;
        const float bx[3] = {cx[sl][best][0], cx[sl][best][1], cx[sl][best][2]};
        for (int i = 0; i < nb; ++i) {
          if (!(cr[sl][i] < INFINITY)) continue;
          const float d0 = cx[sl][i][0] - bx[0], d1 = cx[sl][i][1] - bx[1], d2 = cx[sl][i][2] - bx[2];
          if (d0 * d0 + d1 * d1 + d2 * d2 <= tol2) cr[sl][i] = INFINITY;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) roots[((int64_t)a * K + k) * S + n] = bx[a];
        rbone[(int64_t)k * S + n] = (int16_t)best;
        ++cnt;
      }
      for (int k = cnt; k < K; ++k) {
#pragma unroll
        for (int a = 0; a < 3; ++a) roots[((int64_t)a * K + k) * S + n] = cx[sl][0][a];
        rbone[(int64_t)k * S + n] = -1;
      }
      nroots[n] = cnt;
    }
    __syncthreads();
  }
}

// Per sample, the root with the largest density among its n_roots (ties: the
// lower slot, i.e. the lower residual): its point, bone, density and colour.
__global__ void __launch_bounds__(256) select_max_kernel(int K, int64_t S, const float *__restrict__ sigk,
                                                         const float *__restrict__ rgbk, const float *__restrict__ roots,
                                                         const int16_t *__restrict__ rbone,
                                                         const int32_t *__restrict__ nroots, int64_t ld,
                                                         float *__restrict__ xc, int16_t *__restrict__ bone,
                                                         float *__restrict__ sigma, float *__restrict__ rgb) {
  const int64_t KS = (int64_t)K * S;
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < S; n += (int64_t)gridDim.x * 256) {
    const int cnt = nroots[n];
    int best = -1;
    float bs = -INFINITY;
    for (int k = 0; k < cnt && k < K; ++k) {
      const float v = sigk[(int64_t)k * S + n];
      if (v > bs) {
        bs = v;
        best = k;
      }
    }
    const int kk = best < 0 ? 0 : best;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xc[a * ld + n] = roots[((int64_t)a * K + kk) * S + n];
      rgb[a * ld + n] = best < 0 ? 0.0f : rgbk[a * KS + (int64_t)kk * S + n];
    }
    bone[n] = best < 0 ? (int16_t)-1 : rbone[(int64_t)kk * S + n];
    sigma[n] = best < 0 ? 0.0f : bs;
  }
}

__global__ void __launch_bounds__(kSolveBlock) guided_kernel(
    const float *__restrict__ xp_soa, const float *__restrict__ x0_soa, const int16_t *__restrict__ guide,
    int64_t S, const int64_t *__restrict__ S_dev, int64_t ld, const float *__restrict__ A, Grid gr, Box hbox,
    int max_iter, float tol_stop, float tol_valid, float *__restrict__ xc_soa, int16_t *__restrict__ bone_out,
    float *__restrict__ resid_out, int16_t *__restrict__ steps_out, int32_t *__restrict__ queue,
    int32_t *__restrict__ qlen, int16_t *__restrict__ gsteps) {
  const int64_t Sn = count_of(S, S_dev);
  for (int64_t n = (int64_t)blockIdx.x * kSolveBlock + threadIdx.x; n < Sn; n += (int64_t)gridDim.x * kSolveBlock) {
    const float xp[3] = {xp_soa[n], xp_soa[ld + n], xp_soa[2 * ld + n]};
    float x[3] = {x0_soa[n], x0_soa[ld + n], x0_soa[2 * ld + n]};
    const InitResult q = broyden_from(A, gr, x, true, xp, max_iter, tol_stop);
    gsteps[n] = (int16_t)q.steps;
    if (q.ok && q.r < tol_valid && in_hbox(q.x, hbox)) {
      xc_soa[n] = q.x[0];
      xc_soa[ld + n] = q.x[1];
      xc_soa[2 * ld + n] = q.x[2];
      bone_out[n] = guide[n];
      if (resid_out) resid_out[n] = q.r;
      if (steps_out) steps_out[n] = (int16_t)q.steps;
    } else {
      queue[atomicAdd(qlen, 1)] = (int32_t)n;
    }
  }
}

// Fallback: multi-init solve of the queued samples; the blocks loop over
// the queue (its length is known only on the device).
// 32 lanes per queued sample (one init per lane): the queue is short and
// its samples are the slow ones, so latency, not throughput, sets the time.
constexpr int kFbGroup = 32;

__global__ void __launch_bounds__(kSolveBlock) fallback_kernel(
    const float *__restrict__ xp_soa, int64_t ld, const float *__restrict__ B, int nb, const float *__restrict__ A,
    Grid gr, Box hbox, int max_iter, float tol_stop, float tol_valid, float *__restrict__ xc_soa,
    int16_t *__restrict__ bone_out, float *__restrict__ resid_out, int16_t *__restrict__ steps_out,
    const int32_t *__restrict__ queue, const int32_t *__restrict__ qlen, const int16_t *__restrict__ gsteps,
    int32_t *__restrict__ n_fallback) {
  constexpr int kPerBlock = kSolveBlock / kFbGroup;
  const int64_t nq = *qlen;
  if (n_fallback && blockIdx.x == 0 && threadIdx.x == 0) *n_fallback = (int32_t)nq;
  if ((int64_t)blockIdx.x * kPerBlock >= nq) return;  // the whole block is past the queue
  __shared__ float sBinv[kMaxBones * 12];
  __shared__ int sBok[kMaxBones];
  stage_bone_inverses(B, nb, sBinv, sBok);
  __syncthreads();
  const int j = threadIdx.x % kFbGroup;
  for (int64_t q0 = (int64_t)blockIdx.x * kPerBlock; q0 < nq; q0 += (int64_t)gridDim.x * kPerBlock) {
    const int64_t q = q0 + threadIdx.x / kFbGroup;
    const bool act = q < nq;
    const int64_t n = act ? queue[q] : 0;
    float xp[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      xp[0] = xp_soa[n];
      xp[1] = xp_soa[ld + n];
      xp[2] = xp_soa[2 * ld + n];
    }
    const Choice c = multi_init<kFbGroup>(A, gr, sBinv, sBok, nb, xp, act, j, hbox, max_iter, tol_stop, tol_valid);
    if (act && j == 0) write_choice(c, n, ld, gsteps[n], xc_soa, bone_out, resid_out, steps_out);
  }
}

// ------------------------------------------------------------------------
// Backward (implicit function theorem), three kernels:
//  ift_v: one thread per sample: J = sum_b w_b M_b + sum_b y_b grad w_b^T
//         (y_b = B_b x*_h), v = J^{-T} dL/dx*; dL/dx' = v.
//  ift_q: accumulates the per-vertex moment
//         Q_v = sum_s tri_v(x*_s) v_s x*_h,s^T   (3 x 4 per vertex)
//         with FP32 atomics laid out for few cache lines per instruction
//         (12 floats per corner instead of the 24-bone products).  Both
//         parameter gradients are contractions of Q:
//           dL/dW[v][b] = -sum_ij B_b[i][j] Q_v[i][j]
//           dL/dB_b     = -sum_v W[v][b] Q_v
//  ift_contract: one thread per vertex writes its dL/dW row and adds to a
//         block partial of dL/dB;
//  ift_b: sums the dL/dB partials in a fixed order (double).
// ------------------------------------------------------------------------
constexpr int kBwdBlock = 256;
constexpr int kMaxBonesBwd = 32;  // skinning weights of one sample kept in registers
constexpr int kOwnBlock = 256;

__device__ __forceinline__ void ift_v_one(const float *__restrict__ gxc, const float *__restrict__ xc_soa,
                                          const int16_t *__restrict__ bone, int64_t n, int64_t S, int64_t ld,
                                          const float *sB, int nb, const float *__restrict__ W, const Grid &gr,
                                          int w_vec4, float *__restrict__ gxp, float *__restrict__ vbuf) {
  float v[3] = {0.0f, 0.0f, 0.0f};
  if (bone[n] >= 0) {
    const float x[3] = {xc_soa[n], xc_soa[ld + n], xc_soa[2 * ld + n]};
    const Cell c = locate(gr, x);
    int64_t vtx[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      vtx[k] = ((int64_t)(c.i0[2] + ((k >> 2) & 1)) * gr.D[1] + (c.i0[1] + ((k >> 1) & 1))) * gr.D[0] +
               (c.i0[0] + (k & 1));
    float J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    auto add_bone = [&](int b, const float cv[8]) {
      float w = 0.0f, d[3];
#pragma unroll
      for (int k = 0; k < 8; ++k) w += tri_weight(c.f, k) * cv[k];
      tri_grad(cv, c.f, d);
      const float *Bb = sB + 12 * b;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float y = Bb[4 * i] * x[0] + Bb[4 * i + 1] * x[1] + Bb[4 * i + 2] * x[2] + Bb[4 * i + 3];
#pragma unroll
        for (int j = 0; j < 3; ++j) J[i][j] += w * Bb[4 * i + j] + y * (c.dp[j] * d[j]);
      }
    };
    if (w_vec4) {
      // skinning rows as float4: 4 bones of the 8 corners per step
      const int nq = nb >> 2;
      for (int q = 0; q < nq; ++q) {
        float4 c4[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c4[k] = reinterpret_cast<const float4 *>(W + vtx[k] * nb)[q];
        float cv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) cv[k] = c4[k].x;
        add_bone(4 * q, cv);
#pragma unroll
        for (int k = 0; k < 8; ++k) cv[k] = c4[k].y;
        add_bone(4 * q + 1, cv);
#pragma unroll
        for (int k = 0; k < 8; ++k) cv[k] = c4[k].z;
        add_bone(4 * q + 2, cv);
#pragma unroll
        for (int k = 0; k < 8; ++k) cv[k] = c4[k].w;
        add_bone(4 * q + 3, cv);
      }
    } else {
      for (int b = 0; b < nb; ++b) {
        float cv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) cv[k] = W[vtx[k] * nb + b];
        add_bone(b, cv);
      }
    }
    float Ji[3][3];
    inv3(J, Ji);
    const float u[3] = {gxc[n], gxc[ld + n], gxc[2 * ld + n]};
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = Ji[0][a] * u[0] + Ji[1][a] * u[1] + Ji[2][a] * u[2];
  }
  if (gxp) {
    gxp[n] = v[0];
    gxp[ld + n] = v[1];
    gxp[2 * ld + n] = v[2];
  }
  vbuf[n] = v[0];
  vbuf[S + n] = v[1];
  vbuf[2 * S + n] = v[2];
}

// vbuf [3][S] (S = the capacity) holds v for ift_q.
__global__ void __launch_bounds__(kBwdBlock) ift_v_kernel(const float *__restrict__ gxc, const float *__restrict__ xc_soa,
                                                        const int16_t *__restrict__ bone, int64_t S,
                                                        const int64_t *__restrict__ S_dev, int64_t ld,
                                                        const float *__restrict__ B, int nb,
                                                        const float *__restrict__ W, Grid gr, int w_vec4,
                                                        float *__restrict__ gxp, float *__restrict__ vbuf,
                                                        float4 *__restrict__ Qz, int64_t nq4) {
  __shared__ float sB[kMaxBones * 12];
  for (int i = threadIdx.x; i < nb * 12; i += blockDim.x) sB[i] = B[i];
  // the moment buffer of ift_q is cleared here (its stores hide behind the
  // skinning-row gathers)
  for (int64_t i = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x; i < nq4; i += (int64_t)gridDim.x * kBwdBlock)
    Qz[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  const int64_t Sn = count_of(S, S_dev);
  for (int64_t n = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x; n < Sn; n += (int64_t)gridDim.x * kBwdBlock)
    ift_v_one(gxc, xc_soa, bone, n, S, ld, sB, nb, W, gr, w_vec4, gxp, vbuf);
}


// Q_v += tri_v(x*) v x*_h^T: 64 lanes per sample, lane = 8 * corner + slot,
// slots j and j + 8 (< 12) of the corner's 12 floats.  A corner's 12 floats
// are 48 contiguous bytes and x-neighbouring corners are adjacent vertices,
// so each wave instruction touches about four cache lines (FP32 atomics to
// random lines are limited by L2 requests, not by floats).  A wave takes
// kQRun consecutive samples in turn (samples of a ray follow each other, and
// neighbouring samples often share a skinning-grid cell): contributions are
// summed in registers while the cell stays the same and added to Q when it
// changes, which saves the atomics of the repeats.
constexpr int kQRun = 8;

__global__ void __launch_bounds__(kOwnBlock) ift_q_kernel(const float *__restrict__ xc_soa,
                                                        const int16_t *__restrict__ bone, const float *__restrict__ vbuf,
                                                        int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                        Grid gr, float *__restrict__ Q) {
  const int64_t Sn = count_of(S, S_dev);
  const int lane = (int)(threadIdx.x & 63), k = lane >> 3, j = lane & 7;
  constexpr int kWaves = kOwnBlock / 64;
  const int64_t nruns = ceil_div(Sn, (int64_t)kQRun);
  for (int64_t run = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); run < nruns;
       run += (int64_t)gridDim.x * kWaves) {
    // lane i < kQRun loads sample n0 + i; the samples are then taken in turn
    const int64_t n0 = run * kQRun;
    int lb = -1;
    float lx[3] = {0.0f, 0.0f, 0.0f}, lv[3] = {0.0f, 0.0f, 0.0f};
    if (lane < kQRun && n0 + lane < Sn) {
      const int64_t n = n0 + lane;
      lb = bone[n];
      lx[0] = xc_soa[n];
      lx[1] = xc_soa[ld + n];
      lx[2] = xc_soa[2 * ld + n];
      lv[0] = vbuf[n];
      lv[1] = vbuf[S + n];
      lv[2] = vbuf[2 * S + n];
    }
    int64_t cur = -1, cur_vtx = 0;
    float a0 = 0.0f, a1 = 0.0f;
    for (int i = 0; i < kQRun; ++i) {
      if (__shfl(lb, i, kWave) < 0) continue;  // wave-uniform: invalid or past the count
      const float x[3] = {__shfl(lx[0], i, kWave), __shfl(lx[1], i, kWave), __shfl(lx[2], i, kWave)};
      const float v[3] = {__shfl(lv[0], i, kWave), __shfl(lv[1], i, kWave), __shfl(lv[2], i, kWave)};
      const Cell c = locate(gr, x);
      const int64_t base = ((int64_t)c.i0[2] * gr.D[1] + c.i0[1]) * gr.D[0] + c.i0[0];
      const int64_t vtx = ((int64_t)(c.i0[2] + ((k >> 2) & 1)) * gr.D[1] + (c.i0[1] + ((k >> 1) & 1))) * gr.D[0] +
                          (c.i0[0] + (k & 1));
      const float tw = tri_weight(c.f, k);
      const float xh[4] = {x[0], x[1], x[2], 1.0f};
      const float c0 = tw * v[j >> 2] * xh[j & 3];
      const float c1 = j < 4 ? tw * v[2] * xh[j] : 0.0f;
      if (base != cur) {  // wave-uniform
        if (cur >= 0) {
          float *q = Q + 12 * cur_vtx;
          atomicAdd(q + j, a0);
          if (j < 4) atomicAdd(q + 8 + j, a1);
        }
        cur = base;
        cur_vtx = vtx;
        a0 = c0;
        a1 = c1;
      } else {
        a0 += c0;
        a1 += c1;
      }
    }
    if (cur >= 0) {
      float *q = Q + 12 * cur_vtx;
      atomicAdd(q + j, a0);
      if (j < 4) atomicAdd(q + 8 + j, a1);
    }
  }
}

// Contractions of Q over a block of kConBlock vertices:
//   dL/dW[v][b] = -sum_m B_b[m] Q_v[m]      (one output element per thread
//                                           and step: coalesced row stores)
//   partial of sum_v W[v][b] Q_v[m]         (one (b, m) pair per thread)
// Most vertices of the skinning grid are far from every sample and have
// Q_v = 0; a block whose Q rows are all zero writes zero rows and a zero
// partial without reading its W rows.
constexpr int kConBlock = 64;
constexpr int kConThreads = 256;

__global__ void __launch_bounds__(kConThreads) ift_contract_kernel(const float *__restrict__ Q,
                                                                 const float *__restrict__ B, int nb,
                                                                 const float *__restrict__ W, int64_t nvert,
                                                                 float *__restrict__ gW, float *__restrict__ partB,
                                                                 int overwrite) {
  __shared__ float sB[kMaxBones * 12];
  __shared__ float sQ[kConBlock * 12];
  __shared__ float sW[kConBlock * kMaxBones];
  __shared__ int any;
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kConBlock;
  const int nv = (int)min((int64_t)kConBlock, nvert - v0);
  if (tid == 0) any = 0;
  for (int i = tid; i < nb * 12; i += kConThreads) sB[i] = B[i];
  __syncthreads();
  int mine = 0;
  for (int i = tid; i < kConBlock * 12; i += kConThreads) {
    const float q = i < nv * 12 ? Q[v0 * 12 + i] : 0.0f;
    sQ[i] = q;
    mine |= q != 0.0f;
  }
  if (mine) any = 1;
  __syncthreads();
  const bool live = any != 0;
  if (gW) {
    float *out = gW + v0 * nb;
    for (int e = tid; e < nv * nb; e += kConThreads) {
      float s = 0.0f;
      if (live) {
        const int v = e / nb, b = e - v * nb;
        const float *q = sQ + 12 * v, *Bb = sB + 12 * b;
#pragma unroll
        for (int m = 0; m < 12; ++m) s += Bb[m] * q[m];
      }
      if (overwrite) out[e] = -s;
      else out[e] -= s;
    }
  }
  if (partB) {
    if (live)
      for (int i = tid; i < nv * nb; i += kConThreads) sW[i] = W[v0 * nb + i];
    __syncthreads();
    for (int p = tid; p < nb * 12; p += kConThreads) {
      float s0 = 0.0f, s1 = 0.0f;
      if (live) {
        const int b = p / 12, m = p - 12 * (p / 12);
        int e = 0;
        for (; e + 1 < nv; e += 2) {
          s0 += sW[e * nb + b] * sQ[12 * e + m];
          s1 += sW[(e + 1) * nb + b] * sQ[12 * (e + 1) + m];
        }
        if (e < nv) s0 += sW[e * nb + b] * sQ[12 * e + m];
      }
      partB[(int64_t)blockIdx.x * nb * 12 + p] = s0 + s1;
    }
  }
}

// Sum of the dL/dB block partials: 16 entries x 64 partial groups per
// workgroup, each group summed in double with four accumulators, the groups
// combined in a fixed order.
constexpr int kRedP = 16, kRedG = 64;
__global__ void __launch_bounds__(kRedP *kRedG) ift_b_kernel(const float *__restrict__ partB, int nblk, int n,
                                                             float *__restrict__ gB, int overwrite) {
  __shared__ double part[kRedG][kRedP];
  const int pl = threadIdx.x % kRedP, grp = threadIdx.x / kRedP;
  const int p = blockIdx.x * kRedP + pl;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (p < n) {
    int q = grp;
    for (; q + 3 * kRedG < nblk; q += 4 * kRedG) {
      a0 += (double)partB[(int64_t)q * n + p];
      a1 += (double)partB[(int64_t)(q + kRedG) * n + p];
      a2 += (double)partB[(int64_t)(q + 2 * kRedG) * n + p];
      a3 += (double)partB[(int64_t)(q + 3 * kRedG) * n + p];
    }
    for (; q < nblk; q += kRedG) a0 += (double)partB[(int64_t)q * n + p];
  }
  part[grp][pl] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (grp == 0 && p < n) {
    double sum = 0.0;
    for (int g2 = 0; g2 < kRedG; ++g2) sum += part[g2][pl];
    gB[p] = overwrite ? (float)(-sum) : gB[p] - (float)sum;
  }
}

}  // namespace

extern "C" size_t ia355_deform_workspace_size(int32_t Dx, int32_t Dy, int32_t Dz) {
  if (Dx <= 0 || Dy <= 0 || Dz <= 0) return 0;
  return align256(sizeof(float) * 12 * (size_t)Dx * Dy * Dz);
}

namespace {

// Argument checks shared by ia355_snarf_deform and its allocation-free form.
int32_t deform_args_ok(const float *xp, int64_t S, int64_t ld, const float *B, int32_t nb, const float *W, int32_t Dx,
                       int32_t Dy, int32_t Dz, const float *skin_aabb, const float *hash_aabb, int32_t max_iter,
                       const float *xc, const int16_t *bone) {
  if (S < 0 || ld < S || nb <= 0 || nb > kMaxBones || max_iter < 0 || max_iter > 1000) return IA355_ERR_INVALID_ARG;
  if (!B || !W || !grid_ok(Dx, Dy, Dz, skin_aabb) || !hash_aabb) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!xp || !xc || !bone)) return IA355_ERR_INVALID_ARG;
  return IA355_OK;
}

// Blend, then the multi-init solve, with the blended grid A (12 floats per
// vertex) in device memory the caller of this function provides.
int32_t deform_launch(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld, const float *B, int32_t nb,
                      const float *W, int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                      const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid, float *xc,
                      int16_t *bone, float *resid, int16_t *steps, float *A, hipStream_t s) {
  const int64_t nvert = (int64_t)Dx * Dy * Dz;
  blend_kernel<<<(unsigned)ceil_div(nvert, kBlendBlock), kBlendBlock, 0, s>>>(W, B, nb, nvert, A, nullptr);
  if (S == 0) return launch_status();
  const Grid g = make_grid(Dx, Dy, Dz, skin_aabb);
  Box hb;
  for (int a = 0; a < 3; ++a) {
    hb.lo[a] = hash_aabb[a];
    hb.hi[a] = hash_aabb[3 + a];
  }
  solve_kernel<<<stride_grid(ceil_div(S * kGroup, kSolveBlock), S_dev != nullptr), kSolveBlock, 0, s>>>(
      xp, S, S_dev, ld, B, nb, A, g, hb, max_iter, tol_stop, tol_valid, xc, bone, resid, steps);
  return launch_status();
}

}  // namespace

extern "C" int32_t ia355_snarf_deform(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld, const float *B,
                                      int32_t nb,
                                      const float *W, int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                                      const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid,
                                      float *xc, int16_t *bone, float *resid, int16_t *steps, void *ws,
                                      size_t ws_bytes, ia355_stream_t stream) {
  const int32_t st = deform_args_ok(xp, S, ld, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, xc, bone);
  if (st != IA355_OK) return st;
  if (!ws || ws_bytes < ia355_deform_workspace_size(Dx, Dy, Dz)) return IA355_ERR_WORKSPACE;
  return deform_launch(xp, S, S_dev, ld, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid,
                       xc, bone, resid, steps, (float *)ws, as_stream(stream));
}

// ---------------------------------------------------------------------------
// Allocation-free form: the blended grid lives in `scratch`, a file-scope
// device array of IA355_DEFORM_NOALLOC_MAX_VERTS vertices (each GPU the
// library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): the first call on a device looks its address up
// with hipGetSymbolAddress, with that device current, and keeps it per
// device.  The blend kernel overwrites every vertex the solve reads, so
// nothing has to be cleared between calls; calls that overlap on one GPU
// share the array and race.
static __device__ __align__(256) float scratch[12 * (size_t)IA355_DEFORM_NOALLOC_MAX_VERTS];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on device `dev`, looked up once per device.
int32_t scratch_address(int dev, float **out) {
  static std::mutex mu;
  static float *addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return IA355_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return IA355_ERR_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return IA355_ERR_HIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return IA355_ERR_HIP;
    if (e != hipSuccess || !p) return IA355_ERR_HIP;
    addr[dev] = (float *)p;
  }
  *out = addr[dev];
  return IA355_OK;
}

}  // namespace

extern "C" int32_t ia355_snarf_deform_noalloc(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                                              const float *B, int32_t nb, const float *W, int32_t Dx, int32_t Dy,
                                              int32_t Dz, const float *skin_aabb, const float *hash_aabb,
                                              int32_t max_iter, float tol_stop, float tol_valid, float *xc,
                                              int16_t *bone, float *resid, int16_t *steps, ia355_stream_t stream) {
  int32_t st = deform_args_ok(xp, S, ld, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, xc, bone);
  if (st != IA355_OK) return st;
  if ((int64_t)Dx * Dy * Dz > (int64_t)IA355_DEFORM_NOALLOC_MAX_VERTS) return IA355_ERR_SCRATCH;
  hipStream_t s = as_stream(stream);
  int dev = -1;
  if ((s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev)) != hipSuccess) return IA355_ERR_HIP;
  float *A = nullptr;
  st = scratch_address(dev, &A);
  if (st != IA355_OK) return st;
  return deform_launch(xp, S, S_dev, ld, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid,
                       xc, bone, resid, steps, A, s);
}

extern "C" int32_t ia355_snarf_deform_roots(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                                            const float *B, int32_t nb, const float *W, int32_t Dx, int32_t Dy,
                                            int32_t Dz, const float *skin_aabb, const float *hash_aabb,
                                            int32_t max_iter, float tol_stop, float tol_valid, int32_t K,
                                            float dup_tol, float *roots, int16_t *root_bone, int32_t *n_roots,
                                            void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (S < 0 || ld < S || nb <= 0 || nb > kMaxBones || max_iter < 0 || max_iter > 1000) return IA355_ERR_INVALID_ARG;
  if (K < 1 || K > nb || !(dup_tol >= 0.0f)) return IA355_ERR_INVALID_ARG;
  if (!B || !W || !grid_ok(Dx, Dy, Dz, skin_aabb) || !hash_aabb) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!xp || !roots || !root_bone || !n_roots)) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < ia355_deform_workspace_size(Dx, Dy, Dz)) return IA355_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  const int64_t nvert = (int64_t)Dx * Dy * Dz;
  float *A = (float *)ws;
  blend_kernel<<<(unsigned)ceil_div(nvert, kBlendBlock), kBlendBlock, 0, s>>>(W, B, nb, nvert, A, nullptr);
  if (S == 0) return launch_status();
  const Grid g = make_grid(Dx, Dy, Dz, skin_aabb);
  Box hb;
  for (int a = 0; a < 3; ++a) {
    hb.lo[a] = hash_aabb[a];
    hb.hi[a] = hash_aabb[3 + a];
  }
  roots_kernel<<<stride_grid(ceil_div(S, kRootSamples), S_dev != nullptr), kSolveBlock, 0, s>>>(
      xp, S, S_dev, ld, B, nb, A, g, hb, max_iter, tol_stop, tol_valid, K, dup_tol, roots, root_bone, n_roots);
  return launch_status();
}

extern "C" int32_t ia355_select_max_density(int32_t K, int64_t S, const float *sigma_k, const float *rgb_k,
                                            const float *roots, const int16_t *root_bone, const int32_t *n_roots,
                                            int64_t ld, float *xc, int16_t *bone, float *sigma, float *rgb,
                                            ia355_stream_t stream) {
  if (K < 1 || S < 0 || ld < S) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!sigma_k || !rgb_k || !roots || !root_bone || !n_roots || !xc || !bone || !sigma || !rgb))
    return IA355_ERR_INVALID_ARG;
  if (S == 0) return IA355_OK;
  select_max_kernel<<<grid_for(S, 256), 256, 0, as_stream(stream)>>>(K, S, sigma_k, rgb_k, roots, root_bone, n_roots,
                                                                      ld, xc, bone, sigma, rgb);
  return launch_status();
}

extern "C" size_t ia355_deform_guided_workspace_size(int64_t S, int32_t Dx, int32_t Dy, int32_t Dz) {
  if (S < 0) return 0;
  return ia355_deform_workspace_size(Dx, Dy, Dz) + align256(sizeof(int32_t) * (size_t)(S + 1)) +
         align256(sizeof(int16_t) * (size_t)(S > 0 ? S : 1));
}

extern "C" int32_t ia355_snarf_deform_guided(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                                             const float *x0,
                                             const int16_t *guide_bone, const float *B, int32_t nb, const float *W,
                                             int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                                             const float *hash_aabb, int32_t max_iter, float tol_stop,
                                             float tol_valid, float *xc, int16_t *bone, float *resid, int16_t *steps,
                                             int32_t *n_fallback, void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (S < 0 || ld < S || nb <= 0 || nb > kMaxBones || max_iter < 0 || max_iter > 1000) return IA355_ERR_INVALID_ARG;
  if (S > 0x7ffffffeLL) return IA355_ERR_INVALID_ARG;
  if (!B || !W || !grid_ok(Dx, Dy, Dz, skin_aabb) || !hash_aabb) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!xp || !x0 || !guide_bone || !xc || !bone)) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < ia355_deform_guided_workspace_size(S, Dx, Dy, Dz)) return IA355_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  const int64_t nvert = (int64_t)Dx * Dy * Dz;
  float *A = (float *)ws;
  char *p = (char *)ws + ia355_deform_workspace_size(Dx, Dy, Dz);
  int32_t *qlen = (int32_t *)p;
  int32_t *queue = qlen + 1;
  int16_t *gsteps = (int16_t *)(p + align256(sizeof(int32_t) * (size_t)(S + 1)));
  blend_kernel<<<(unsigned)ceil_div(nvert, kBlendBlock), kBlendBlock, 0, s>>>(W, B, nb, nvert, A, qlen);
  int32_t st = IA355_OK;
  if (S > 0) {
    const Grid g = make_grid(Dx, Dy, Dz, skin_aabb);
    Box hb;
    for (int a = 0; a < 3; ++a) {
      hb.lo[a] = hash_aabb[a];
      hb.hi[a] = hash_aabb[3 + a];
    }
    const bool dev = S_dev != nullptr;
    // up to one sample per lane at frame sizes (more waves in flight to
    // hide the gathers' latency)
    guided_kernel<<<stride_grid(ceil_div(S, kSolveBlock), dev, 8192), kSolveBlock, 0, s>>>(
        xp, x0, guide_bone, S, S_dev, ld, A, g, hb, max_iter, tol_stop, tol_valid, xc, bone, resid, steps, queue,
        qlen, gsteps);
    fallback_kernel<<<stride_grid(ceil_div(S * kFbGroup, kSolveBlock), dev), kSolveBlock, 0, s>>>(
        xp, ld, B, nb, A, g, hb, max_iter, tol_stop, tol_valid, xc, bone, resid, steps, queue, qlen, gsteps,
        n_fallback);
  } else if (n_fallback) {
    st = ia355_zero(n_fallback, sizeof(int32_t), stream);
    if (st != IA355_OK) return st;
  }
  return launch_status();
}

extern "C" size_t ia355_deform_bwd_workspace_size(int64_t S, int32_t Dx, int32_t Dy, int32_t Dz, int32_t nb) {
  if (S < 0 || Dx <= 0 || Dy <= 0 || Dz <= 0 || nb <= 0) return 0;
  const int64_t nvert = (int64_t)Dx * Dy * Dz;
  return align256(sizeof(float) * 3 * (size_t)S) + align256(sizeof(float) * 12 * (size_t)nvert) +
         align256(sizeof(float) * 12 * (size_t)nb * ceil_div(nvert, kConBlock));
}

extern "C" int32_t ia355_snarf_deform_bwd(const float *grad_xc, const float *xc, const int16_t *bone, int64_t S,
                                          const int64_t *S_dev, int64_t ld, const float *B, int32_t nb,
                                          const float *W, int32_t Dx,
                                          int32_t Dy, int32_t Dz, const float *skin_aabb, float *grad_xp,
                                          float *grad_B, float *grad_W, uint32_t flags, void *ws, size_t ws_bytes,
                                          ia355_stream_t stream) {
  if (S < 0 || ld < S || nb <= 0 || nb > kMaxBones) return IA355_ERR_INVALID_ARG;
  if (!B || !W || !grid_ok(Dx, Dy, Dz, skin_aabb)) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!grad_xc || !xc || !bone)) return IA355_ERR_INVALID_ARG;
  if (flags & ~(uint32_t)IA355_OVERWRITE) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < ia355_deform_bwd_workspace_size(S, Dx, Dy, Dz, nb)) return IA355_ERR_WORKSPACE;
  const int overwrite = (flags & IA355_OVERWRITE) != 0;
  const Grid g = make_grid(Dx, Dy, Dz, skin_aabb);
  hipStream_t s = as_stream(stream);
  const int64_t nvert = (int64_t)Dx * Dy * Dz;
  const int nblk = (int)ceil_div(nvert, kConBlock);
  float *vbuf = (float *)ws;
  float *Q = (float *)((char *)ws + align256(sizeof(float) * 3 * (size_t)S));
  float *partB = (float *)((char *)Q + align256(sizeof(float) * 12 * (size_t)nvert));
  const bool params = grad_W || grad_B;
  if (S > 0) {
    const int w_vec4 = (nb % 4 == 0) && ((reinterpret_cast<uintptr_t>(W) & 15) == 0);
    // Q (12 floats per vertex, 256-byte aligned in the workspace) is cleared
    // by this kernel when the parameter gradients are wanted
    ift_v_kernel<<<stride_grid(ceil_div(S, kBwdBlock), S_dev != nullptr), kBwdBlock, 0, s>>>(
        grad_xc, xc, bone, S, S_dev, ld, B, nb, W, g, w_vec4, grad_xp, vbuf, params ? (float4 *)Q : nullptr,
        params ? 3 * nvert : 0);
  }
  if (params) {
    if (S == 0) {
      const int32_t st = ia355_zero(Q, sizeof(float) * 12 * (size_t)nvert, stream);
      if (st != IA355_OK) return st;
    }
    if (S > 0)
      ift_q_kernel<<<stride_grid(ceil_div(ceil_div(S, kQRun) * 64, kOwnBlock), S_dev != nullptr, 8192), kOwnBlock, 0,
                     s>>>(
          xc, bone, vbuf, S, S_dev, ld, g, Q);
    ift_contract_kernel<<<(unsigned)nblk, kConThreads, 0, s>>>(Q, B, nb, W, nvert, grad_W, grad_B ? partB : nullptr,
                                                               overwrite);
    if (grad_B)
      ift_b_kernel<<<(unsigned)ceil_div(nb * 12, kRedP), kRedP * kRedG, 0, s>>>(partB, nblk, nb * 12, grad_B, overwrite);
  }
  return launch_status();
}
