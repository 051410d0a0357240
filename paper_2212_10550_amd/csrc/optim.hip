// Training loss of Sec. 3.4 and the Adam update of the field's parameters.
//
// Loss, averaged over the R rays: the Huber function of the colour error
// norm (L_rgb), lam_alpha |A - A_gt| (L_alpha, A the rendered opacity) and
// lam_hard (-log(exp(-|A|) + exp(-|A - 1|)) + log(1 + exp(-1))) (L_hard, the
// constant makes its minimum zero).  One workgroup sums the rays in a fixed
// order and writes the gradients with respect to the colour and the opacity
// that the compositing backward takes.
//
// Adam (bias-corrected) over a flat FP32 parameter array; the FP16 copy of
// the hash table read by the mixed-precision forward is written in the same
// pass.  The step count may live in device memory (incremented once per
// step by its own call), so a captured training loop needs no host value.
#include <hip/hip_fp16.h>

#include "common.h"

using namespace ia355;

namespace {

constexpr int kLossBlock = 1024;
constexpr float kHardConst = 0.31326168751822284f;  // log(1 + e^-1)

__device__ __forceinline__ float sgnf(float v) { return v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f); }

__global__ void __launch_bounds__(kLossBlock) loss_full_kernel(const float *__restrict__ color,
                                                               const float *__restrict__ opacity,
                                                               const float *__restrict__ target,
                                                               const float *__restrict__ alpha_gt, int64_t R,
                                                               float delta, float lam_alpha, float lam_hard,
                                                               float *__restrict__ loss, float *__restrict__ gC,
                                                               float *__restrict__ gA) {
  __shared__ float part[3][kLossBlock / kWave];
  const float inv_r = 1.0f / (float)R;
  float s_rgb = 0.0f, s_alpha = 0.0f, s_hard = 0.0f;
  for (int64_t r = threadIdx.x; r < R; r += kLossBlock) {
    float e[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) e[c] = color[3 * r + c] - target[3 * r + c];
    const float rn = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const bool quad = rn <= delta;
    s_rgb += quad ? 0.5f * rn * rn : delta * (rn - 0.5f * delta);
    const float scale = (quad ? 1.0f : delta / rn) * inv_r;
#pragma unroll
    for (int c = 0; c < 3; ++c) gC[3 * r + c] = e[c] * scale;
    const float A = opacity[r];
    float g = 0.0f;
    if (alpha_gt) {
      const float d = A - alpha_gt[r];
      s_alpha += fabsf(d);
      g += lam_alpha * sgnf(d);
    }
    const float ea = expf(-fabsf(A)), eb = expf(-fabsf(A - 1.0f));
    s_hard += -logf(ea + eb) + kHardConst;
    g += lam_hard * (ea * sgnf(A) + eb * sgnf(A - 1.0f)) / (ea + eb);
    gA[r] = g * inv_r;
  }
  const float v[3] = {wave_sum(s_rgb), wave_sum(s_alpha), wave_sum(s_hard)};
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) part[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    float t[3] = {0.0f, 0.0f, 0.0f};
    for (int i = 0; i < kLossBlock / kWave; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) t[k] += part[k][i];
    const float rgb = t[0] * inv_r, al = lam_alpha * t[1] * inv_r, hd = lam_hard * t[2] * inv_r;
    loss[0] = rgb + (alpha_gt ? al : 0.0f) + hd;
    loss[1] = rgb;
    loss[2] = alpha_gt ? al : 0.0f;
    loss[3] = hd;
  }
}

constexpr int kAdamBlock = 256;

__global__ void __launch_bounds__(kAdamBlock) adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                          float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                          float lr, float beta1, float beta2, float eps, int32_t step,
                                                          const int32_t *__restrict__ step_dev,
                                                          __half *__restrict__ p16) {
  const int32_t t = step_dev ? *step_dev : step;
  const float c1 = 1.0f / (1.0f - powf(beta1, (float)t));
  const float c2 = 1.0f / (1.0f - powf(beta2, (float)t));
  for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kAdamBlock) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (p16) p16[i] = __float2half_rn(pi);
  }
}

__global__ void step_count_kernel(int32_t *step_dev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step_dev[0] += 1;  // vector store (a global store from lane 0)
}

}  // namespace

extern "C" int32_t ia355_loss_full(const float *color, const float *opacity, const float *target,
                                   const float *alpha_gt, int64_t R, float delta, float lam_alpha, float lam_hard,
                                   float *loss, float *grad_color, float *grad_opacity, ia355_stream_t stream) {
  if (R <= 0 || !color || !opacity || !target || !loss || !grad_color || !grad_opacity) return IA355_ERR_INVALID_ARG;
  if (!(delta > 0.0f)) return IA355_ERR_INVALID_ARG;
  loss_full_kernel<<<1, kLossBlock, 0, as_stream(stream)>>>(color, opacity, target, alpha_gt, R, delta, lam_alpha,
                                                             lam_hard, loss, grad_color, grad_opacity);
  return launch_status();
}

extern "C" int32_t ia355_count_step(int32_t *step_dev, ia355_stream_t stream) {
  if (!step_dev) return IA355_ERR_INVALID_ARG;
  step_count_kernel<<<1, 64, 0, as_stream(stream)>>>(step_dev);
  return launch_status();
}

extern "C" int32_t ia355_adam(float *param, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                              float beta2, float eps, int32_t step, const int32_t *step_dev, void *param_f16,
                              ia355_stream_t stream) {
  if (n < 0 || (n > 0 && (!param || !grad || !m || !v))) return IA355_ERR_INVALID_ARG;
  if (!step_dev && step < 1) return IA355_ERR_INVALID_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f)) return IA355_ERR_INVALID_ARG;
  if (n > 0)
    adam_kernel<<<grid_for(n, kAdamBlock, 256 * 8), kAdamBlock, 0, as_stream(stream)>>>(
        param, grad, m, v, n, lr, beta1, beta2, eps, step, step_dev, (__half *)param_f16);
  return launch_status();
}
