// Volume rendering (Sec. 3.2, Eq. 8) with early ray termination (Sec. 3.4),
// forward and backward, one thread per ray walking its compacted samples in
// order.  alpha_i = -expm1(-sigma_i delta) and T_{i+1} = T_i exp(-sigma_i delta)
// (the same quantities as 1 - exp(-sigma delta) and T_i (1 - alpha_i),
// without the cancellation of 1 - exp(.) for small sigma delta).
#include "common.h"

using namespace ia355;

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) render_fwd(const float *__restrict__ sigma, const float *__restrict__ rgb,
                                                     int64_t ld, const int64_t *__restrict__ ray_off,
                                                     const float *__restrict__ ray_dt, int64_t R, float T_thresh,
                                                     float *__restrict__ color, float *__restrict__ opacity,
                                                     int32_t *__restrict__ n_used, float *__restrict__ T_final) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= R) return;
  // a march that overflowed the sample buffer (count > ld, reported by the
  // march) leaves offsets past ld: those samples were never written
  const int64_t b = min(ray_off[r], ld), e = min(ray_off[r + 1], ld);
  const float dt = ray_dt[r];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, A = 0.0f;
  int used = 0;
  for (int64_t i = b; i < e; ++i) {
    if (T < T_thresh) break;
    const float x = sigma[i] * dt;
    const float alpha = -expm1f(-x);
    const float w = T * alpha;
    C0 += w * rgb[i];
    C1 += w * rgb[ld + i];
    C2 += w * rgb[2 * ld + i];
    A += w;
    T *= expf(-x);
    ++used;
  }
  color[3 * r] = C0;
  color[3 * r + 1] = C1;
  color[3 * r + 2] = C2;
  opacity[r] = A;
  n_used[r] = used;
  T_final[r] = T;
}

__global__ void __launch_bounds__(kBlock) render_bwd(const float *__restrict__ gC, const float *__restrict__ gA,
                                                     const float *__restrict__ sigma, const float *__restrict__ rgb,
                                                     int64_t ld, const int64_t *__restrict__ ray_off,
                                                     const float *__restrict__ ray_dt, const int32_t *__restrict__ n_used,
                                                     const float *__restrict__ color, const float *__restrict__ T_final,
                                                     int64_t R, float *__restrict__ gsig, float *__restrict__ grgb) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= R) return;
  const int64_t b = min(ray_off[r], ld), e = min(ray_off[r + 1], ld), u = min(b + n_used[r], e);
  const float dt = ray_dt[r];
  const float g0 = gC[3 * r], g1 = gC[3 * r + 1], g2 = gC[3 * r + 2];
  const float ga = gA ? gA[r] : 0.0f;
  const float Cc0 = color[3 * r], Cc1 = color[3 * r + 1], Cc2 = color[3 * r + 2];
  const float tail = ga * dt * T_final[r];
  float T = 1.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
  for (int64_t i = b; i < u; ++i) {
    const float x = sigma[i] * dt;
    const float alpha = -expm1f(-x);
    const float w = T * alpha;
    const float c0 = rgb[i], c1 = rgb[ld + i], c2 = rgb[2 * ld + i];
    P0 += w * c0;
    P1 += w * c1;
    P2 += w * c2;
    const float Tn = T * expf(-x);
    const float gc = g0 * c0 + g1 * c1 + g2 * c2;
    const float after = g0 * (Cc0 - P0) + g1 * (Cc1 - P1) + g2 * (Cc2 - P2);
    gsig[i] = dt * (Tn * gc - after) + tail;
    grgb[i] = w * g0;
    grgb[ld + i] = w * g1;
    grgb[2 * ld + i] = w * g2;
    T = Tn;
  }
  for (int64_t i = u; i < e; ++i) {
    gsig[i] = 0.0f;
    grgb[i] = 0.0f;
    grgb[ld + i] = 0.0f;
    grgb[2 * ld + i] = 0.0f;
  }
}

}  // namespace

extern "C" int32_t ia355_volrender_fwd(const float *sigma, const float *rgb, int64_t ld, const int64_t *ray_off,
                                       const float *ray_dt, int64_t R, float T_thresh, float *color, float *opacity,
                                       int32_t *n_used, float *T_final, ia355_stream_t stream) {
  if (R < 0 || ld < 0) return IA355_ERR_INVALID_ARG;
  if (R == 0) return IA355_OK;
  if (!ray_off || !ray_dt || !color || !opacity || !n_used || !T_final) return IA355_ERR_INVALID_ARG;
  if (ld > 0 && (!sigma || !rgb)) return IA355_ERR_INVALID_ARG;
  render_fwd<<<(unsigned)ceil_div(R, kBlock), kBlock, 0, as_stream(stream)>>>(sigma, rgb, ld, ray_off, ray_dt, R,
                                                                              T_thresh, color, opacity, n_used, T_final);
  return launch_status();
}

extern "C" int32_t ia355_volrender_bwd(const float *grad_color, const float *grad_opacity, const float *sigma,
                                       const float *rgb, int64_t ld, const int64_t *ray_off, const float *ray_dt,
                                       const int32_t *n_used, const float *color, const float *T_final, int64_t R,
                                       float *grad_sigma, float *grad_rgb, ia355_stream_t stream) {
  if (R < 0 || ld < 0) return IA355_ERR_INVALID_ARG;
  if (R == 0) return IA355_OK;
  if (!grad_color || !ray_off || !ray_dt || !n_used || !color || !T_final) return IA355_ERR_INVALID_ARG;
  if (ld > 0 && (!sigma || !rgb || !grad_sigma || !grad_rgb)) return IA355_ERR_INVALID_ARG;
  render_bwd<<<(unsigned)ceil_div(R, kBlock), kBlock, 0, as_stream(stream)>>>(grad_color, grad_opacity, sigma, rgb, ld,
                                                                              ray_off, ray_dt, n_used, color, T_final,
                                                                              R, grad_sigma, grad_rgb);
  return launch_status();
}
