// Volume rendering (Sec. 3.2, Eq. 8) with early ray termination (Sec. 3.4),
// forward and backward.  alpha_i = -expm1(-sigma_i delta) and
// T_{i+1} = T_i exp(-sigma_i delta) (the same quantities as 1 - exp(-sigma
// delta) and T_i (1 - alpha_i), without the cancellation of 1 - exp(.) for
// small sigma delta).
//
// A ray is a segment of 16 lanes (four rays per wave) that walks its
// compacted samples 16 at a time: within a chunk the transmittances are a
// product scan of exp(-sigma delta) across the lanes (and, backward, the
// partial colours sum_{j<=i} w_j c_j a sum scan), carried from chunk to
// chunk.  Densities are non-negative, so T never grows along a ray and the
// samples kept by the termination test T_i >= T_thresh are a prefix of the
// chunk; the ray stops at the first chunk that has an unused sample.
#include "common.h"
#include "render_dev.h"

using namespace ia355;
using namespace ia355::rnd;

namespace {

constexpr int kBlock = 256;
constexpr int kRaysPerBlock = kBlock / kSeg;
__global__ void __launch_bounds__(kBlock) render_fwd(const float *__restrict__ sigma, const float *__restrict__ rgb,
                                                     int64_t ld, const int64_t *__restrict__ ray_off,
                                                     const float *__restrict__ ray_dt, int64_t R, float T_thresh,
                                                     float *__restrict__ color, float *__restrict__ opacity,
                                                     int32_t *__restrict__ n_used, float *__restrict__ T_final) {
  const int j = threadIdx.x % kSeg;
  const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + threadIdx.x / kSeg;
  if (r >= R) return;  // whole segments leave together
  // a march that overflowed the sample buffer (count > ld, reported by the
  // march) leaves offsets past ld: those samples were never written
  const int64_t b = min(ray_off[r], ld), e = min(ray_off[r + 1], ld);
  const RayOut q = composite_ray(PlanarSrc{sigma, rgb, ld}, b, e, ray_dt[r], T_thresh, j);
  if (j == 0) {
    color[3 * r] = q.C[0];
    color[3 * r + 1] = q.C[1];
    color[3 * r + 2] = q.C[2];
    opacity[r] = q.A;
    n_used[r] = q.used;
    T_final[r] = q.T;
  }
}

__global__ void __launch_bounds__(kBlock) render_bwd(const float *__restrict__ gC, const float *__restrict__ gA,
                                                     const float *__restrict__ sigma, const float *__restrict__ rgb,
                                                     int64_t ld, const int64_t *__restrict__ ray_off,
                                                     const float *__restrict__ ray_dt, const int32_t *__restrict__ n_used,
                                                     const float *__restrict__ color, const float *__restrict__ T_final,
                                                     int64_t R, float *__restrict__ gsig, float *__restrict__ grgb) {
  const int j = threadIdx.x % kSeg;
  const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + threadIdx.x / kSeg;
  if (r >= R) return;
  const int64_t b = min(ray_off[r], ld), e = min(ray_off[r + 1], ld), u = min(b + n_used[r], e);
  const float dt = ray_dt[r];
  const float g0 = gC[3 * r], g1 = gC[3 * r + 1], g2 = gC[3 * r + 2];
  const float ga = gA ? gA[r] : 0.0f;
  const float Cc0 = color[3 * r], Cc1 = color[3 * r + 1], Cc2 = color[3 * r + 2];
  const float tail = ga * dt * T_final[r];
  float T = 1.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;  // carried into each chunk
  for (int64_t base = b; base < e; base += kSeg) {
    const int64_t i = base + j;
    const bool use = i < u;
    float x = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    if (use) {
      x = sigma[i] * dt;
      c0 = rgb[i];
      c1 = rgb[ld + i];
      c2 = rgb[2 * ld + i];
    }
    const float ex = use ? expf(-x) : 1.0f;
    float prod;
    const float Ti = seg_trans(T, ex, j, &prod);
    const float w = use ? Ti * -expm1f(-x) : 0.0f;
    const float Q0 = P0 + seg_scan_add(w * c0, j), Q1 = P1 + seg_scan_add(w * c1, j),
                Q2 = P2 + seg_scan_add(w * c2, j);  // sum over samples up to and including i
    if (i < e) {
      if (use) {
        const float gc = g0 * c0 + g1 * c1 + g2 * c2;
        const float after = g0 * (Cc0 - Q0) + g1 * (Cc1 - Q1) + g2 * (Cc2 - Q2);
        gsig[i] = dt * (Ti * ex * gc - after) + tail;
        grgb[i] = w * g0;
        grgb[ld + i] = w * g1;
        grgb[2 * ld + i] = w * g2;
      } else {
        gsig[i] = 0.0f;
        grgb[i] = 0.0f;
        grgb[ld + i] = 0.0f;
        grgb[2 * ld + i] = 0.0f;
      }
    }
    T *= prod;
    P0 = __shfl(Q0, kSeg - 1, kSeg);
    P1 = __shfl(Q1, kSeg - 1, kSeg);
    P2 = __shfl(Q2, kSeg - 1, kSeg);
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
  render_fwd<<<(unsigned)ceil_div(R, kRaysPerBlock), kBlock, 0, as_stream(stream)>>>(
      sigma, rgb, ld, ray_off, ray_dt, R, T_thresh, color, opacity, n_used, T_final);
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
  render_bwd<<<(unsigned)ceil_div(R, kRaysPerBlock), kBlock, 0, as_stream(stream)>>>(
      grad_color, grad_opacity, sigma, rgb, ld, ray_off, ray_dt, n_used, color, T_final, R, grad_sigma, grad_rgb);
  return launch_status();
}
