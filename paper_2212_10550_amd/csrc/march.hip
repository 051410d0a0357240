// Ray marching with empty-space skipping (Sec. 3.2 ray sampling, Sec. 3.3
// occupancy-grid skipping), as a three-kernel stream compaction:
//   count  -- one thread per ray walks its midpoint samples, counts the ones
//             in occupied cells and writes its block-local exclusive offset;
//   scan   -- one block turns the per-block totals into global offsets;
//   fill   -- one thread per ray walks again and writes its kept samples
//             at its global offset (structure-of-arrays, coalesced per row).
// Every position and keep/skip decision is computed with individually
// rounded IEEE single operations (contraction is switched off: the
// compiler would otherwise fuse o + t d into one FMA), so the sample set is
// exactly reproducible.
#include "common.h"

using namespace ia355;

namespace {

struct Box {
  float lo[3], hi[3];
};

struct RaySpan {
  float tn, tf, dt;
  bool hit;
};

__device__ __forceinline__ RaySpan ray_span(const float o[3], const float d[3], const Box &b, float dt_fixed,
                                            int n_per_ray) {
#pragma clang fp contract(off)
  float tmin = -INFINITY, tmax = INFINITY;
  RaySpan s{0.0f, 0.0f, 0.0f, false};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0f) {
      const float ta = (b.lo[a] - o[a]) / d[a];
      const float tb = (b.hi[a] - o[a]) / d[a];
      const float t0 = ta < tb ? ta : tb;
      const float t1 = ta < tb ? tb : ta;
      if (t0 > tmin) tmin = t0;
      if (t1 < tmax) tmax = t1;
    } else if (o[a] < b.lo[a] || o[a] > b.hi[a]) {
      return s;
    }
  }
  const float tn = tmin > 0.0f ? tmin : 0.0f;
  if (!(tmax > tn)) return s;
  s.tn = tn;
  s.tf = tmax;
  s.dt = n_per_ray > 0 ? (tmax - tn) / (float)n_per_ray : dt_fixed;
  s.hit = true;
  return s;
}

// Sample k of a ray: position and whether its cell is occupied.
__device__ __forceinline__ bool sample_at(const float o[3], const float d[3], const RaySpan &s, int k, const Box &b,
                                          const uint32_t *bits, int G, float *t_out, float x[3]) {
#pragma clang fp contract(off)
  const float t = s.tn + ((float)k + 0.5f) * s.dt;
  *t_out = t;
  int cell[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a] = o[a] + t * d[a];
    const float u = (x[a] - b.lo[a]) / (b.hi[a] - b.lo[a]) * (float)G;
    int c = (int)floorf(u);
    cell[a] = c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
  }
  if (!bits) return true;
  const uint32_t idx = (uint32_t)cell[0] + (uint32_t)G * ((uint32_t)cell[1] + (uint32_t)G * (uint32_t)cell[2]);
  return (bits[idx >> 5] >> (idx & 31)) & 1u;
}

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) march_count(const float *ro, const float *rd, int64_t R,
                                                      const uint32_t *bits, int G, Box box, float dt_fixed,
                                                      int n_per_ray, int max_steps, int64_t *ray_off,
                                                      int32_t *ray_cnt, float *ray_dt, int64_t *block_sum) {
  __shared__ int wsum[kBlock / kWave];
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int cnt = 0;
  if (r < R) {
    const float o[3] = {ro[3 * r], ro[3 * r + 1], ro[3 * r + 2]};
    const float d[3] = {rd[3 * r], rd[3 * r + 1], rd[3 * r + 2]};
    const RaySpan s = ray_span(o, d, box, dt_fixed, n_per_ray);
    if (s.hit) {
      for (int k = 0; k < max_steps; ++k) {
        float t, x[3];
        const bool keep = sample_at(o, d, s, k, box, bits, G, &t, x);
        if (!(t < s.tf)) break;
        cnt += keep;
      }
    }
    ray_cnt[r] = cnt;
    ray_dt[r] = s.dt;
  }
  // block-local exclusive scan of the counts
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int incl = wave_incl_scan(cnt);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  int base = 0;
  for (int i = 0; i < wid; ++i) base += wsum[i];
  if (r < R) ray_off[r] = base + incl - cnt;
  if (threadIdx.x == kBlock - 1) block_sum[blockIdx.x] = base + incl;
}

// Exclusive scan of the per-block totals in one block (in place), total to
// n_samples and ray_off[R].
__global__ void __launch_bounds__(1024) march_scan(int64_t *block_sum, int64_t nblk, int64_t *ray_off, int64_t R,
                                                   int64_t *n_samples) {
  __shared__ int64_t wsum[1024 / kWave];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int64_t b0 = 0; b0 < nblk; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nblk ? block_sum[i] : 0;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t t = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    int64_t base = carry;
    for (int w = 0; w < wid; ++w) base += wsum[w];
    if (i < nblk) block_sum[i] = base + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = base + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    n_samples[0] = carry;
    ray_off[R] = carry;
  }
}

__global__ void __launch_bounds__(kBlock) march_fill(const float *ro, const float *rd, int64_t R,
                                                     const uint32_t *bits, int G, Box box, int max_steps,
                                                     const int64_t *block_off, int64_t *ray_off,
                                                     const float *ray_dt, float *xs, float *ts, int32_t *ray_id,
                                                     int64_t cap) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= R) return;
  int64_t off = ray_off[r] + block_off[blockIdx.x];
  ray_off[r] = off;
  const float o[3] = {ro[3 * r], ro[3 * r + 1], ro[3 * r + 2]};
  const float d[3] = {rd[3 * r], rd[3 * r + 1], rd[3 * r + 2]};
  RaySpan s = ray_span(o, d, box, ray_dt[r], 0);
  if (!s.hit) return;
  s.dt = ray_dt[r];
  for (int k = 0; k < max_steps; ++k) {
    float t, x[3];
    const bool keep = sample_at(o, d, s, k, box, bits, G, &t, x);
    if (!(t < s.tf)) break;
    if (!keep) continue;
    if (off < cap) {
      xs[off] = x[0];
      xs[cap + off] = x[1];
      xs[2 * cap + off] = x[2];
      ts[off] = t;
      ray_id[off] = (int32_t)r;
    }
    ++off;
  }
}

}  // namespace

extern "C" size_t ia355_march_workspace_size(int64_t R) {
  return align256(sizeof(int64_t) * (size_t)(ceil_div(R > 0 ? R : 1, kBlock)));
}

extern "C" int32_t ia355_occgrid_march(const float *rays_o, const float *rays_d, int64_t R, const uint32_t *occ_bits,
                                       int32_t G, const float *aabb, float dt, int32_t n_per_ray, int32_t max_steps,
                                       float *xs, float *ts, int32_t *ray_id, int64_t cap, int64_t *ray_off,
                                       int32_t *ray_cnt, float *ray_dt, int64_t *n_samples, void *ws,
                                       size_t ws_bytes, ia355_stream_t stream) {
  if (R < 0 || !aabb || max_steps < 0 || cap < 0) return IA355_ERR_INVALID_ARG;
  if (!ray_off || !n_samples) return IA355_ERR_INVALID_ARG;
  if (R > 0 && (!rays_o || !rays_d || !ray_cnt || !ray_dt)) return IA355_ERR_INVALID_ARG;
  if (cap > 0 && (!xs || !ts || !ray_id)) return IA355_ERR_INVALID_ARG;
  if (occ_bits && (G <= 0 || G > 2048)) return IA355_ERR_INVALID_ARG;
  if (n_per_ray <= 0 && !(dt > 0.0f)) return IA355_ERR_INVALID_ARG;
  if ((int64_t)cap * 3 < cap) return IA355_ERR_INVALID_ARG;
  if (ws_bytes < ia355_march_workspace_size(R) || !ws) return IA355_ERR_WORKSPACE;
  Box box;
  for (int a = 0; a < 3; ++a) {
    box.lo[a] = aabb[a];
    box.hi[a] = aabb[3 + a];
    if (!(box.hi[a] > box.lo[a])) return IA355_ERR_INVALID_ARG;
  }
  hipStream_t s = as_stream(stream);
  int64_t *block_sum = (int64_t *)ws;
  const int64_t nblk = ceil_div(R, kBlock);
  if (R > 0)
    march_count<<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray, max_steps,
                                                  ray_off, ray_cnt, ray_dt, block_sum);
  march_scan<<<1, 1024, 0, s>>>(block_sum, nblk, ray_off, R, n_samples);
  if (R > 0)
    march_fill<<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, max_steps, block_sum, ray_off,
                                                 ray_dt, xs, ts, ray_id, cap);
  return launch_status();
}
