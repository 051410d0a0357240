// Ray marching with empty-space skipping (Sec. 3.2 ray sampling, Sec. 3.3
// occupancy-grid skipping), as a three-kernel stream compaction:
//   count  -- one wave per ray, one lane per midpoint sample: a ballot of
//             the samples in occupied cells gives the ray's count;
//   scan   -- one block turns the per-block totals into global offsets;
//   fill   -- one wave per ray again; each kept sample's slot is the ray's
//             offset plus the popcount of kept lanes below it, so a ray's
//             samples are written in t order by consecutive lanes
//             (structure-of-arrays, coalesced).
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

// One wave per ray: lane l handles steps k = l, l + 64, ... of its ray, so a
// 128-step ray is two ballots.  kRays rays per workgroup.
constexpr int kRays = 4;
constexpr int kBlock = kRays * kWave;

__device__ __forceinline__ void load_ray(const float *ro, const float *rd, int64_t r, float o[3], float d[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = ro[3 * r + a];
    d[a] = rd[3 * r + a];
  }
}

__global__ void __launch_bounds__(kBlock) march_count(const float *ro, const float *rd, int64_t R,
                                                      const uint32_t *bits, int G, Box box, float dt_fixed,
                                                      int n_per_ray, int max_steps, int64_t *ray_off,
                                                      int32_t *ray_cnt, float *ray_dt, int64_t *block_sum) {
  __shared__ int cnts[kRays];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t r = (int64_t)blockIdx.x * kRays + wid;
  int cnt = 0;
  if (r < R) {
    float o[3], d[3];
    load_ray(ro, rd, r, o, d);
    const RaySpan s = ray_span(o, d, box, dt_fixed, n_per_ray);
    if (s.hit) {
      for (int k0 = 0; k0 < max_steps; k0 += kWave) {
        const int k = k0 + lane;
        float t = 0.0f, x[3];
        bool keep = false, inside = false;
        if (k < max_steps) {
          keep = sample_at(o, d, s, k, box, bits, G, &t, x);
          inside = t < s.tf;
          keep = keep && inside;
        }
        cnt += __popcll(__ballot(keep));
        // t grows with k: once the last lane is beyond t_far, so is every later step
        if (!__shfl((int)inside, kWave - 1, kWave)) break;
      }
    }
    if (lane == 0) {
      ray_cnt[r] = cnt;
      ray_dt[r] = s.dt;
    }
  }
  if (lane == 0) cnts[wid] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int i = 0; i < kRays; ++i) {
      const int64_t ri = (int64_t)blockIdx.x * kRays + i;
      if (ri < R) ray_off[ri] = acc;
      acc += cnts[i];
    }
    block_sum[blockIdx.x] = acc;
  }
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
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t r = (int64_t)blockIdx.x * kRays + wid;
  if (r >= R) return;
  int64_t off = ray_off[r] + block_off[blockIdx.x];
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) ray_off[r] = off;
  float o[3], d[3];
  load_ray(ro, rd, r, o, d);
  RaySpan s = ray_span(o, d, box, ray_dt[r], 0);
  if (!s.hit) return;
  s.dt = ray_dt[r];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int k0 = 0; k0 < max_steps; k0 += kWave) {
    const int k = k0 + lane;
    float t = 0.0f, x[3];
    bool keep = false, inside = false;
    if (k < max_steps) {
      keep = sample_at(o, d, s, k, box, bits, G, &t, x);
      inside = t < s.tf;
      keep = keep && inside;
    }
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int64_t at = off + __popcll(m & below);
      if (at < cap) {
        xs[at] = x[0];
        xs[cap + at] = x[1];
        xs[2 * cap + at] = x[2];
        ts[at] = t;
        ray_id[at] = (int32_t)r;
      }
    }
    off += __popcll(m);
    if (!__shfl((int)inside, kWave - 1, kWave)) break;
  }
}

}  // namespace

extern "C" size_t ia355_march_workspace_size(int64_t R) {
  return align256(sizeof(int64_t) * (size_t)(ceil_div(R > 0 ? R : 1, kRays)));
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
  const int64_t nblk = ceil_div(R, kRays);
  if (R > 0)
    march_count<<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray, max_steps,
                                                  ray_off, ray_cnt, ray_dt, block_sum);
  march_scan<<<1, 1024, 0, s>>>(block_sum, nblk, ray_off, R, n_samples);
  if (R > 0 && cap > 0)
    march_fill<<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, max_steps, block_sum, ray_off,
                                                 ray_dt, xs, ts, ray_id, cap);
  return launch_status();
}
