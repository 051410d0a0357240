// Ray marching with empty-space skipping (Sec. 3.2 ray sampling, Sec. 3.3
// occupancy-grid skipping), as a stream compaction in four kernels:
//   count  -- one wave per ray, one lane per midpoint sample: a ballot of
//             the samples in occupied cells gives the ray's count, and the
//             block's total;
//   chunk  -- each block scans 4096 block totals (exclusive, in place) and
//             writes its chunk total;
//   top    -- one block scans the chunk totals and writes the sample count
//             (skipped when there is one chunk: the chunk kernel writes it);
//   fill   -- one wave per ray again, from the keep masks the count kernel
//             saved (one 64-bit ballot per 64 steps) and the ray's entry
//             distance: only kept samples' positions are recomputed (the same
//             expression, so the same floats), no cell lookups; each kept
//             sample's slot is the ray's offset plus the popcount of kept
//             lanes below it, so a ray's samples are written in t order by
//             consecutive lanes (structure-of-arrays, coalesced).
// The occupancy bits are stored in bricks of 8 x 8 x 16 cells, one 128-byte
// cache line each, so the consecutive samples of a ray (one wave) touch a
// few lines rather than one line per sample.
// Every position and keep/skip decision is computed with individually
// rounded IEEE single operations (contraction is switched off: the
// compiler would otherwise fuse o + t d into one FMA), so the sample set is
// exactly reproducible.
#include <cmath>

#include "common.h"
#include "march_dev.h"

using namespace ia355;
using namespace ia355::mch;

namespace {

// kRaysPerWave rays per wave, four waves per workgroup: lane l handles
// steps k = l, l + 64, ... of each of the wave's rays, so a 128-step ray is
// two ballots, and the occupancy loads of the wave's rays (two words at a
// time) are in flight together.  Large ray counts take four rays per wave
// (fewer, longer waves); small ones one ray per wave, which keeps enough
// waves in flight.
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWavesPerBlock * kWave;
constexpr int64_t kManyRays = 65536;  // from here on, four rays per wave

__host__ __device__ inline int rays_per_wave(int64_t R) { return R >= kManyRays ? 4 : 1; }
__host__ __device__ inline int rays_per_block(int64_t R) { return rays_per_wave(R) * kWavesPerBlock; }

template <bool kPow2Ext, int kRaysPerWave>
__global__ void __launch_bounds__(kBlock) march_count(const float *ro, const float *rd, int64_t R,
                                                      const uint32_t *bits, int G, Box box, float dt_fixed,
                                                      int n_per_ray, int max_steps, int64_t *ray_off,
                                                      int32_t *ray_cnt, float *ray_dt, int64_t *block_sum,
                                                      uint64_t *masks, int nw, float *ray_tn) {
  constexpr int kRays = kRaysPerWave * kWavesPerBlock;
  __shared__ int cnts[kRays];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t r0 = (int64_t)blockIdx.x * kRays + wid * kRaysPerWave;
  float o[kRaysPerWave][3], d[kRaysPerWave][3];
  RaySpan s[kRaysPerWave];
#pragma unroll
  for (int u = 0; u < kRaysPerWave; ++u) {
    const int64_t r = r0 + u < R ? r0 + u : R - 1;  // a tail wave repeats the last ray, writes nothing for it
    load_ray(ro, rd, r, o[u], d[u]);
    s[u] = ray_span(o[u], d[u], box, dt_fixed, n_per_ray);
  }
  int cnt[kRaysPerWave];
#pragma unroll
  for (int u = 0; u < kRaysPerWave; ++u) cnt[u] = 0;
  for (int w0 = 0; w0 < nw; w0 += 2) {
    bool keep[kRaysPerWave][2];
#pragma unroll
    for (int u = 0; u < kRaysPerWave; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = (w0 + h) * kWave + lane;
        float t = 0.0f, x[3];
        keep[u][h] = false;
        // a step past t_far is not kept, so its cell is not looked up
        if (s[u].hit && k < max_steps && step_t(s[u], k) < s[u].tf)
          keep[u][h] = sample_at<kPow2Ext>(o[u], d[u], s[u], k, box, bits, G, &t, x) && t < s[u].tf;
      }
#pragma unroll
    for (int u = 0; u < kRaysPerWave; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t m = __ballot(keep[u][h]);
        cnt[u] += __popcll(m);
        if (lane == 0 && r0 + u < R && w0 + h < nw) masks[(r0 + u) * nw + w0 + h] = m;
      }
  }
#pragma unroll
  for (int u = 0; u < kRaysPerWave; ++u) {
    if (lane == 0 && r0 + u < R) {
      ray_cnt[r0 + u] = cnt[u];
      ray_dt[r0 + u] = s[u].dt;
      ray_tn[r0 + u] = s[u].tn;
    }
    if (lane == 0) cnts[wid * kRaysPerWave + u] = r0 + u < R ? cnt[u] : 0;
  }
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

// Exclusive scan in one block of 1024 threads: thread t holds `v`; returns
// the sum of the values of threads below it, and the block total in *total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *wsum, int64_t *total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int64_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  int64_t base = 0, all = 0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    base += w < wid ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - v;
}

// Chunk c of the per-block totals, kScanPer per thread: exclusive scan in
// place (offsets within the chunk) and the chunk's total.
constexpr int kScanPer = 4;
constexpr int64_t kScanChunk = 1024 * kScanPer;

__global__ void __launch_bounds__(1024) march_scan_chunk(int64_t *block_sum, int64_t nblk, int64_t *chunk_sum,
                                                         int64_t *ray_off, int64_t R, int64_t *n_samples) {
  __shared__ int64_t wsum[1024 / kWave];
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer], run = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    v[j] = i0 + j < nblk ? block_sum[i0 + j] : 0;
    run += v[j];
  }
  int64_t total;
  int64_t off = block_exclusive_scan(run, wsum, &total);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    if (i0 + j < nblk) block_sum[i0 + j] = off;
    off += v[j];
  }
  if (threadIdx.x == 0) {
    chunk_sum[blockIdx.x] = total;
    if (gridDim.x == 1) {  // a single chunk: its total is the sample count
      chunk_sum[0] = 0;
      n_samples[0] = total;
      ray_off[R] = total;
    }
  }
}

// Exclusive scan of the chunk totals (in place) in one block; the grand
// total goes to n_samples and ray_off[R].
__global__ void __launch_bounds__(1024) march_scan_top(int64_t *chunk_sum, int64_t nchunk, int64_t *ray_off,
                                                       int64_t R, int64_t *n_samples) {
  __shared__ int64_t wsum[1024 / kWave];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nchunk; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nchunk ? chunk_sum[i] : 0;
    int64_t total;
    const int64_t off = block_exclusive_scan(v, wsum, &total);
    if (i < nchunk) chunk_sum[i] = carry + off;
    carry += total;
  }
  if (threadIdx.x == 0) {
    n_samples[0] = carry;
    ray_off[R] = carry;
  }
}

template <int kRaysPerWave>
__global__ void __launch_bounds__(kBlock) march_fill(const float *__restrict__ ro, const float *__restrict__ rd,
                                                     int64_t R, const uint64_t *__restrict__ masks, int nw,
                                                     const float *__restrict__ ray_tn, const int64_t *block_off,
                                                     const int64_t *chunk_off, int64_t *ray_off,
                                                     const float *__restrict__ ray_dt, float *xs, float *ts,
                                                     int32_t *ray_id, int64_t cap) {
#pragma clang fp contract(off)
  constexpr int kRays = kRaysPerWave * kWavesPerBlock;
  // the wave index is uniform: a ray's inputs and masks go through the
  // scalar cache
  const int lane = threadIdx.x & (kWave - 1), wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int64_t r0 = (int64_t)blockIdx.x * kRays + wid * kRaysPerWave;
  if (r0 >= R) return;
  const int64_t base = block_off[blockIdx.x] + chunk_off[blockIdx.x / kScanChunk];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  // every ray's inputs first, so that their loads are in flight together
  float o[kRaysPerWave][3], d[kRaysPerWave][3], tn[kRaysPerWave], dt[kRaysPerWave];
  int64_t off[kRaysPerWave];
#pragma unroll
  for (int u = 0; u < kRaysPerWave; ++u) {
    const int64_t r = r0 + u < R ? r0 + u : R - 1;
    load_ray(ro, rd, r, o[u], d[u]);
    tn[u] = ray_tn[r];
    dt[u] = ray_dt[r];
    off[u] = ray_off[r] + base;
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int u = 0; u < kRaysPerWave; ++u) {
    const int64_t r = r0 + u;
    if (r >= R) break;
    if (lane == 0) ray_off[r] = off[u];
    const uint64_t *mr = masks + r * nw;
    int64_t at0 = off[u];
    for (int w = 0; w < nw; ++w) {
      const uint64_t m = mr[w];
      if (m == 0ull) continue;
      if ((m >> lane) & 1ull) {
        const int64_t at = at0 + __popcll(m & below);
        if (at < cap) {
          float t, x[3];
          sample_pos(o[u], d[u], tn[u], dt[u], w * kWave + lane, &t, x);
          xs[at] = x[0];
          xs[cap + at] = x[1];
          xs[2 * cap + at] = x[2];
          ts[at] = t;
          ray_id[at] = (int32_t)r;
        }
      }
      at0 += __popcll(m);
    }
  }
}

}  // namespace

// Workspace: block totals, chunk totals, keep masks [R][ceil(max_steps/64)]
// and entry distances [R], each slice 256-byte aligned.
struct MarchWs {
  int64_t *block_sum, *chunk_sum;
  uint64_t *masks;
  float *tn;
  size_t bytes;
};

static MarchWs march_ws(void *base, int64_t R, int32_t max_steps) {
  const int64_t Rp = R > 0 ? R : 1;
  const int64_t nblk = ceil_div(Rp, rays_per_block(Rp));
  const int64_t nw = ceil_div(max_steps > 0 ? max_steps : 1, kWave);
  char *p = (char *)base;
  MarchWs w;
  size_t o = 0;
  w.block_sum = (int64_t *)(p + o);
  o += align256(sizeof(int64_t) * (size_t)nblk);
  w.chunk_sum = (int64_t *)(p + o);
  o += align256(sizeof(int64_t) * (size_t)ceil_div(nblk, kScanChunk));
  w.masks = (uint64_t *)(p + o);
  o += align256(sizeof(uint64_t) * (size_t)(Rp * nw));
  w.tn = (float *)(p + o);
  o += align256(sizeof(float) * (size_t)Rp);
  w.bytes = o;
  return w;
}

extern "C" size_t ia355_march_workspace_size(int64_t R, int32_t max_steps) {
  if (R < 0 || max_steps < 0) return 0;
  return march_ws(nullptr, R, max_steps).bytes;
}

extern "C" int32_t ia355_occgrid_march(const float *rays_o, const float *rays_d, int64_t R, const uint32_t *occ_bits,
                                       int32_t G, const float *aabb, float dt, int32_t n_per_ray, int32_t max_steps,
                                       float *xs, float *ts, int32_t *ray_id, int64_t cap, int64_t *ray_off,
                                       int32_t *ray_cnt, float *ray_dt, int64_t *n_samples, int64_t *n_required,
                                       void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (R < 0 || !aabb || max_steps < 0 || cap < 0) return IA355_ERR_INVALID_ARG;
  if (!ray_off || !n_samples) return IA355_ERR_INVALID_ARG;
  if (R > 0 && (!rays_o || !rays_d || !ray_cnt || !ray_dt)) return IA355_ERR_INVALID_ARG;
  if (cap > 0 && (!xs || !ts || !ray_id)) return IA355_ERR_INVALID_ARG;
  if (occ_bits && (G <= 0 || G > 2048)) return IA355_ERR_INVALID_ARG;
  if (n_per_ray <= 0 && !(dt > 0.0f)) return IA355_ERR_INVALID_ARG;
  if ((int64_t)cap * 3 < cap) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < ia355_march_workspace_size(R, max_steps)) return IA355_ERR_WORKSPACE;
  Box box;
  bool pow2;
  if (!make_box(aabb, &box, &pow2)) return IA355_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  const int64_t nblk = ceil_div(R, rays_per_block(R));
  const int64_t nchunk = ceil_div(nblk, kScanChunk);
  const int nw = (int)ceil_div(max_steps, kWave);
  const MarchWs mw = march_ws(ws, R, max_steps);
  int64_t *block_sum = mw.block_sum, *chunk_sum = mw.chunk_sum;
  const bool many = rays_per_wave(R) == 4;
  if (R > 0) {
    if (pow2 && many)
      march_count<true, 4><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray,
                                                             max_steps, ray_off, ray_cnt, ray_dt, block_sum,
                                                             mw.masks, nw, mw.tn);
    else if (pow2)
      march_count<true, 1><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray,
                                                             max_steps, ray_off, ray_cnt, ray_dt, block_sum,
                                                             mw.masks, nw, mw.tn);
    else if (many)
      march_count<false, 4><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray,
                                                              max_steps, ray_off, ray_cnt, ray_dt, block_sum,
                                                              mw.masks, nw, mw.tn);
    else
      march_count<false, 1><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, occ_bits, G, box, dt, n_per_ray,
                                                              max_steps, ray_off, ray_cnt, ray_dt, block_sum,
                                                              mw.masks, nw, mw.tn);
    march_scan_chunk<<<(unsigned)nchunk, 1024, 0, s>>>(block_sum, nblk, chunk_sum, ray_off, R, n_samples);
  }
  if (nchunk != 1) march_scan_top<<<1, 1024, 0, s>>>(chunk_sum, nchunk, ray_off, R, n_samples);
  if (R > 0 && cap > 0) {
    if (many)
      march_fill<4><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, mw.masks, nw, mw.tn, block_sum, chunk_sum,
                                                      ray_off, ray_dt, xs, ts, ray_id, cap);
    else
      march_fill<1><<<(unsigned)nblk, kBlock, 0, s>>>(rays_o, rays_d, R, mw.masks, nw, mw.tn, block_sum, chunk_sum,
                                                      ray_off, ray_dt, xs, ts, ray_id, cap);
  }
  const int32_t st = launch_status();
  if (st != IA355_OK || !n_required) return st;
  // synchronous capacity check, on request only
  int64_t n = 0;
  if (hipMemcpyAsync(&n, n_samples, sizeof n, hipMemcpyDeviceToHost, s) != hipSuccess) return IA355_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return IA355_ERR_HIP;
  *n_required = n;
  return n > cap ? IA355_ERR_CAPACITY : IA355_OK;
}
