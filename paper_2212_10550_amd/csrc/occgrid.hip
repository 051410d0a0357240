// Per-pose occupancy grid for rendering (Sec. 3.3, inference stage): the
// centres of a G^3 lattice in posed space are mapped to canonical space by
// the multi-init root finding (Sec. 3.1), their densities are queried from
// the canonical field (hash encoding and MLP, Eq. 1-2; a point without a
// valid root has density 0), thresholded, and the occupied region is
// dilated so that the coarse lattice does not clip the subject.  The result
// is the packed occupancy bitfield the march reads.
//
// The lattice, deform, encode and MLP steps reuse the library's stages on
// one lattice point per sample; the threshold, the dilation and the packing
// are one kernel with a thread per output word.
//
// Training stage (Sec. 3.3): one shared grid, updated every few iterations
// from the densities of one random point per cell in the posed space of a
// training frame, as a moving average of the grid's values; and the
// occupancy-based density regulariser (Sec. 3.4), |sigma| of points that
// fall in empty cells.
#include "common.h"

using namespace ia355;

namespace {

constexpr int kBlock = 256;
constexpr int kMaxDilate = 4;

// One point per cell, point n = x + G (y + G z): lo + ((i + u) / G) ext per
// axis with u = 1/2 (cell centres) or u = jitter [3][G^3] in [0, 1), each
// operation rounded once (the oracle evaluates the same expression in IEEE
// single).
__global__ void __launch_bounds__(kBlock) lattice_kernel(int G, float lo0, float lo1, float lo2, float ext0,
                                                         float ext1, float ext2, int64_t N,
                                                         const float *__restrict__ jitter,
                                                         const int32_t *__restrict__ cells, float *__restrict__ xp) {
#pragma clang fp contract(off)
  const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n >= N) return;
  int64_t c = cells ? (int64_t)cells[n] : n;  // the cell of point n
  if (c < 0 || c >= (int64_t)G * G * G) c = 0;  // an invalid index: any in-grid point (its update is skipped)
  const int ix = (int)(c % G), iy = (int)((c / G) % G), iz = (int)(c / ((int64_t)G * G));
  const float g = (float)G;
  const float u0 = jitter ? jitter[n] : 0.5f, u1 = jitter ? jitter[N + n] : 0.5f, u2 = jitter ? jitter[2 * N + n] : 0.5f;
  xp[n] = lo0 + (((float)ix + u0) / g) * ext0;
  xp[N + n] = lo1 + (((float)iy + u1) / g) * ext1;
  xp[2 * N + n] = lo2 + (((float)iz + u2) / g) * ext2;
}

// v <- beta v + (1 - beta) sigma (the moving average of the training grid),
// point n updating its cell (cells[n], or n).
__global__ void __launch_bounds__(kBlock) ema_kernel(float *__restrict__ v, const float *__restrict__ sigma,
                                                     const int32_t *__restrict__ cells, float beta, int64_t N,
                                                     int64_t ncell) {
#pragma clang fp contract(off)
  const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n >= N) return;
  const int64_t c = cells ? (int64_t)cells[n] : n;
  if (c < 0 || c >= ncell) return;
  v[c] = beta * v[c] + (1.0f - beta) * sigma[n];
}

// Density regulariser in two kernels with a fixed summation order: a
// grid-stride pass (the grid depends only on the capacity S) writes dL/dsigma
// and one partial sum of |sigma| over empty-cell points per workgroup, then
// one workgroup adds the partials in order.  A point is in an empty cell when
// its cell's bit is 0 (cell as in the march's keep test, IEEE single without
// fused operations).
constexpr int kRegBlock = 256;
constexpr int kRegMaxBlocks = 1024;

__device__ __forceinline__ float block_sum256(float v, float *part) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  float t = 0.0f;
  for (int i = 0; i < kRegBlock / kWave; ++i) t += part[i];
  return t;
}

__global__ void __launch_bounds__(kRegBlock) density_reg_kernel(const float *__restrict__ x, const float *__restrict__ sigma,
                                                                int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                                const uint32_t *__restrict__ bits, int G, float lo0,
                                                                float lo1, float lo2, float ext0, float ext1, float ext2,
                                                                float lam, float *__restrict__ grad,
                                                                float *__restrict__ partial) {
#pragma clang fp contract(off)
  __shared__ float part[kRegBlock / kWave];
  const int64_t n_pts = count_of(S, S_dev);
  const float inv_n = n_pts > 0 ? 1.0f / (float)n_pts : 0.0f;
  const float lo[3] = {lo0, lo1, lo2}, ext[3] = {ext0, ext1, ext2};
  float acc = 0.0f;
  for (int64_t n = (int64_t)blockIdx.x * kRegBlock + threadIdx.x; n < n_pts; n += (int64_t)gridDim.x * kRegBlock) {
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float u = (x[a * ld + n] - lo[a]) / ext[a] * (float)G;
      const int i = (int)floorf(u);
      c[a] = i < 0 ? 0 : (i > G - 1 ? G - 1 : i);
    }
    const bool empty = !((bits[occ_word(c[0], c[1], c[2], G)] >> occ_bit(c[0], c[1])) & 1u);
    const float s = sigma[n];
    const float sgn = s > 0.0f ? 1.0f : (s < 0.0f ? -1.0f : 0.0f);
    grad[n] = empty ? lam * sgn * inv_n : 0.0f;
    if (empty) acc += fabsf(s);
  }
  const float t = block_sum256(acc, part);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kRegBlock) density_reg_sum_kernel(const float *__restrict__ partial, int nblk,
                                                                    int64_t S, const int64_t *__restrict__ S_dev,
                                                                    float lam, float *__restrict__ loss) {
  __shared__ float part[kRegBlock / kWave];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < nblk; i += kRegBlock) acc += partial[i];
  const float t = block_sum256(acc, part);
  if (threadIdx.x == 0) {
    const int64_t n_pts = count_of(S, S_dev);
    loss[0] = n_pts > 0 ? lam * t * (1.0f / (float)n_pts) : 0.0f;
  }
}

int reg_blocks(int64_t S) {
  int64_t b = ceil_div(S > 0 ? S : 1, kRegBlock);
  return (int)(b > kRegMaxBlocks ? kRegMaxBlocks : b);
}

// One thread per output word of the brick layout (32 cells: 8 along x, 4
// along y); a cell is occupied when any density within r cells (Chebyshev
// distance, clipped at the grid) exceeds the threshold.
__global__ void __launch_bounds__(kBlock) occ_from_density_kernel(const float *__restrict__ sigma, int G,
                                                                  float thresh, int r, uint32_t *__restrict__ bits,
                                                                  int64_t nword) {
  const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (w >= nword) return;
  const int64_t nb = (G + 7) / 8;
  const int64_t brick = w >> 5;
  const int q = (int)(w & 31);
  const int x0 = (int)(brick % nb) * 8, y0 = (int)((brick / nb) % nb) * 8 + (q & 1) * 4;
  const int z = (int)(brick / (nb * nb)) * 16 + (q >> 1);
  uint32_t v = 0;
  if (z < G) {
    const int z0 = z - r < 0 ? 0 : z - r, z1 = z + r > G - 1 ? G - 1 : z + r;
    for (int j = 0; j < 32; ++j) {
      const int x = x0 + (j & 7), y = y0 + (j >> 3);
      if (x >= G || y >= G) continue;
      const int xa = x - r < 0 ? 0 : x - r, xb = x + r > G - 1 ? G - 1 : x + r;
      const int ya = y - r < 0 ? 0 : y - r, yb = y + r > G - 1 ? G - 1 : y + r;
      bool occ = false;
      for (int zz = z0; zz <= z1 && !occ; ++zz)
        for (int yy = ya; yy <= yb && !occ; ++yy) {
          const float *row = sigma + ((int64_t)zz * G + yy) * G;
          for (int xx = xa; xx <= xb; ++xx) occ = occ || row[xx] > thresh;
        }
      if (occ) v |= 1u << j;
    }
  }
  bits[w] = v;
}

struct OccWs {
  float *xp, *xc, *sigma, *rgb;
  int16_t *bone;
  void *feat, *deform_ws;
  size_t deform_bytes, bytes;
};

OccWs occ_ws(void *base, int32_t G, int32_t L, int32_t F, int32_t mlp_dtype, int32_t Dx, int32_t Dy, int32_t Dz) {
  const size_t N = (size_t)G * G * G;
  const size_t fbytes = mlp_dtype == IA355_F32 ? 4 : 2;
  char *p = (char *)base;
  size_t o = 0;
  OccWs w;
  w.xp = (float *)(p + o);
  o += align256(12 * N);
  w.xc = (float *)(p + o);
  o += align256(12 * N);
  w.sigma = (float *)(p + o);
  o += align256(4 * N);
  w.rgb = (float *)(p + o);
  o += align256(12 * N);
  w.bone = (int16_t *)(p + o);
  o += align256(2 * N);
  w.feat = (void *)(p + o);
  o += align256(fbytes * (size_t)L * (size_t)F * N);
  w.deform_ws = (void *)(p + o);
  w.deform_bytes = ia355_deform_workspace_size(Dx, Dy, Dz);
  o += align256(w.deform_bytes);
  w.bytes = o;
  return w;
}

}  // namespace

extern "C" int32_t ia355_occ_from_density(const float *sigma, int32_t G, float sigma_thresh, int32_t dilate,
                                          uint32_t *occ_bits, ia355_stream_t stream) {
  if (G <= 0 || G > 2048 || dilate < 0 || dilate > kMaxDilate || !sigma || !occ_bits) return IA355_ERR_INVALID_ARG;
  const int64_t nword = occ_words(G);
  occ_from_density_kernel<<<(unsigned)ceil_div(nword, kBlock), kBlock, 0, as_stream(stream)>>>(
      sigma, G, sigma_thresh, dilate, occ_bits, nword);
  return launch_status();
}

extern "C" size_t ia355_occgrid_build_workspace_size(int32_t G, int32_t L, int32_t F, int32_t mlp_dtype, int32_t Dx,
                                                     int32_t Dy, int32_t Dz) {
  if (G <= 0 || G > 256 || L <= 0 || F <= 0) return 0;
  return occ_ws(nullptr, G, L, F, mlp_dtype, Dx, Dy, Dz).bytes;
}

// Densities of one point per cell (cell centres, or jittered): lattice,
// root finding, encoding, MLP.  Writes sig [G^3].
static int32_t lattice_density(int32_t G, const float *aabb, const float *jitter, const int32_t *cells, int64_t M,
                               const float *B, int32_t nb,
                               const float *W, int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                               const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid,
                               const void *table, int32_t table_dtype, int32_t L, int32_t F, int32_t log2T,
                               double base_res, double growth, const float *params, int32_t mlp_dtype, float *sigma,
                               void *ws, size_t ws_bytes, ia355_stream_t stream, float **sig_out) {
  if (G <= 0 || G > 256 || !aabb) return IA355_ERR_INVALID_ARG;
  if (mlp_dtype != IA355_F32 && mlp_dtype != IA355_BF16) return IA355_ERR_INVALID_ARG;
  float lo[3], ext[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = aabb[a];
    ext[a] = aabb[3 + a] - aabb[a];
    if (!(ext[a] > 0.0f)) return IA355_ERR_INVALID_ARG;
  }
  const size_t need = ia355_occgrid_build_workspace_size(G, L, F, mlp_dtype, Dx, Dy, Dz);
  if (!ws || need == 0 || ws_bytes < need) return IA355_ERR_WORKSPACE;
  const OccWs w = occ_ws(ws, G, L, F, mlp_dtype, Dx, Dy, Dz);
  const int64_t N = cells ? M : (int64_t)G * G * G;  // points: the listed cells, or every cell
  float *sig = sigma ? sigma : w.sigma;
  *sig_out = sig;
  const int32_t feat_dtype = mlp_dtype == IA355_F32 ? IA355_F32 : IA355_BF16;
  hipStream_t s = as_stream(stream);
  lattice_kernel<<<(unsigned)ceil_div(N, kBlock), kBlock, 0, s>>>(G, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], N,
                                                                   jitter, cells, w.xp);
  int32_t st = launch_status();
  if (st != IA355_OK) return st;
  st = ia355_snarf_deform(w.xp, N, nullptr, N, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, tol_stop,
                          tol_valid, w.xc, w.bone, nullptr, nullptr, w.deform_ws, w.deform_bytes, stream);
  if (st != IA355_OK) return st;
  st = ia355_hashgrid_encode(w.xc, w.bone, N, nullptr, N, table, table_dtype, L, F, log2T, base_res, growth,
                             hash_aabb, w.feat, feat_dtype, stream);
  if (st != IA355_OK) return st;
  static const int32_t kWidths[4] = {32, 64, 64, 4};
  return ia355_mlp_fwd(w.feat, feat_dtype, w.bone, N, nullptr, N, params, kWidths, 3, mlp_dtype, sig, w.rgb, stream);
}

extern "C" int32_t ia355_occgrid_build(int32_t G, const float *aabb, const float *B, int32_t nb, const float *W,
                                       int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                                       const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid,
                                       const void *table, int32_t table_dtype, int32_t L, int32_t F, int32_t log2T,
                                       double base_res, double growth, const float *params, int32_t mlp_dtype,
                                       float sigma_thresh, int32_t dilate, uint32_t *occ_bits, float *sigma,
                                       void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (!occ_bits || dilate < 0 || dilate > kMaxDilate) return IA355_ERR_INVALID_ARG;
  float *sig = nullptr;
  const int32_t st = lattice_density(G, aabb, nullptr, nullptr, 0, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter,
                                     tol_stop, tol_valid, table, table_dtype, L, F, log2T, base_res, growth, params,
                                     mlp_dtype, sigma, ws, ws_bytes, stream, &sig);
  if (st != IA355_OK) return st;
  return ia355_occ_from_density(sig, G, sigma_thresh, dilate, occ_bits, stream);
}

extern "C" int32_t ia355_occgrid_update(int32_t G, const float *aabb, const float *jitter, const int32_t *cells,
                                        int64_t M, const float *B, int32_t nb, const float *W, int32_t Dx,
                                        int32_t Dy, int32_t Dz,
                                        const float *skin_aabb, const float *hash_aabb, int32_t max_iter,
                                        float tol_stop, float tol_valid, const void *table, int32_t table_dtype,
                                        int32_t L, int32_t F, int32_t log2T, double base_res, double growth,
                                        const float *params, int32_t mlp_dtype, float beta, float sigma_thresh,
                                        int32_t dilate, float *values, uint32_t *occ_bits, void *ws,
                                        size_t ws_bytes, ia355_stream_t stream) {
  if (!jitter || !values || !occ_bits || dilate < 0 || dilate > kMaxDilate) return IA355_ERR_INVALID_ARG;
  if (!(beta >= 0.0f && beta <= 1.0f)) return IA355_ERR_INVALID_ARG;
  if (G <= 0 || G > 256 || (cells && (M < 1 || M > (int64_t)G * G * G))) return IA355_ERR_INVALID_ARG;
  float *sig = nullptr;
  int32_t st = lattice_density(G, aabb, jitter, cells, M, B, nb, W, Dx, Dy, Dz, skin_aabb, hash_aabb, max_iter, tol_stop,
                               tol_valid, table, table_dtype, L, F, log2T, base_res, growth, params, mlp_dtype,
                               nullptr, ws, ws_bytes, stream, &sig);
  if (st != IA355_OK) return st;
  const int64_t N = cells ? M : (int64_t)G * G * G;
  ema_kernel<<<(unsigned)ceil_div(N, kBlock), kBlock, 0, as_stream(stream)>>>(values, sig, cells, beta, N,
                                                                               (int64_t)G * G * G);
  st = launch_status();
  if (st != IA355_OK) return st;
  return ia355_occ_from_density(values, G, sigma_thresh, dilate, occ_bits, stream);
}

extern "C" size_t ia355_density_reg_workspace_size(int64_t S) {
  return S < 0 ? 0 : align256(sizeof(float) * (size_t)reg_blocks(S));
}

extern "C" int32_t ia355_density_reg(const float *x, const float *sigma, int64_t S, const int64_t *S_dev, int64_t ld,
                                     const uint32_t *occ_bits, int32_t G, const float *aabb, float lam,
                                     float *loss, float *grad_sigma, void *ws, size_t ws_bytes,
                                     ia355_stream_t stream) {
  if (S < 0 || ld < S || !occ_bits || !aabb || !loss || G <= 0 || G > 2048) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!x || !sigma || !grad_sigma)) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < ia355_density_reg_workspace_size(S)) return IA355_ERR_WORKSPACE;
  float lo[3], ext[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = aabb[a];
    ext[a] = aabb[3 + a] - aabb[a];
    if (!(ext[a] > 0.0f)) return IA355_ERR_INVALID_ARG;
  }
  hipStream_t s = as_stream(stream);
  const int nblk = reg_blocks(S);
  float *partial = (float *)ws;
  density_reg_kernel<<<nblk, kRegBlock, 0, s>>>(x, sigma, S, S_dev, ld, occ_bits, G, lo[0], lo[1], lo[2], ext[0],
                                                ext[1], ext[2], lam, grad_sigma, partial);
  density_reg_sum_kernel<<<1, kRegBlock, 0, s>>>(partial, nblk, S, S_dev, lam, loss);
  return launch_status();
}
