// Batched inference render of many poses of one avatar in one persistent
// launch: for every ray of every pose, the sampling with empty-space
// skipping of Sec. 3.2-3.3, the canonical correspondence of Sec. 3.1 (learned
// initialiser, one guided Broyden solve, the multi-init solve as fallback),
// the hash-grid encoding and decoder MLP of Eq. 1-2 in their FP16/BF16 form,
// and the volume rendering of Eq. 8 with early termination.
//
// Two kernels per call:
//  * prep: blends each pose's transform grid A (Eq. 5-7 pre-blended, as the
//    deform kernels do), folds the pose into the initialiser's first layer,
//    inverts the bone transforms, and clears the work queue and counters;
//  * render: persistent.  256 x blocks_per_cu workgroups of four waves;
//    every wave takes tiles of consecutive rays of one pose from a global
//    atomic counter and carries each through the whole path on its own:
//      march   -- each ray's keep masks (one ballot per 64 steps, the march
//                 kernels' test) and sample counts into the wave's LDS;
//      segment -- the tile's rays are cut into segments of whole rays with
//                 at most samples_per_segment samples; per segment, chunks
//                 of 64 samples (one per lane) run position -> initialiser
//                 (four 16-sample MFMA tiles) -> guided Broyden; accepted
//                 samples go on to encode + decoder (lane r + 16 g of tile
//                 t encodes levels 4g..4g+3 of sample 16t + r, which is
//                 exactly the decoder's BF16 A-operand layout, so features
//                 never leave registers); rejected samples wait in an LDS
//                 queue and take the 24-init solve two at a time (32 lanes
//                 each), then encode + decoder;
//      composite -- 16 lanes per ray over the segment's densities and
//                 colours in LDS; pixels are written to the pose's outputs.
//    No sample ever goes to global memory.  The decoder's and initialiser's
//    MFMA fragments are built once per workgroup into LDS and reloaded per
//    chunk, which keeps them out of the registers the solver needs.
// Every per-sample and per-ray operation is the same device code as in the
// staged kernels (march_dev.h, rootinit_dev.h, deform_dev.h, hash_dev.h,
// mlp_dev.h, render_dev.h), so a pose rendered here gives the same bits as
// the staged path.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <mutex>

#include "common.h"
#include "deform_dev.h"
#include "geometry.h"
#include "hash_dev.h"
#include "march_dev.h"
#include "mlp_dev.h"
#include "render_dev.h"
#include "rootinit_dev.h"

using namespace ia355;

namespace {

constexpr int kMaxPoses = IA355_BATCH_MAX_POSES;
constexpr int kMaxTileRays = 64;   // one lane per ray in the span pass
constexpr int kMaxSteps = 128;     // two 64-bit keep masks per ray
constexpr int kPrepBlock = dfm::kBlendBlock;
constexpr int kLevels = 16;        // decoder input 32 = 16 levels x 2 features
constexpr uint32_t kMagic = 0x1a355b01u;

struct PoseDev {
  const float *ro, *rd;
  int64_t R;
  const uint32_t *bits;
  int G, pow2, n_per_ray, max_steps;
  mch::Box box;
  float dt_fixed;
  const float *B, *pose;
  float *color, *opacity, *T_final;
  int32_t *n_used, *n_fallback, *n_evaluated;
  float *A, *c1, *binv;  // workspace: blended grid, folded layer-1 constant, bone inverses
  int *bok;
};

struct Plan {
  uint32_t magic;
  int n_poses, nb;
  size_t ws_need;
  const float *W;
  int64_t nvert, nblend;
  dfm::Grid gr;
  dfm::Box hbox;
  int max_iter;
  float tol_stop, tol_valid;
  const __half *table;
  uint32_t T, Tmask;
  hsh::Box ebox;
  hsh::Levels lv;
  const float *mlp, *init;
  float T_thresh;
  PoseDev pose[kMaxPoses];
};

// Workgroup-shared LDS: MFMA fragments of the decoder (14 per lane) and the
// initialiser's layers 2-3 (12 per lane), lane-contiguous; biases; the
// initialiser's layer-1 position weights; level constants; tile prefix.
struct Store {
  bf16x8 mw[14][kWave];
  bf16x8 rw[12][kWave];
  float mb1[64], mb2[64], mb3[4];
  float rb2[64], rb3[rid::kMaxOut];
  float w1x[rid::H * 3];
  int res[kLevels], dense[kLevels];
  int64_t tile0[kMaxPoses + 1];
};
static_assert(offsetof(Store, mb1) % 16 == 0 && offsetof(Store, mb2) % 16 == 0 && offsetof(Store, mb3) % 16 == 0 &&
                  offsetof(Store, rb2) % 16 == 0 && offsetof(Store, rb3) % 16 == 0 && sizeof(Store) % 16 == 0,
              "16-byte bias vectors and wave regions");

// Per-wave LDS, carved from one block (sizes from the tile shape).
struct WaveMem {
  uint64_t *mask;  // [rt][2]
  float *o, *d;    // [rt][3]
  float *tn, *tf, *dt;
  float *T;        // [rt] transmittance before the segment's next group, per ray
  float *c1;       // [64] the tile's pose's folded initialiser constant
  int *off;        // [rt + 1] first sample of each ray in the tile
  int *alive;      // [rt] the ray has groups left and has not terminated
  int *roff;       // [rt + 1] first sample of each ray in the current round
  float *sig;      // [ch]
  float *rgb;      // [ch][3]
  int16_t *queue;  // [ch]
};

__host__ __device__ inline size_t wave_bytes(int rt, int ch) {
  size_t b = 16 * (size_t)rt;                      // masks
  b += sizeof(float) * (10 * (size_t)rt + 64);     // o, d, tn, tf, dt, T, c1
  b += sizeof(int) * (3 * (size_t)rt + 2);         // off, alive, roff
  b += sizeof(float) * 4 * (size_t)ch;             // sig, rgb
  b += sizeof(int16_t) * (size_t)ch;               // queue
  return (b + 15) & ~(size_t)15;
}

__device__ inline WaveMem carve(char *p, int rt, int ch) {
  WaveMem w;
  w.mask = reinterpret_cast<uint64_t *>(p);
  p += 16 * (size_t)rt;
  w.o = reinterpret_cast<float *>(p);
  w.d = w.o + 3 * rt;
  w.tn = w.d + 3 * rt;
  w.tf = w.tn + rt;
  w.dt = w.tf + rt;
  w.T = w.dt + rt;
  w.c1 = w.T + rt;
  w.off = reinterpret_cast<int *>(w.c1 + 64);
  w.alive = w.off + rt + 1;
  w.roff = w.alive + rt;
  w.sig = reinterpret_cast<float *>(w.roff + rt + 1);
  w.rgb = w.sig + ch;
  w.queue = reinterpret_cast<int16_t *>(w.rgb + 3 * ch);
  return w;
}

// Position of the q-th (from 0) set bit of the 128-bit mask (m0, m1).
__host__ __device__ inline int select_bit(uint64_t m0, uint64_t m1, int q) {
  const int c0 = __builtin_popcountll(m0);
  uint64_t m = q < c0 ? m0 : m1;
  int pos = q < c0 ? 0 : 64;
  if (q >= c0) q -= c0;
  for (int w = 32; w >= 1; w >>= 1) {
    const int c = __builtin_popcountll(m & ((1ull << w) - 1ull));
    if (q >= c) {
      q -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// Ray (in [ra, rb)) holding tile sample j: the last ray whose first sample
// is at or before j.
__device__ inline int ray_of(const int *off, int ra, int rb, int j) {
  int lo = ra, hi = rb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Posed position of the q-th kept sample of tile ray rr (the march's
// expression for its step).
__device__ inline void ray_sample_xp(const WaveMem &wm, int rr, int q, float xp[3]) {
  const int k = select_bit(wm.mask[2 * rr], wm.mask[2 * rr + 1], q);
  float t;
  mch::sample_pos(wm.o + 3 * rr, wm.d + 3 * rr, wm.tn[rr], wm.dt[rr], k, &t, xp);
}

// Posed position of tile sample j (rays [ra, rb) hold it).
__device__ inline void sample_xp(const WaveMem &wm, int ra, int rb, int j, float xp[3]) {
  const int rr = ray_of(wm.off, ra, rb, j);
  ray_sample_xp(wm, rr, j - wm.off[rr], xp);
}

// Decoder weights fetched from the workgroup's LDS as the MFMAs use them
// (the same bf16 fragments and FP32 biases as the decoder kernel's FragBf).
struct LdsMW {
  const Store &st;
  int lane, g;
  __device__ __forceinline__ bf16x8 w1(int mt) const { return st.mw[mt][lane]; }
  __device__ __forceinline__ bf16x8 w2(int mt, int c) const { return st.mw[4 + 2 * mt + c][lane]; }
  __device__ __forceinline__ bf16x8 w3(int c) const { return st.mw[12 + c][lane]; }
  __device__ __forceinline__ f32x4 b1(int mt) const {
    return *reinterpret_cast<const f32x4 *>(st.mb1 + 16 * mt + 4 * g);
  }
  __device__ __forceinline__ f32x4 b2(int mt) const {
    return *reinterpret_cast<const f32x4 *>(st.mb2 + 16 * mt + 4 * g);
  }
  __device__ __forceinline__ f32x4 b3() const {
    return g == 0 ? *reinterpret_cast<const f32x4 *>(st.mb3) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
};

// A compiler-only barrier: keeps the fragment fetches of one tile from being
// hoisted out of the tile loop (which would hold every fragment in registers).
__device__ __forceinline__ void keep_in_loop() { asm volatile("" ::: "memory"); }

__device__ inline __bf16 to_bf16(float v) {
  return __builtin_bit_cast(__bf16, __builtin_bit_cast(uint16_t, __float2bfloat16(v)));
}

// Encode + decoder of one 16-sample tile: lane r + 16 g encodes levels
// 4g..4g+3 of its row's sample (x, bone; bone < 0 gives zero features and
// zero outputs, as the staged encode and decoder do); rows with store set
// write sigma and colour at slot.
__device__ inline void encode_decode(const Plan &pl, const Store &st, int lane, const float x[3], int bone,
                                     bool store, int slot, int g, float *sig, float *rgb, int ch) {
  bf16x8 X;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int l = 4 * g + jj;
    float a = 0.0f, b = 0.0f;
    if (bone >= 0)
      hsh::encode_level(x, pl.ebox, st.res[l], st.dense[l] != 0, pl.Tmask, pl.table + (int64_t)l * pl.T * 2, &a, &b);
    X[2 * jj] = to_bf16(a);
    X[2 * jj + 1] = to_bf16(b);
  }
  f32x4 z1[4], z2[4], o;
  mlpd::fwd_bf_src(LdsMW{st, lane, g}, X, z1, z2, o);
  if (g == 0 && store) {
    float sg = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
    if (bone >= 0) {
      const float ov[4] = {o[0], o[1], o[2], o[3]};
      mlpd::head(ov, &sg, c);
    }
    sig[slot] = sg;
    rgb[slot] = c[0];
    rgb[ch + slot] = c[1];
    rgb[2 * ch + slot] = c[2];
  }
}

struct LdsSrc {
  const float *sig, *rgb;
  int ch;
  __device__ __forceinline__ void operator()(int64_t i, float *s, float c[3]) const {
    *s = sig[i];
    c[0] = rgb[i];
    c[1] = rgb[ch + i];
    c[2] = rgb[2 * ch + i];
  }
};

// Keep masks of the tile's rays (lanes = steps k and k + 64), kMarchRays
// rays at a time so that their occupancy loads are in flight together; the
// test is the march kernels' (sample_at, then t < t_far).
constexpr int kMarchRays = 4;
template <bool kPow2>
__device__ inline void march_masks(const PoseDev &pd, const WaveMem &wm, int nr, int lane) {
  for (int rr0 = 0; rr0 < nr; rr0 += kMarchRays) {
    bool keep[kMarchRays][2];
#pragma unroll
    for (int u = 0; u < kMarchRays; ++u) {
      const int rr = min(rr0 + u, nr - 1);
      const float tf = wm.tf[rr];
      const float o[3] = {wm.o[3 * rr], wm.o[3 * rr + 1], wm.o[3 * rr + 2]};
      const float d[3] = {wm.d[3 * rr], wm.d[3 * rr + 1], wm.d[3 * rr + 2]};
      const mch::RaySpan s{wm.tn[rr], tf, wm.dt[rr], true};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = lane + h * kWave;
        float t, x[3];
        // a step past t_far is not kept, so its cell is not looked up (a ray
        // that misses the box has t_far = -inf: nothing is kept)
        keep[u][h] = k < pd.max_steps && mch::step_t(s, k) < tf &&
                     mch::sample_at<kPow2>(o, d, s, k, pd.box, pd.bits, pd.G, &t, x) && t < tf;
      }
    }
#pragma unroll
    for (int u = 0; u < kMarchRays; ++u) {
      const uint64_t m0 = __ballot(keep[u][0]), m1 = __ballot(keep[u][1]);
      if (lane == 0 && rr0 + u < nr) {
        wm.mask[2 * (rr0 + u)] = m0;
        wm.mask[2 * (rr0 + u) + 1] = m1;
      }
    }
  }
}

__global__ void __launch_bounds__(kPrepBlock) prep_kernel(const Plan *__restrict__ plp, size_t ws_bytes,
                                                          int *__restrict__ queue) {
  const Plan &pl = *plp;
  if (pl.magic != kMagic || pl.ws_need > ws_bytes) return;
  __shared__ float sB[dfm::kMaxBones * 12];
  __shared__ __attribute__((aligned(16))) float sW[dfm::kBlendBlock * dfm::kBlendMaxBones];
  if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
  const int64_t per = pl.nblend + 1;
  const int64_t items = per * pl.n_poses;
  const rid::Layout l = rid::layout(pl.nb);
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int p = (int)(it / per);
    const int64_t sub = it - (int64_t)p * per;
    const PoseDev &pd = pl.pose[p];
    if (sub < pl.nblend) {
      dfm::blend_block(pl.W, pd.B, pl.nb, pl.nvert, pd.A, sub, sB, sW);
    } else {
      rid::fold_pose(pl.init, l, pd.pose, pl.nb, pd.c1);
      stage_bone_inverses(pd.B, pl.nb, pd.binv, pd.bok);
      if (threadIdx.x == 0 && pd.n_fallback) *pd.n_fallback = 0;
      if (threadIdx.x == 0 && pd.n_evaluated) *pd.n_evaluated = 0;
    }
    __syncthreads();
  }
}

// kW waves per workgroup, at least kMinGroups workgroups per CU: the second
// launch bound is the waves per SIMD, kMinGroups kW / 4, which caps the
// registers per lane at 512 / (kMinGroups kW / 4).
template <int kW, int kMinGroups>
__global__ void __launch_bounds__(kW * kWave, kMinGroups * kW / 4) render_kernel(const Plan *__restrict__ plp,
                                                                        size_t ws_bytes, int *__restrict__ queue,
                                                                        int rt, int ch) {
  constexpr int kBlock = kW * kWave;
  const Plan &pl = *plp;
  if (pl.magic != kMagic || pl.ws_need > ws_bytes) return;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Store &st = *reinterpret_cast<Store *>(lds);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, r = lane & 15,
            g = lane >> 4;
  const int nb = pl.nb;
  // ---- workgroup set-up: fragments and constants (the same values as the
  // staged kernels build from their LDS copies of the parameters)
  const rid::Layout rl = rid::layout(nb);
  // one fragment per thread at a time (whole fragment sets in registers
  // would set the kernel's register count)
  for (int e = threadIdx.x; e < 14 * kWave; e += kBlock) {
    const int q = e / kWave, ln = e % kWave;
    st.mw[q][ln] = mlpd::frag_bf(pl.mlp, q, ln & 15, ln >> 4);
  }
  for (int e = threadIdx.x; e < 12 * kWave; e += kBlock) {
    const int q = e / kWave, ln = e % kWave;
    st.rw[q][ln] = rid::frag_bf(pl.init, rl, q, ln & 15, ln >> 4);
  }
  for (int i = threadIdx.x; i < 64; i += kBlock) {
    st.mb1[i] = pl.mlp[mlpd::OFF_B1 + i];
    st.mb2[i] = pl.mlp[mlpd::OFF_B2 + i];
    st.rb2[i] = pl.init[rl.offb2 + i];
  }
  for (int i = threadIdx.x; i < rid::kMaxOut; i += kBlock) st.rb3[i] = i < rl.nout ? pl.init[rl.offb3 + i] : 0.0f;
  for (int i = threadIdx.x; i < 4; i += kBlock) st.mb3[i] = pl.mlp[mlpd::OFF_B3 + i];
  for (int e = threadIdx.x; e < rid::H * 3; e += kBlock) st.w1x[e] = pl.init[rl.offW1 + (e / 3) * rl.nin + (e % 3)];
  for (int i = threadIdx.x; i < kLevels; i += kBlock) {
    st.res[i] = pl.lv.res[i];
    st.dense[i] = pl.lv.dense[i];
  }
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int p = 0; p < pl.n_poses; ++p) {
      st.tile0[p] = t;
      t += (pl.pose[p].R + rt - 1) / rt;
    }
    st.tile0[pl.n_poses] = t;
  }
  __syncthreads();
  const int64_t n_tiles = st.tile0[pl.n_poses];
  const WaveMem wm = carve(lds + sizeof(Store) + (size_t)wid * wave_bytes(rt, ch), rt, ch);
  const uint64_t below = (1ull << lane) - 1ull;
  const int C = ch - kMaxSteps;  // segment start stride: a segment holds at most C + 128 = ch samples

  // ---- tiles, one wave each, until the queue is drained (no wave ever
  // waits for another: the loop ends for every wave)
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(queue, 1);
    item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, kWave));
    if ((int64_t)item >= n_tiles) break;
    int p = 0;
    while (p + 1 < pl.n_poses && st.tile0[p + 1] <= item) ++p;
    p = __builtin_amdgcn_readfirstlane(p);
    const PoseDev &pd = pl.pose[p];
    const int64_t ray0 = (int64_t)(item - st.tile0[p]) * rt;
    const int nr = (int)min((int64_t)rt, pd.R - ray0);
    wm.c1[lane] = pd.c1[lane];

    // march: spans (one lane per ray), then keep masks (lanes = steps)
    if (lane < nr) {
      float o[3], d[3];
      mch::load_ray(pd.ro, pd.rd, ray0 + lane, o, d);
      const mch::RaySpan s = mch::ray_span(o, d, pd.box, pd.dt_fixed, pd.n_per_ray);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wm.o[3 * lane + a] = o[a];
        wm.d[3 * lane + a] = d[a];
      }
      wm.tn[lane] = s.tn;
      wm.tf[lane] = s.hit ? s.tf : -INFINITY;
      wm.dt[lane] = s.dt;
    }
    mlpd::wave_sync();
    if (pd.pow2)
      march_masks<true>(pd, wm, nr, lane);
    else
      march_masks<false>(pd, wm, nr, lane);
    mlpd::wave_sync();
    {
      const int cnt = lane < nr ? __popcll(wm.mask[2 * lane]) + __popcll(wm.mask[2 * lane + 1]) : 0;
      const int incl = wave_incl_scan(cnt);
      if (lane < nr) wm.off[lane + 1] = incl;
      if (lane == 0) wm.off[0] = 0;
    }
    mlpd::wave_sync();
    const int total = __builtin_amdgcn_readfirstlane(wm.off[nr]);
    const int nseg = total == 0 ? 1 : (total + C - 1) / C;
    const float *A = pd.A;
    int nfb = 0, nev = 0;
    int ra = 0;
    for (int sgi = 0; sgi < nseg; ++sgi) {
      int rb = nr;
      if (sgi + 1 < nseg) {
        const int v = (sgi + 1) * C;
        const uint64_t bm = __ballot(lane < nr && wm.off[lane] >= v);
        rb = bm ? (int)__builtin_ctzll(bm) : nr;
      }
      const int sb = __builtin_amdgcn_readfirstlane(wm.off[ra]), se = __builtin_amdgcn_readfirstlane(wm.off[rb]);
      const int nrs = rb - ra;  // rays of the segment
      // Rounds: round k evaluates group k (kept samples 16k .. 16k + 15,
      // the compositor's groups) of every ray still alive, then steps each
      // such ray's transmittance through that group with the compositor's
      // own group step; a ray whose group has an unused sample (T_i below
      // the threshold) is finished, and its later samples are never
      // evaluated.  The final composite reads only evaluated groups.
      if (lane < nrs) {
        wm.T[lane] = 1.0f;
        wm.alive[lane] = wm.off[ra + lane + 1] > wm.off[ra + lane];
      }
      mlpd::wave_sync();
      const LdsSrc src{wm.sig, wm.rgb, ch};
      for (int k = 0;; ++k) {
        {
          int m = 0;
          if (lane < nrs && wm.alive[lane]) m = min(rnd::kSeg, wm.off[ra + lane + 1] - wm.off[ra + lane] - rnd::kSeg * k);
          const int incl = wave_incl_scan(m);
          if (lane < nrs) wm.roff[lane + 1] = incl;
          if (lane == 0) wm.roff[0] = 0;
        }
        mlpd::wave_sync();
        const int nk = __builtin_amdgcn_readfirstlane(wm.roff[nrs]);  // samples of this round
        if (nk == 0) break;
        nev += nk;
        int qn = 0;
        for (int c0 = 0; c0 < nk; c0 += kWave) {
          const int jr = c0 + lane;
          const bool act = jr < nk;
          const int nt = (min(kWave, nk - c0) + 15) >> 4;  // 16-sample tiles in this chunk
          int slot = 0;  // the sample's index in the segment
          float xp[3] = {0.0f, 0.0f, 0.0f};
          if (act) {
            const int rl = ray_of(wm.roff, 0, nrs, jr);
            const int q = rnd::kSeg * k + (jr - wm.roff[rl]);
            slot = wm.off[ra + rl] - sb + q;
            ray_sample_xp(wm, ra + rl, q, xp);
          }
          // learned initialiser: lane r + 16 t's sample is row r of tile t,
          // and that lane holds the tile's result for it
          int ibone = 0;
          float x0[3] = {0.0f, 0.0f, 0.0f};
          for (int t = 0; t < nt; ++t) {
            keep_in_loop();
            const int sr = 16 * t + r;
            const float xs[3] = {__shfl(xp[0], sr, kWave), __shfl(xp[1], sr, kWave), __shfl(xp[2], sr, kWave)};
            int bi;
            float off3[3], h1[4][4];
            rid::layer1(xs, wm.c1, st.w1x, g, h1);
            rid::tile_tail<true>(h1, rid::LdsFragW{st.rw, st.rb2, st.rb3, lane, g}, nb, g, &bi, off3);
            if (g == t) {
              const int kb = bi < nb ? bi : 0;
              ibone = kb;
              rid::start_point(pd.binv + 12 * kb, xs, off3, x0);
            }
          }
          // guided solve
          bool fb = false;
          int bone = -1;
          float xc[3] = {0.0f, 0.0f, 0.0f};
          if (act) {
            const dfm::InitResult q = dfm::broyden_from(A, pl.gr, x0, true, xp, pl.max_iter, pl.tol_stop);
            if (q.ok && q.r < pl.tol_valid && dfm::in_hbox(q.x, pl.hbox)) {
              xc[0] = q.x[0];
              xc[1] = q.x[1];
              xc[2] = q.x[2];
              bone = ibone;
            } else {
              fb = true;
            }
          }
          const uint64_t fm = __ballot(fb);
          if (fb) wm.queue[qn + __popcll(fm & below)] = (int16_t)slot;
          qn += __popcll(fm);
          // encode + decoder of the accepted samples
          for (int t = 0; t < nt; ++t) {
            keep_in_loop();
            const int sr = 16 * t + r;
            const float xs[3] = {__shfl(xc[0], sr, kWave), __shfl(xc[1], sr, kWave), __shfl(xc[2], sr, kWave)};
            const int bs = __shfl(bone, sr, kWave);
            const int ss = __shfl(slot, sr, kWave);
            encode_decode(pl, st, lane, xs, bs, bs >= 0, ss, g, wm.sig, wm.rgb, ch);
          }
        }
        mlpd::wave_sync();
        // fallback: the multi-init solve of the round's queued samples, two
        // at a time (32 lanes each), then their encode + decoder as rows 0
        // and 1 of a tile
        for (int q0 = 0; q0 < qn; q0 += 2) {
          const int h = lane >> 5;
          const bool qa = q0 + h < qn;
          const int sj = qa ? (int)wm.queue[q0 + h] : 0;
          float xp[3] = {0.0f, 0.0f, 0.0f};
          if (qa) sample_xp(wm, ra, rb, sb + sj, xp);
          const dfm::Choice cc = dfm::multi_init<32>(A, pl.gr, pd.binv, pd.bok, nb, xp, qa, lane & 31, pl.hbox,
                                                     pl.max_iter, pl.tol_stop, pl.tol_valid);
          const int sr = r < 2 ? 32 * r : 0;
          const float xs[3] = {__shfl(cc.x[0], sr, kWave), __shfl(cc.x[1], sr, kWave), __shfl(cc.x[2], sr, kWave)};
          const bool qs = __shfl((int)qa, sr, kWave) != 0 && r < 2;
          const int bs = qs ? __shfl(cc.bone, sr, kWave) : -1;
          const int ss = __shfl(sj, sr, kWave);
          keep_in_loop();
          encode_decode(pl, st, lane, xs, bs, qs, ss, g, wm.sig, wm.rgb, ch);
        }
        nfb += qn;
        mlpd::wave_sync();
        // transmittance through group k of every ray of this round
        for (int r0 = 0; r0 < nrs; r0 += 4) {
          const int rl = r0 + (lane >> 4), jj = lane & 15;
          if (rl < nrs && wm.roff[rl + 1] > wm.roff[rl]) {
            const int rr = ra + rl;
            rnd::RayState rs = rnd::ray_start();
            rs.T = wm.T[rl];
            const int b0 = wm.off[rr] - sb, e0 = wm.off[rr + 1] - sb;
            rnd::composite_group(src, b0 + rnd::kSeg * k, e0, wm.dt[rr], pl.T_thresh, jj, rs);
            if (jj == 0) {
              wm.T[rl] = rs.T;
              wm.alive[rl] = !rs.done && e0 - b0 > rnd::kSeg * (k + 1);
            }
          }
        }
        mlpd::wave_sync();
      }
      // composite: 16 lanes per ray, four rays at a time
      for (int r0 = ra; r0 < rb; r0 += 4) {
        const int rr = r0 + (lane >> 4), jj = lane & 15;
        if (rr < rb) {
          const rnd::RayOut q =
              rnd::composite_ray(src, wm.off[rr] - sb, wm.off[rr + 1] - sb, wm.dt[rr], pl.T_thresh, jj);
          if (jj == 0) {
            const int64_t gr = ray0 + rr;
            pd.color[3 * gr] = q.C[0];
            pd.color[3 * gr + 1] = q.C[1];
            pd.color[3 * gr + 2] = q.C[2];
            pd.opacity[gr] = q.A;
            pd.n_used[gr] = q.used;
            pd.T_final[gr] = q.T;
          }
        }
      }
      mlpd::wave_sync();
      ra = rb;
    }
    if (lane == 0 && nfb > 0 && pd.n_fallback) atomicAdd(pd.n_fallback, nfb);
    if (lane == 0 && nev > 0 && pd.n_evaluated) atomicAdd(pd.n_evaluated, nev);
  }
}

struct WsLayout {
  size_t plan, queue, pose0, A, c1, binv, bok, per_pose, total;
};

WsLayout ws_layout(int n_poses, int64_t nvert, int nb) {
  WsLayout w;
  w.plan = 0;
  w.queue = align256(sizeof(Plan));
  w.pose0 = w.queue + 256;
  w.A = 0;
  w.c1 = align256(sizeof(float) * 12 * (size_t)nvert);
  w.binv = w.c1 + 256;
  w.bok = w.binv + align256(sizeof(float) * 12 * (size_t)nb);
  w.per_pose = w.bok + align256(sizeof(int) * (size_t)nb);
  w.total = w.pose0 + (size_t)n_poses * w.per_pose;
  return w;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" size_t ia355_batch_workspace_size(int32_t n_poses, int32_t Dx, int32_t Dy, int32_t Dz, int32_t nb) {
  if (n_poses < 1 || n_poses > kMaxPoses || Dx < 2 || Dy < 2 || Dz < 2 || nb < 1 || nb > dfm::kMaxBones ||
      nb + 3 > rid::kMaxOut)
    return 0;
  return ws_layout(n_poses, (int64_t)Dx * Dy * Dz, nb).total;
}

extern "C" int32_t ia355_batch_plan(const ia355_batch_pose *poses, int32_t n_poses, const ia355_batch_model *m,
                                    void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (!poses || !m || n_poses < 1 || n_poses > kMaxPoses) return IA355_ERR_INVALID_ARG;
  const int nb = m->nb;
  if (nb < 1 || nb > dfm::kMaxBones || nb + 3 > rid::kMaxOut) return IA355_ERR_INVALID_ARG;
  if (!m->W || !dfm::grid_ok(m->Dx, m->Dy, m->Dz, m->skin_aabb)) return IA355_ERR_INVALID_ARG;
  if (m->max_iter < 0 || m->max_iter > 1000) return IA355_ERR_INVALID_ARG;
  if (!m->table || !aligned16(m->table) || !m->mlp_params || !aligned16(m->mlp_params) || !m->init_params)
    return IA355_ERR_INVALID_ARG;
  if (m->L != kLevels || m->log2T < 2 || m->log2T > 30) return IA355_ERR_UNSUPPORTED;
  if (m->init_hidden != rid::H) return IA355_ERR_UNSUPPORTED;
  Plan pl{};
  pl.magic = kMagic;
  pl.n_poses = n_poses;
  pl.nb = nb;
  pl.W = m->W;
  pl.nvert = (int64_t)m->Dx * m->Dy * m->Dz;
  pl.nblend = ceil_div(pl.nvert, dfm::kBlendBlock);
  pl.gr = dfm::make_grid(m->Dx, m->Dy, m->Dz, m->skin_aabb);
  for (int a = 0; a < 3; ++a) {
    pl.hbox.lo[a] = m->hash_aabb[a];
    pl.hbox.hi[a] = m->hash_aabb[3 + a];
  }
  pl.max_iter = m->max_iter;
  pl.tol_stop = m->tol_stop;
  pl.tol_valid = m->tol_valid;
  pl.table = (const __half *)m->table;
  pl.T = 1u << m->log2T;
  pl.Tmask = pl.T - 1u;
  if (hsh::make_levels(m->L, m->log2T, m->base_res, m->growth, &pl.lv) || hsh::make_box(m->hash_aabb, &pl.ebox))
    return IA355_ERR_INVALID_ARG;
  pl.mlp = m->mlp_params;
  pl.init = m->init_params;
  pl.T_thresh = m->T_thresh;
  const WsLayout wl = ws_layout(n_poses, pl.nvert, nb);
  pl.ws_need = wl.total;
  if (!ws || ws_bytes < wl.total) return IA355_ERR_WORKSPACE;
  char *base = (char *)ws;
  for (int p = 0; p < n_poses; ++p) {
    const ia355_batch_pose &q = poses[p];
    PoseDev &d = pl.pose[p];
    if (q.R < 0 || q.R > 0x7fffffffLL - 64) return IA355_ERR_INVALID_ARG;
    if (q.R > 0 && (!q.rays_o || !q.rays_d || !q.color || !q.opacity || !q.n_used || !q.T_final))
      return IA355_ERR_INVALID_ARG;
    if (!q.B || !q.pose) return IA355_ERR_INVALID_ARG;
    if (q.occ_bits && (q.G <= 0 || q.G > 2048)) return IA355_ERR_INVALID_ARG;
    if (q.max_steps < 0 || q.max_steps > kMaxSteps) return IA355_ERR_UNSUPPORTED;
    if (q.n_per_ray <= 0 && !(q.dt > 0.0f)) return IA355_ERR_INVALID_ARG;
    bool pow2 = false;
    if (!mch::make_box(q.occ_aabb, &d.box, &pow2)) return IA355_ERR_INVALID_ARG;
    d.pow2 = pow2;
    d.ro = q.rays_o;
    d.rd = q.rays_d;
    d.R = q.R;
    d.bits = q.occ_bits;
    d.G = q.G;
    d.n_per_ray = q.n_per_ray;
    d.max_steps = q.max_steps;
    d.dt_fixed = q.dt;
    d.B = q.B;
    d.pose = q.pose;
    d.color = q.color;
    d.opacity = q.opacity;
    d.T_final = q.T_final;
    d.n_used = q.n_used;
    d.n_fallback = q.n_fallback;
    d.n_evaluated = q.n_evaluated;
    char *pp = base + wl.pose0 + (size_t)p * wl.per_pose;
    d.A = (float *)(pp + wl.A);
    d.c1 = (float *)(pp + wl.c1);
    d.binv = (float *)(pp + wl.binv);
    d.bok = (int *)(pp + wl.bok);
  }
  hipStream_t s = as_stream(stream);
  if (hipMemcpyAsync(ws, &pl, sizeof(Plan), hipMemcpyHostToDevice, s) != hipSuccess) return IA355_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return IA355_ERR_HIP;
  return IA355_OK;
}

extern "C" size_t ia355_batch_lds_bytes(int32_t rays_per_tile, int32_t samples_per_segment,
                                        int32_t waves_per_group) {
  if (rays_per_tile < 1 || rays_per_tile > kMaxTileRays || samples_per_segment < 2 * kMaxSteps ||
      samples_per_segment > 8192 || (waves_per_group != 4 && waves_per_group != 8))
    return 0;
  return sizeof(Store) + (size_t)waves_per_group * wave_bytes(rays_per_tile, samples_per_segment);
}

namespace {

typedef void (*RenderFn)(const Plan *, size_t, int *, int, int);

// The instantiation for (waves per workgroup, workgroups per CU), or null.
RenderFn render_fn(int waves, int groups) {
  if (waves == 4 && groups == 1) return render_kernel<4, 1>;
  if (waves == 4 && groups == 2) return render_kernel<4, 2>;
  if (waves == 4 && groups == 3) return render_kernel<4, 3>;
  if (waves == 4 && groups == 4) return render_kernel<4, 4>;
  if (waves == 8 && groups == 1) return render_kernel<8, 1>;
  if (waves == 8 && groups == 2) return render_kernel<8, 2>;
  return nullptr;
}

// LDS a workgroup may take on the current device (cached per device).
int32_t lds_limit(size_t *limit) {
  static std::mutex mu;
  static int cached[64];
  static bool have[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return IA355_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!have[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return IA355_ERR_HIP;
    cached[dev] = v;
    have[dev] = true;
  }
  *limit = (size_t)cached[dev];
  return IA355_OK;
}

}  // namespace

extern "C" int32_t ia355_batch_render(const void *ws, size_t ws_bytes, int32_t rays_per_tile,
                                      int32_t samples_per_segment, int32_t waves_per_group, int32_t blocks_per_cu,
                                      ia355_stream_t stream) {
  if (!ws || ws_bytes < align256(sizeof(Plan)) + 256) return IA355_ERR_WORKSPACE;
  const size_t lds = ia355_batch_lds_bytes(rays_per_tile, samples_per_segment, waves_per_group);
  if (lds == 0 || blocks_per_cu < 1) return IA355_ERR_INVALID_ARG;
  const RenderFn fn = render_fn(waves_per_group, blocks_per_cu);
  if (!fn) return IA355_ERR_UNSUPPORTED;
  size_t limit = 0;
  const int32_t st = lds_limit(&limit);
  if (st != IA355_OK) return st;
  if (lds > limit) return IA355_ERR_UNSUPPORTED;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return IA355_ERR_HIP;
  hipStream_t s = as_stream(stream);
  const Plan *pl = (const Plan *)ws;
  int *queue = (int *)((char *)ws + align256(sizeof(Plan)));
  prep_kernel<<<1024, kPrepBlock, 0, s>>>(pl, ws_bytes, queue);
  hipLaunchKernelGGL(fn, dim3(256 * blocks_per_cu), dim3(waves_per_group * kWave), lds, s, pl, ws_bytes, queue,
                     rays_per_tile, samples_per_segment);
  return launch_status();
}
