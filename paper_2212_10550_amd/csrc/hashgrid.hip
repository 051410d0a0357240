// Multiresolution hash encoding (Sec. 3.1, Instant-NGP) forward and backward.
//
// Forward design (gfx950, 8 XCDs with a private 4 MB L2 each):
//  * one thread per (sample, level); a block covers 256 consecutive samples
//    of ONE level, so its gathers stay inside one level's table;
//  * workgroups are dispatched round-robin over the 8 XCDs, so block b runs
//    on XCD b % 8.  Levels are assigned to XCDs by that residue (XCD k gets
//    levels k, k+8, ...), so each XCD's L2 caches only its own levels'
//    tables (2 x 2 MiB at T = 2^19 in FP16) instead of all sixteen;
//  * the position scaling u = x N_l is split into a rounded product and its
//    exact FMA remainder, so the cell and fraction are accurate to FP32
//    relative precision even at N_l ~ 2000;
//  * features are written level-major [L][S][F]: each block writes one
//    contiguous run (coalesced 8-byte / 4-byte stores per lane).
// Backward: the table gradient is FP32 atomics laid out so that each wave
// instruction touches few cache lines (see table_grad_kernel); the position
// gradient runs one wave per 4 samples x 16 levels (lane = level + 16 *
// sample) and is reduced across the 16 level lanes with shuffles
// (deterministic).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "hash_dev.h"

using namespace ia355;
using namespace ia355::hsh;

namespace {

constexpr int kFwdBlock = 256;
constexpr int64_t kTwoSampleMin = (int64_t)1 << 22;  // samples (or capacity) from which a lane takes two

// Level of a lane's slot t in level group g on XCD x, or -1 (no level).  With
// two levels per lane and at most 16 levels, XCD x serves level x and level
// L - 1 - x (when that is 8 or more): coarse levels, whose samples share
// cells, pair with fine ones, whose gathers are scattered, so every XCD gets
// a similar load and at most one fine table.  Otherwise XCD x serves levels
// x + 8 (kLv g + t).
template <int kLv>
__device__ __forceinline__ int xcd_level(int x, int g, int t, int L) {
  if (kLv == 2 && L <= 2 * kXcd) {
    const int l = t == 0 ? x : L - 1 - x;
    return (t == 0 ? l < L : l >= kXcd) ? l : -1;
  }
  const int l = x + kXcd * (kLv * g + t);
  return l < L ? l : -1;
}

// Block b works for XCD b % 8 on the levels xcd_level gives its slots t <
// kLv in level group g = slot % ngroup (slot = b / 8), on chunks of
// 256 kSp samples slot / ngroup, + nslot, + 2 nslot ...  A lane takes kSp
// samples of a chunk (256 apart) and reads each sample's position and bone
// once for its kLv levels; all their corner gathers are in flight together.
template <typename TT, typename FT, int kLv, int kSp>
__global__ void __launch_bounds__(kFwdBlock) encode_kernel(const float *__restrict__ xc, const int16_t *__restrict__ bone,
                                                           int64_t S, const int64_t *__restrict__ S_dev, int64_t ld,
                                                           const TT *__restrict__ table, int L, int log2T, Levels lv,
                                                           Box box, FT *__restrict__ feat, int ngroup) {
  const int xcd = blockIdx.x % kXcd;
  const int slot = blockIdx.x / kXcd;
  int lev[kLv];
#pragma unroll
  for (int t = 0; t < kLv; ++t) lev[t] = xcd_level<kLv>(xcd, slot % ngroup, t, L);
  if (lev[0] < 0) return;
  const int64_t Sn = count_of(S, S_dev);
  const int64_t nslot = gridDim.x / (kXcd * ngroup);
  const uint32_t T = 1u << log2T;
  constexpr int64_t kSpan = (int64_t)kFwdBlock * kSp;
  for (int64_t chunk = slot / ngroup; chunk * kSpan < Sn; chunk += nslot) {
    int64_t n[kSp];
    float x[kSp][3];
    int bv[kSp];
    bool in[kSp], use[kSp];
    // positions and bones loaded together (one round trip; the bones are
    // tested only after every load is issued)
#pragma unroll
    for (int sp = 0; sp < kSp; ++sp) {
      n[sp] = chunk * kSpan + sp * kFwdBlock + threadIdx.x;
      in[sp] = n[sp] < Sn;
      const int64_t m = in[sp] ? n[sp] : 0;
      x[sp][0] = xc[m];
      x[sp][1] = xc[ld + m];
      x[sp][2] = xc[2 * ld + m];
      bv[sp] = 0;
    }
    if (bone)
#pragma unroll
      for (int sp = 0; sp < kSp; ++sp) bv[sp] = bone[in[sp] ? n[sp] : 0];
#pragma unroll
    for (int sp = 0; sp < kSp; ++sp) use[sp] = in[sp] && bv[sp] >= 0;
    float a[kSp][kLv], b[kSp][kLv];
#pragma unroll
    for (int sp = 0; sp < kSp; ++sp)
#pragma unroll
      for (int t = 0; t < kLv; ++t) a[sp][t] = b[sp][t] = 0.0f;
    // every lane encodes (no branch around the gathers, so all of them are
    // in flight together; any position gives in-range cells); samples
    // without a root then store zeros
#pragma unroll
    for (int sp = 0; sp < kSp; ++sp)
#pragma unroll
      for (int t = 0; t < kLv; ++t) {
        const int level = lev[t];
        if (level >= 0)
          encode_level(x[sp], box, lv.res[level], lv.dense[level], T - 1u, table + (int64_t)level * T * 2, &a[sp][t],
                       &b[sp][t]);
      }
#pragma unroll
    for (int sp = 0; sp < kSp; ++sp)
      if (in[sp])
#pragma unroll
        for (int t = 0; t < kLv; ++t) {
          const int level = lev[t];
          if (level >= 0)
            store_feat2(feat, (int64_t)level * ld + n[sp], use[sp] ? a[sp][t] : 0.0f, use[sp] ? b[sp][t] : 0.0f);
        }
  }
}

struct EncodeArgs {
  const float *xc;
  const int16_t *bone;
  int64_t S;
  const int64_t *S_dev;
  int64_t ld;
  const void *table;
  int L, log2T;
  Levels lv;
  Box box;
  void *feat;
  int ngroup;
};

template <typename TT, typename FT>
void launch_encode(const EncodeArgs &a, int lv_lane, int sp_lane, unsigned g, hipStream_t s) {
  const TT *t = static_cast<const TT *>(a.table);
  FT *f = static_cast<FT *>(a.feat);
  if (lv_lane == 2 && sp_lane == 2)
    encode_kernel<TT, FT, 2, 2><<<g, kFwdBlock, 0, s>>>(a.xc, a.bone, a.S, a.S_dev, a.ld, t, a.L, a.log2T, a.lv, a.box,
                                                        f, a.ngroup);
  else if (lv_lane == 2)
    encode_kernel<TT, FT, 2, 1><<<g, kFwdBlock, 0, s>>>(a.xc, a.bone, a.S, a.S_dev, a.ld, t, a.L, a.log2T, a.lv, a.box,
                                                        f, a.ngroup);
  else
    encode_kernel<TT, FT, 1, 1><<<g, kFwdBlock, 0, s>>>(a.xc, a.bone, a.S, a.S_dev, a.ld, t, a.L, a.log2T, a.lv, a.box,
                                                        f, a.ngroup);
}

// Position gradient dL/dx = sum_l sum_c (grad w_c) (theta_c . dL/dfeat_l),
// in two kernels.  The first has the forward's mapping (block b on XCD
// b % 8, the levels xcd_level gives, one lane per sample): every sample of a
// level is served by one XCD's L2, so cells shared by samples are fetched
// once rather than once per XCD; it writes each level's contribution to a
// workspace part [L][3][S].  The second sums the levels in a fixed order.
constexpr int kBwdBlock = 256;
constexpr int kBwdMaxLevels = 16;  // the backward's level limit

template <typename TT, int kLv>
__global__ void __launch_bounds__(kBwdBlock) xgrad_level_kernel(
    const float *__restrict__ gfeat, const float *__restrict__ xc, const int16_t *__restrict__ bone, int64_t S,
    const int64_t *__restrict__ S_dev, int64_t ld, const TT *__restrict__ table, int L, int log2T, Levels lv, Box box,
    float *__restrict__ part, int ngroup) {
  // the encode's mapping: kLv levels (b % 8) + 8 (kLv g + t) per lane
  const int xcd = blockIdx.x % kXcd;
  const int slot = blockIdx.x / kXcd;
  int lev[kLv];
#pragma unroll
  for (int t = 0; t < kLv; ++t) lev[t] = xcd_level<kLv>(xcd, slot % ngroup, t, L);
  if (lev[0] < 0) return;
  const int64_t Sn = count_of(S, S_dev);
  const int64_t nslot = gridDim.x / (kXcd * ngroup);
  const uint32_t T = 1u << log2T;
  for (int64_t chunk = slot / ngroup; chunk * kBwdBlock < Sn; chunk += nslot) {
    const int64_t n = chunk * kBwdBlock + threadIdx.x;
    if (n >= Sn) break;
    float gx[kLv][3];
    float2 g[kLv];
    // position, incoming gradients and bone loaded together (one round trip)
    const float x[3] = {xc[n], xc[ld + n], xc[2 * ld + n]};
#pragma unroll
    for (int t = 0; t < kLv; ++t) {
      const int level = lev[t];
      g[t] = level >= 0 ? reinterpret_cast<const float2 *>(gfeat)[(int64_t)level * ld + n] : make_float2(0.0f, 0.0f);
      gx[t][0] = gx[t][1] = gx[t][2] = 0.0f;
    }
    if (!bone || bone[n] >= 0) {
      // every level's gathers first, then the sums (a missing second level
      // repeats the first with a zero gradient and is not stored)
      Corners c[kLv];
      float2 vv[kLv][8];
#pragma unroll
      for (int t = 0; t < kLv; ++t) {
        const int level = lev[t] >= 0 ? lev[t] : lev[0];
        level_cell(x, box, lv.res[level], lv.dense[level], T - 1u, c[t], true);
        gather8(table + (int64_t)level * T * 2, c[t], vv[t]);
      }
#pragma unroll
      for (int t = 0; t < kLv; ++t)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float d = vv[t][k].x * g[t].x + vv[t][k].y * g[t].y;
          gx[t][0] += c[t].dw[k][0] * d;
          gx[t][1] += c[t].dw[k][1] * d;
          gx[t][2] += c[t].dw[k][2] * d;
        }
    }
#pragma unroll
    for (int t = 0; t < kLv; ++t) {
      const int level = lev[t];
      if (level < 0) continue;
      float *pl = part + (int64_t)level * 3 * S;
      pl[n] = gx[t][0];
      pl[S + n] = gx[t][1];
      pl[2 * S + n] = gx[t][2];
    }
  }
}

template <typename TT>
void launch_xgrad(int lv_lane, unsigned blocks, hipStream_t s, const float *gfeat, const float *xc,
                  const int16_t *bone, int64_t S, const int64_t *S_dev, int64_t ld, const void *table, int L, int log2T,
                  const Levels &lv, const Box &box, float *part, int ngroup) {
  const TT *t = static_cast<const TT *>(table);
  if (lv_lane == 2)
    xgrad_level_kernel<TT, 2><<<blocks, kBwdBlock, 0, s>>>(gfeat, xc, bone, S, S_dev, ld, t, L, log2T, lv, box, part,
                                                           ngroup);
  else
    xgrad_level_kernel<TT, 1><<<blocks, kBwdBlock, 0, s>>>(gfeat, xc, bone, S, S_dev, ld, t, L, log2T, lv, box, part,
                                                           ngroup);
}

__global__ void __launch_bounds__(kBwdBlock) xgrad_sum_kernel(const float *__restrict__ part, int64_t S,
                                                              const int64_t *__restrict__ S_dev, int L, int64_t ld,
                                                              float *__restrict__ gxc) {
  const int64_t Sn = count_of(S, S_dev);
  for (int64_t n = (int64_t)blockIdx.x * kBwdBlock + threadIdx.x; n < Sn; n += (int64_t)gridDim.x * kBwdBlock) {
    // all loads first (independent addresses), then the sums in level order
    float v[kBwdMaxLevels][3];
#pragma unroll
    for (int l = 0; l < kBwdMaxLevels; ++l)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[l][a] = l < L ? part[((int64_t)l * 3 + a) * S + n] : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float acc = 0.0f;
#pragma unroll
      for (int l = 0; l < kBwdMaxLevels; ++l)
        if (l < L) acc += v[l][a];
      gxc[a * ld + n] = acc;
    }
  }
}

// Table gradient with coalesced atomics.  FP32 atomics to random addresses
// are limited by L2 requests (one per touched cache line per instruction),
// not by the number of floats added, so the mapping packs updates that
// share lines into the same wave instruction: 16 lanes per (level, sample)
// item, lane = 2 * corner + feature.  The two features of a corner are
// adjacent floats and x-neighbouring corners are adjacent entries (dense
// levels) or differ only in low bits (hashed levels, x prime = 1), so the
// 16 updates of an item touch about four lines.  Items are level-major, so
// the four items of a wave are consecutive samples of one level and share
// lines on the coarse levels as well.
constexpr int kTgBlock = 256;
constexpr int kTgMaxGrid = 1024;      // 4 blocks per CU
constexpr int kTgDenseMaxGrid = 512;  // 2 blocks per CU

__global__ void __launch_bounds__(kTgBlock) table_grad_kernel(const float *__restrict__ gfeat,
                                                             const float *__restrict__ xc,
                                                             const int16_t *__restrict__ bone, int64_t S,
                                                             const int64_t *__restrict__ S_dev, int64_t ld, int l0,
                                                             int L, int log2T, Levels lv, Box box,
                                                             float *__restrict__ gtable) {
  const int64_t Sn = count_of(S, S_dev);
  const int64_t items = (int64_t)(L - l0) * Sn;
  const int sub = (int)(threadIdx.x & 15), k = sub >> 1, f = sub & 1;
  const uint32_t T = 1u << log2T;
  for (int64_t item = ((int64_t)blockIdx.x * kTgBlock + threadIdx.x) >> 4; item < items;
       item += (int64_t)gridDim.x * (kTgBlock / 16)) {
    const int level = l0 + (int)(item / Sn);
    const int64_t n = item - (int64_t)(level - l0) * Sn;  // 0 <= n < Sn
    if (bone && bone[n] < 0) continue;
    const float x[3] = {xc[n], xc[ld + n], xc[2 * ld + n]};
    // this lane's corner only (a runtime-indexed corner array would live in
    // scratch memory)
    const int N = lv.res[level];
    const CellPos cp = level_pos(x, box, N);
    const uint32_t idx = corner_index(cp, k, N, lv.dense[level] != 0, T - 1u);
    const float g = gfeat[2 * ((int64_t)level * ld + n) + f];
    atomicAdd(gtable + 2 * ((int64_t)level * T + idx) + f, corner_weight(cp, k) * g);
  }
}

// Dense (coarse) levels: many consecutive samples fall in the same cell, so
// the same table entries are hit again and again (atomic contention).  One
// lane per sample (a wave = 64 consecutive samples of one level); for each
// corner the lanes are segmented into runs of equal table index and a
// segmented wave scan sums each run, so only the last lane of a run issues
// the atomic adds.
constexpr int kDgBlock = 256;
constexpr int kAggMaxRes = 32;  // finest resolution handled by run aggregation

__global__ void __launch_bounds__(kDgBlock) table_grad_dense_kernel(const float *__restrict__ gfeat,
                                                                   const float *__restrict__ xc,
                                                                   const int16_t *__restrict__ bone, int64_t S,
                                                                   const int64_t *__restrict__ S_dev, int64_t ld,
                                                                   int ndense, int log2T, Levels lv, Box box,
                                                                   float *__restrict__ gtable) {
  const int64_t Sn = count_of(S, S_dev);
  const int64_t chunks = ceil_div(Sn, kDgBlock);
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t T = 1u << log2T;
  // one (level, chunk) pair per block and step; the whole wave takes part
  // in the scans below
  for (int64_t p = blockIdx.x; p < (int64_t)ndense * chunks; p += gridDim.x) {
    const int level = (int)(p / chunks);
    const int64_t n = (p % chunks) * kDgBlock + threadIdx.x;
    const bool act = n < Sn && (!bone || bone[n] >= 0);
    Corners c;
    float2 g = make_float2(0.0f, 0.0f);
    if (act) {
      const float x[3] = {xc[n], xc[ld + n], xc[2 * ld + n]};
      level_cell(x, box, lv.res[level], true, T - 1u, c, false);
      g = reinterpret_cast<const float2 *>(gfeat)[(int64_t)level * ld + n];
    }
    float *gl = gtable + (int64_t)level * T * 2;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int key = act ? (int)c.idx[k] : -1 - lane;  // inactive lanes: unique keys, no atomics
      float v0 = act ? c.w[k] * g.x : 0.0f, v1 = act ? c.w[k] * g.y : 0.0f;
      const int prev = __shfl_up(key, 1, kWave);
      int hs = (lane == 0 || prev != key) ? lane : 0;  // run head index
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(hs, o, kWave);
        if (lane >= o) hs = max(hs, t);
      }
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const float t0 = __shfl_up(v0, o, kWave), t1 = __shfl_up(v1, o, kWave);
        if (lane - o >= hs) {
          v0 += t0;
          v1 += t1;
        }
      }
      const int next = __shfl_down(key, 1, kWave);
      if ((lane == kWave - 1 || next != key) && key >= 0) {
        atomicAdd(gl + 2 * key, v0);
        atomicAdd(gl + 2 * key + 1, v1);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Table gradient without global atomics (binned).  Each level's table is cut
// into tiles of E = 2^tb entries (2 E 8-byte sums fit in LDS); a corner update
// (level, entry, w_c dL/dfeat_l) belongs to bin (level, tile), bins in
// level-major order.  Five passes:
//  1. count: every block counts its updates per bin in LDS and writes its
//     row of the histogram hist[block][bin] (contiguous: a column per block
//     would cost a 32-byte sector per 4-byte count, written and read back);
//  2. scan: exclusive scan of the histogram in bin-major order (bin, then
//     block), in chunks of 4096 (offsets inside the chunk, chunk totals),
//     each count replaced by its offset in place;
//  3. plan (one block): offsets of the chunks, the record range of every bin
//     and the number of accumulation chunks it needs (<= kAccChunk records
//     each);
//  4. scatter: the same blocks regenerate the same updates (same items, same
//     arithmetic) and append them to their run inside their bin's records,
//     one 12-byte record each (the two values, the entry inside the tile);
//  5. accumulate: one workgroup per chunk sums its records into an LDS copy
//     of the tile and writes the tile with plain vector stores; a bin split
//     over several chunks (only bins with many updates, on the coarse
//     levels) adds its nonzero entries with global atomics instead, after a
//     pass that clears those tiles when overwriting.
// The LDS sums are 64-bit fixed point, added exactly: LDS float atomic adds run at
// about a sixteenth of the rate of integer ones on gfx950, so each chunk
// scales its values by a power of two 2^s chosen from its largest |value| m
// and record count (no overflow), adds them as integers and converts each
// entry back once.  Each record is rounded to the quantum 2^-s < m 2^-46, so
// an entry's error is at most (its records) x m 2^-47 plus one FP32
// rounding: an absolute bound relative to the chunk's largest value.  An
// entry near m is as accurate as FP32 adds leave it or better; one far
// below m (under about m 2^-24) is less accurate than FP32 adds, and a
// record below m 2^-48 rounds to zero.  Integer addition is associative, so
// a tile summed by one workgroup does not depend on the order of its records.
// Every tile of the selected levels is written, so an overwrite needs no
// separate clear.  The HBM traffic is the records (12 bytes per corner
// update, written once and read once) and one pass over the table slice.
constexpr int kBinBlock = 1024;       // count / scatter
constexpr int kBinMaxBlocks = 256;    // one block per CU
constexpr int kBinUnroll = 4;         // items per thread whose loads are in flight together
constexpr int kMaxBins = 16384;       // LDS counters of one block: 64 KB
constexpr int kTileLog2Max = 12;      // 4096 entries x 2 x 8 B = 64 KB of LDS
constexpr int kHsPer = 4;
constexpr int kHsChunk = 1024 * kHsPer;
constexpr int kMaxHsChunks = 4096;
constexpr int kAccBlock = 1024;
constexpr uint32_t kAccChunk = 4096;  // records per accumulation workgroup
constexpr int kAccPer = kAccChunk / kAccBlock;  // records per thread, held in registers
constexpr int kAccWr = (1 << (kTileLog2Max - 1)) / kAccBlock;  // float4 of a tile per thread
constexpr int kAccMaxGrid = 2048;
static_assert(kAccChunk <= (1u << 12) && kAccChunk % kAccBlock == 0, "bin_accum_kernel: scale and record slots");

struct BinGeom {
  int tb;         // log2 entries per tile
  int tpl_log2;   // log2 tiles per level
  int nbins;
  int P;          // count / scatter blocks
  int64_t H;      // histogram entries nbins * P
  int nchunk;     // histogram scan chunks
  int64_t rmax;   // record capacity: levels * S * 8
  int64_t qmax;   // accumulation chunks at most
};

inline bool bin_geom(int nl, int64_t S, int log2T, BinGeom *g) {
  if (nl <= 0 || S < 0 || log2T < 1 || log2T > 30) return false;
  g->tb = log2T < kTileLog2Max ? log2T : kTileLog2Max;
  g->tpl_log2 = log2T - g->tb;
  const int64_t nb = (int64_t)nl << g->tpl_log2;
  if (nb > kMaxBins) return false;
  g->nbins = (int)nb;
  int64_t p = ceil_div((int64_t)nl * (S > 0 ? S : 1), (int64_t)kBinBlock);
  g->P = (int)(p < 1 ? 1 : (p > kBinMaxBlocks ? kBinMaxBlocks : p));
  g->H = (int64_t)g->nbins * g->P;
  g->nchunk = (int)ceil_div(g->H, kHsChunk);
  g->rmax = (int64_t)nl * S * 8;
  g->qmax = g->nbins + ceil_div(g->rmax, (int64_t)kAccChunk);
  return g->nchunk <= kMaxHsChunks && g->rmax < 0xffffffffLL;
}

struct BinWs {
  uint32_t *hist, *csum, *chunk_first;
  uint4 *chunk_info;  // per accumulation chunk: bin, first record, end, chunks of the bin
  float3 *rec;  // (value 0, value 1, entry inside the tile as bits)
  size_t bytes;
};

inline BinWs bin_ws(const BinGeom &g, void *base) {
  BinWs w;
  char *p = (char *)base;
  size_t o = 0;
  w.hist = (uint32_t *)(p + o);
  o += align256(sizeof(uint32_t) * (size_t)g.H);
  w.csum = (uint32_t *)(p + o);
  o += align256(sizeof(uint32_t) * (size_t)g.nchunk);
  w.chunk_first = (uint32_t *)(p + o);
  o += align256(sizeof(uint32_t) * ((size_t)g.nbins + 1));
  w.chunk_info = (uint4 *)(p + o);
  o += align256(sizeof(uint4) * (size_t)g.qmax);
  w.rec = (float3 *)(p + o);
  o += align256(sizeof(float3) * (size_t)(g.rmax > 0 ? g.rmax : 1));
  w.bytes = o;
  return w;
}

// Exclusive scan of one value per thread over a 1024-thread block; *total
// gets the block's sum (the same in every thread).
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t *wsum, uint32_t *total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    base += w < wid ? wsum[w] : 0u;
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - v;
}

// Adds 1 to the LDS counter c[bin] for each lane with act and returns the
// counter's old value plus the lane's rank among the wave's lanes with the
// same bin.  When every active lane has the same bin (coarse levels: one
// tile per level, consecutive samples) the wave does one add of the lane
// count instead of 64 adds serialised on one LDS address.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t *c, int bin, bool act) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t am = __ballot(act);
  if (am == 0ull) return 0u;
  const int first = __ffsll((unsigned long long)am) - 1;
  const int b0 = __shfl(bin, first, kWave);
  const uint64_t same = __ballot(act && bin == b0);
  if (same == am) {
    uint32_t base = 0u;
    if (lane == first) base = atomicAdd(&c[bin], (uint32_t)__popcll(am));
    base = __shfl(base, first, kWave);
    return base + (uint32_t)__popcll(am & ((1ull << lane) - 1ull));
  }
  return act ? atomicAdd(&c[bin], 1u) : 0u;
}

// Items of the count and scatter passes: item it = level (l0 + it / Sn),
// sample it % Sn; thread t of block b takes items b * 1024 + t + j * stride
// (stride = blocks * 1024), kBinUnroll of them per round with their loads
// issued together.  Both passes visit the same items in the same blocks and
// compute the corner entries with the same code, so their per-(bin, block)
// counts agree.
struct BinItem {
  int lr;
  bool act;
  float x[3];
  float2 g;
};

template <bool kWithGrad>
__device__ __forceinline__ void load_items(int64_t i0, int64_t stride, int64_t items, int64_t Sn,
                                           const float *__restrict__ xc, const int16_t *__restrict__ bone,
                                           const float *__restrict__ gfeat, int64_t ld, int l0,
                                           BinItem (&b)[kBinUnroll]) {
#pragma unroll
  for (int j = 0; j < kBinUnroll; ++j) {
    const int64_t it = i0 + j * stride;
    const bool in = it < items;
    // items < 2^32 (the record count is), so 32-bit division suffices
    const uint32_t lr = in ? (uint32_t)it / (uint32_t)Sn : 0u;
    const int64_t n = in ? it - (int64_t)lr * Sn : 0;
    b[j].lr = (int)lr;
    // all loads issued together; n < Sn keeps them in bounds
    const bool valid = !bone || bone[n] >= 0;
    b[j].x[0] = xc[n];
    b[j].x[1] = xc[ld + n];
    b[j].x[2] = xc[2 * ld + n];
    b[j].g = kWithGrad ? reinterpret_cast<const float2 *>(gfeat)[(int64_t)(l0 + b[j].lr) * ld + n]
                       : make_float2(0.0f, 0.0f);
    b[j].act = in && valid;
  }
}

__global__ void __launch_bounds__(kBinBlock) bin_count_kernel(const float *__restrict__ xc,
                                                             const int16_t *__restrict__ bone, int64_t S,
                                                             const int64_t *__restrict__ S_dev, int64_t ld, int l0,
                                                             int nl, int log2T, int tb, Levels lv, Box box,
                                                             uint32_t *__restrict__ hist) {
  extern __shared__ uint32_t cnt[];
  const int tpl_log2 = log2T - tb;
  const int nbins = nl << tpl_log2;
  for (int i = threadIdx.x; i < nbins; i += kBinBlock) cnt[i] = 0u;
  __syncthreads();
  const int64_t Sn = count_of(S, S_dev);
  const int64_t items = (int64_t)nl * Sn;
  const uint32_t T = 1u << log2T;
  const int64_t stride = (int64_t)gridDim.x * kBinBlock;
  // the loop bound is wave-uniform at kBinUnroll granularity: lanes past the
  // end stay in with act = false (the reservations use wave ballots)
  for (int64_t w0 = (int64_t)blockIdx.x * kBinBlock + (threadIdx.x & ~(kWave - 1)); w0 < items;
       w0 += stride * kBinUnroll) {
    BinItem b[kBinUnroll];
    load_items<false>(w0 + (threadIdx.x & (kWave - 1)), stride, items, Sn, xc, bone, nullptr, ld, l0, b);
#pragma unroll
    for (int j = 0; j < kBinUnroll; ++j) {
      const int level = l0 + b[j].lr;
      const int N = lv.res[level];
      const CellPos cp = level_pos(b[j].x, box, N);
      const bool dense = lv.dense[level] != 0;
      // dense levels: few tiles, neighbouring samples share them (one add
      // per wave); hashed levels: bins spread over the tiles (plain adds)
      if (__ballot(b[j].act && dense) != 0ull) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t idx = corner_index(cp, k, N, dense, T - 1u);
          wave_reserve(cnt, (b[j].lr << tpl_log2) + (int)(idx >> tb), b[j].act);
        }
      } else if (b[j].act) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t idx = corner_index(cp, k, N, dense, T - 1u);
          atomicAdd(&cnt[(b[j].lr << tpl_log2) + (int)(idx >> tb)], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += kBinBlock) hist[(int64_t)blockIdx.x * nbins + i] = cnt[i];
}

// Exclusive scan of one chunk of the histogram in bin-major order (element
// j = bin P + block), in place in hist[block][bin].  The chunk's elements
// sit in a rectangle of rows (blocks) by a few bins; they are read and
// written row by row (neighbouring threads, neighbouring bins) through an
// LDS copy in j order, whose rows of P are padded by one word so a row
// walk does not fall on one bank.  H = nbins P < 2^23.
__global__ void __launch_bounds__(1024) bin_hist_scan_kernel(uint32_t *__restrict__ hist, int64_t H, int P, int nbins,
                                                            uint32_t *__restrict__ csum) {
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t sv[2 * kHsChunk + 1];  // e + e / P for e < kHsChunk
  const uint32_t up = (uint32_t)P;
  const uint32_t j0 = (uint32_t)blockIdx.x * kHsChunk;
  const uint32_t j1 = (int64_t)j0 + kHsChunk < H ? j0 + kHsChunk : (uint32_t)H;
  const uint32_t b_lo = j0 / up, nb = (j1 - 1) / up - b_lo + 1;  // bins the chunk touches
  const uint32_t R = up * nb;                                     // rectangle: P rows by nb bins
  for (uint32_t r = threadIdx.x; r < R; r += 1024) {
    const uint32_t p = r / nb, b = b_lo + r % nb, j = b * up + p;
    if (j >= j0 && j < j1) {
      const uint32_t e = j - j0;
      sv[e + e / up] = hist[(int64_t)p * nbins + b];
    }
  }
  __syncthreads();
  const uint32_t e0 = threadIdx.x * kHsPer;
  uint32_t v[kHsPer], run = 0;
#pragma unroll
  for (int q = 0; q < kHsPer; ++q) {
    const uint32_t e = e0 + q;
    v[q] = j0 + e < j1 ? sv[e + e / up] : 0u;
    run += v[q];
  }
  uint32_t total;
  uint32_t off = block_scan_u32(run, wsum, &total);  // its barriers order the reads above and the writes below
#pragma unroll
  for (int q = 0; q < kHsPer; ++q) {
    const uint32_t e = e0 + q;
    if (j0 + e < j1) sv[e + e / up] = off;
    off += v[q];
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < R; r += 1024) {
    const uint32_t p = r / nb, b = b_lo + r % nb, j = b * up + p;
    if (j >= j0 && j < j1) {
      const uint32_t e = j - j0;
      hist[(int64_t)p * nbins + b] = sv[e + e / up];
    }
  }
  if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) bin_plan_kernel(const uint32_t *__restrict__ hist, uint32_t *__restrict__ csum,
                                                       int nchunk, int nbins, int P,
                                                       uint32_t *__restrict__ chunk_first,
                                                       uint4 *__restrict__ chunk_info) {
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t coff[kMaxHsChunks];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nchunk; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const uint32_t v = i < nchunk ? csum[i] : 0u;
    uint32_t total;
    const uint32_t off = block_scan_u32(v, wsum, &total);
    if (i < nchunk) coff[i] = carry + off;
    carry += total;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nchunk; i += 1024) csum[i] = coff[i];  // chunk offsets for the scatter pass
  const uint32_t n_rec = carry;
  uint32_t ccarry = 0;
  for (int b0 = 0; b0 < nbins; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    uint32_t nch = 0, st = 0, en = 0;
    if (b < nbins) {
      // block 0's offset of bin b (row 0 of hist[block][bin])
      const int64_t j = (int64_t)b * P;
      st = hist[b] + coff[j / kHsChunk];
      en = n_rec;
      if (b + 1 < nbins) {
        const int64_t j1 = j + P;
        en = hist[b + 1] + coff[j1 / kHsChunk];
      }
      nch = en > st ? (en - st + kAccChunk - 1) / kAccChunk : 1u;
    }
    uint32_t total;
    const uint32_t off = block_scan_u32(nch, wsum, &total);
    if (b < nbins) {
      chunk_first[b] = ccarry + off;
      for (uint32_t c = 0; c < nch; ++c) {
        const uint32_t rb = st + c * kAccChunk;
        chunk_info[ccarry + off + c] = make_uint4((uint32_t)b, rb, en - rb > kAccChunk ? rb + kAccChunk : en, nch);
      }
    }
    ccarry += total;
  }
  if (threadIdx.x == 0) {
    chunk_first[nbins] = ccarry;
  }
}

__global__ void __launch_bounds__(kBinBlock) bin_scatter_kernel(
    const float *__restrict__ gfeat, const float *__restrict__ xc, const int16_t *__restrict__ bone, int64_t S,
    const int64_t *__restrict__ S_dev, int64_t ld, int l0, int nl, int log2T, int tb, Levels lv, Box box,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ coff, float3 *__restrict__ rec, uint32_t rmax) {
  extern __shared__ uint32_t cur[];
  const int tpl_log2 = log2T - tb;
  const int nbins = nl << tpl_log2;
  const int P = gridDim.x;
  for (int i = threadIdx.x; i < nbins; i += kBinBlock) {
    const int64_t j = (int64_t)i * P + blockIdx.x;  // bin-major position
    cur[i] = hist[(int64_t)blockIdx.x * nbins + i] + coff[j / kHsChunk];
  }
  __syncthreads();
  const int64_t Sn = count_of(S, S_dev);
  const int64_t items = (int64_t)nl * Sn;
  const uint32_t T = 1u << log2T;
  const uint32_t emask = (1u << tb) - 1u;
  const int64_t stride = (int64_t)gridDim.x * kBinBlock;
  for (int64_t w0 = (int64_t)blockIdx.x * kBinBlock + (threadIdx.x & ~(kWave - 1)); w0 < items;
       w0 += stride * kBinUnroll) {
    BinItem b[kBinUnroll];
    load_items<true>(w0 + (threadIdx.x & (kWave - 1)), stride, items, Sn, xc, bone, gfeat, ld, l0, b);
#pragma unroll
    for (int j = 0; j < kBinUnroll; ++j) {
      const int level = l0 + b[j].lr;
      const int N = lv.res[level];
      const CellPos cp = level_pos(b[j].x, box, N);
      const bool dense = lv.dense[level] != 0;
      if (__ballot(b[j].act && dense) != 0ull) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t idx = corner_index(cp, k, N, dense, T - 1u);
          const float w = corner_weight(cp, k);
          const uint32_t pos = wave_reserve(cur, (b[j].lr << tpl_log2) + (int)(idx >> tb), b[j].act);
          if (b[j].act && pos < rmax)
            rec[pos] = make_float3(w * b[j].g.x, w * b[j].g.y, __uint_as_float(idx & emask));
        }
      } else if (b[j].act) {
        uint32_t idx[8], pos[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          idx[k] = corner_index(cp, k, N, dense, T - 1u);
          pos[k] = atomicAdd(&cur[(b[j].lr << tpl_log2) + (int)(idx[k] >> tb)], 1u);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float w = corner_weight(cp, k);
          if (pos[k] < rmax) rec[pos[k]] = make_float3(w * b[j].g.x, w * b[j].g.y, __uint_as_float(idx[k] & emask));
        }
      }
    }
  }
}

// Base of bin b's tile in the table gradient.
__device__ __forceinline__ float4 *tile_ptr(float *gtable, int b, int l0, int log2T, int tb) {
  const int tpl_log2 = log2T - tb;
  const int64_t level = l0 + (b >> tpl_log2);
  const int64_t tile = b & ((1 << tpl_log2) - 1);
  return reinterpret_cast<float4 *>(gtable + 2 * ((level << log2T) + (tile << tb)));
}

// Clears the tiles of bins split over several chunks (they are then summed
// with atomics); overwrite only.
__global__ void __launch_bounds__(256) bin_clear_split_kernel(const uint32_t *__restrict__ chunk_first, int nbins,
                                                             int l0, int log2T, int tb, float *__restrict__ gtable) {
  const int n4 = 1 << (tb - 1);  // float4 per tile (2 entries each)
  for (int b = blockIdx.x; b < nbins; b += gridDim.x) {
    if (chunk_first[b + 1] - chunk_first[b] <= 1u) continue;
    float4 *dst = tile_ptr(gtable, b, l0, log2T, tb);
    for (int j = threadIdx.x; j < n4; j += 256) dst[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// Block-wide max of v and OR of flag (1024 threads).
__device__ __forceinline__ float block_max(float v, bool flag, float *red, int *redf, bool *any) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  const bool wf = __ballot(flag) != 0ull;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
    red[wid] = v;
    redf[wid] = wf;
  }
  __syncthreads();
  float m = 0.0f;
  int f = 0;
  for (int w = 0; w < kAccBlock / kWave; ++w) {
    m = fmaxf(m, red[w]);
    f |= redf[w];
  }
  __syncthreads();
  *any = f != 0;
  return m;
}

// Four consecutive fixed-point sums back to FP32 (one rounding each).
__device__ __forceinline__ float4 from_fixed4(const unsigned long long *a, int s) {
  return make_float4((float)ldexp((double)(long long)a[0], -s), (float)ldexp((double)(long long)a[1], -s),
                     (float)ldexp((double)(long long)a[2], -s), (float)ldexp((double)(long long)a[3], -s));
}

// v * 2^s rounded to an integer, as two's complement bits (|v| 2^s < 2^48)
__device__ __forceinline__ unsigned long long to_fixed(float v, int s) {
  return (unsigned long long)(long long)rint((double)ldexpf(v, s));
}

__global__ void __launch_bounds__(kAccBlock) bin_accum_kernel(const float3 *__restrict__ rec,
                                                             const uint32_t *__restrict__ chunk_first,
                                                             const uint4 *__restrict__ chunk_info, int nbins,
                                                             uint32_t qmax, uint32_t rmax, int l0, int log2T, int tb,
                                                             int overwrite, float *__restrict__ gtable) {
  extern __shared__ unsigned long long acc[];  // 2 E fixed-point sums
  __shared__ float red[kAccBlock / kWave];
  __shared__ int redf[kAccBlock / kWave];
  const int n2 = 1 << tb;  // entries of a tile (2 sums each)
  const int n4 = n2 / 2;   // float4 (2 entries) per tile
  ulonglong2 *a2 = reinterpret_cast<ulonglong2 *>(acc);
  const uint32_t Q = chunk_first[nbins] < qmax ? chunk_first[nbins] : qmax;
  for (uint32_t q = blockIdx.x; q < Q; q += gridDim.x) {
    const uint4 ci = chunk_info[q];  // bin, first record, end, chunks of the bin
    const int b = (int)ci.x;
    const uint32_t rb = ci.y, re = ci.z, nch = ci.w;
    // a plan from this workspace always passes; the checks keep a misused
    // one (IA355_TABLE_REUSE_PLAN without a plan) inside the buffers
    if (ci.x >= (uint32_t)nbins || rb > re || re > rmax || re - rb > kAccChunk) continue;
    float4 *dst = tile_ptr(gtable, b, l0, log2T, tb);
    if (rb == re) {  // no update in this tile (then nch == 1)
      if (overwrite)
        for (int j = threadIdx.x; j < n4; j += kAccBlock) dst[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      continue;
    }
    // this thread's records (at most kAccPer), read once; non-finite values
    // stay out of the scale and the integer sums (added with atomics below)
    float3 v[kAccPer];
    float m = 0.0f;
    bool odd = false;
#pragma unroll
    for (int j = 0; j < kAccPer; ++j) {
      const uint32_t r = rb + threadIdx.x + j * kAccBlock;
      v[j] = r < re ? rec[r] : make_float3(0.0f, 0.0f, 0.0f);
      const bool fx = isfinite(v[j].x), fy = isfinite(v[j].y);
      m = fmaxf(m, fmaxf(fx ? fabsf(v[j].x) : 0.0f, fy ? fabsf(v[j].y) : 0.0f));
      odd = odd || !fx || !fy;
    }
    for (int j = threadIdx.x; j < n2; j += kAccBlock) a2[j] = make_ulonglong2(0ull, 0ull);
    // scale: |sum of the chunk's values| <= n max|v| < 2^(ex + 12) with
    // max|v| < 2^ex and n <= 2^12 records, so 2^s with s = 47 - ex keeps
    // every partial sum below 2^59
    bool odd_tile;  // some value of the chunk is NaN or infinite
    m = block_max(m, odd, red, redf, &odd_tile);  // its barriers also order the clear above
    int ex = 0;
    frexpf(m, &ex);  // m < 2^ex (m = 0: ex = 0)
    const int sc = 47 - ex;
#pragma unroll
    for (int j = 0; j < kAccPer; ++j) {
      if (rb + threadIdx.x + j * kAccBlock < re) {
        const uint32_t e = __float_as_uint(v[j].z) & (uint32_t)(n2 - 1);  // < E for every record written here
        if (isfinite(v[j].x)) atomicAdd(&acc[2 * e], to_fixed(v[j].x, sc));
        if (isfinite(v[j].y)) atomicAdd(&acc[2 * e + 1], to_fixed(v[j].y, sc));
      }
    }
    // NaN or infinite values (kept out of the integer sums) are added to a
    // float copy of the tile in LDS, so they reach their own entries as FP32
    // adds would; only chunks that hold such a value take this path
    float *fv = reinterpret_cast<float *>(acc);
    __syncthreads();  // the integer adds are complete
    if (odd_tile) {
      float4 tmp[kAccWr];
#pragma unroll
      for (int q = 0; q < kAccWr; ++q) {
        const int j = threadIdx.x + q * kAccBlock;
        if (j < n4) tmp[q] = from_fixed4(acc + 4 * j, sc);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kAccWr; ++q) {
        const int j = threadIdx.x + q * kAccBlock;
        if (j < n4) reinterpret_cast<float4 *>(fv)[j] = tmp[q];
      }
      __syncthreads();
      // the records again (from cache): keeping them in registers across
      // the write-out would cost occupancy on every chunk
      for (uint32_t r = rb + threadIdx.x; r < re; r += kAccBlock) {
        const float3 w = rec[r];
        const uint32_t e = __float_as_uint(w.z) & (uint32_t)(n2 - 1);
        if (!isfinite(w.x)) atomicAdd(&fv[2 * e], w.x);
        if (!isfinite(w.y)) atomicAdd(&fv[2 * e + 1], w.y);
      }
      __syncthreads();
    }
    for (int j = threadIdx.x; j < n4; j += kAccBlock) {
      float4 o = odd_tile ? reinterpret_cast<const float4 *>(fv)[j] : from_fixed4(acc + 4 * j, sc);
      if (nch == 1u) {  // the only writer of this tile
        if (!overwrite) {
          const float4 p = dst[j];
          o.x += p.x;
          o.y += p.y;
          o.z += p.z;
          o.w += p.w;
        }
        dst[j] = o;
      } else {
        float *df = reinterpret_cast<float *>(dst + j);
        if (o.x != 0.0f) atomicAdd(df, o.x);
        if (o.y != 0.0f) atomicAdd(df + 1, o.y);
        if (o.z != 0.0f) atomicAdd(df + 2, o.z);
        if (o.w != 0.0f) atomicAdd(df + 3, o.w);
      }
    }
    __syncthreads();  // the sums are cleared for the next chunk
  }
}

}  // namespace

extern "C" int32_t ia355_hashgrid_encode(const float *xc, const int16_t *bone, int64_t S, const int64_t *S_dev,
                                         int64_t ld, const void *table, int32_t table_dtype, int32_t L, int32_t F,
                                         int32_t log2T, double base_res, double growth, const float *aabb, void *feat,
                                         int32_t feat_dtype, ia355_stream_t stream) {
  if (S < 0 || ld < S || L <= 0 || L > kMaxLevels || F != 2 || log2T < 1 || log2T > 30) return IA355_ERR_INVALID_ARG;
  if (!table || (S > 0 && (!xc || !feat))) return IA355_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(table) & 15) != 0 || log2T < 2) return IA355_ERR_INVALID_ARG;  // block gathers
  if (table_dtype != IA355_F32 && table_dtype != IA355_F16) return IA355_ERR_INVALID_ARG;
  if (feat_dtype != IA355_F32 && feat_dtype != IA355_BF16) return IA355_ERR_INVALID_ARG;
  Levels lv;
  Box box;
  if (make_levels(L, log2T, base_res, growth, &lv) || make_box(aabb, &box)) return IA355_ERR_INVALID_ARG;
  if (S == 0) return IA355_OK;
  const int per_xcd = (L + kXcd - 1) / kXcd;
  // two levels per lane where an XCD serves several levels
  const int lv_lane = per_xcd >= 2 ? 2 : 1;
  const int ngroup = (per_xcd + lv_lane - 1) / lv_lane;
  // two samples per lane as well for frame-sized calls (more gathers in
  // flight per lane; at training-step sizes the halved lane count costs more)
  const int sp_lane = lv_lane == 2 && S >= kTwoSampleMin ? 2 : 1;
  // chunk slots per (XCD, level group); with a device count at most 1024 per
  // group, the blocks loop over the rest (blocks past the count exit at once)
  int64_t nslot = ceil_div(S, (int64_t)kFwdBlock * sp_lane);
  if (S_dev && nslot > 1024) nslot = 1024;
  const int64_t blocks = nslot * ngroup * kXcd;
  if (blocks > 0x7fffffffLL) return IA355_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  const unsigned g = (unsigned)blocks;
  const EncodeArgs ea{xc, bone, S, S_dev, ld, table, L, log2T, lv, box, feat, ngroup};
  if (table_dtype == IA355_F32 && feat_dtype == IA355_F32)
    launch_encode<float, float>(ea, lv_lane, sp_lane, g, s);
  else if (table_dtype == IA355_F32)
    launch_encode<float, __hip_bfloat16>(ea, lv_lane, sp_lane, g, s);
  else if (feat_dtype == IA355_F32)
    launch_encode<__half, float>(ea, lv_lane, sp_lane, g, s);
  else
    launch_encode<__half, __hip_bfloat16>(ea, lv_lane, sp_lane, g, s);
  return launch_status();
}

extern "C" size_t ia355_hashgrid_encode_bwd_workspace_size(int64_t S, int32_t L) {
  if (S < 0 || L <= 0) return 0;
  return align256(sizeof(float) * 3 * (size_t)L * (size_t)(S > 0 ? S : 1));
}

extern "C" int32_t ia355_hashgrid_encode_bwd(const float *grad_feat, const float *xc, const int16_t *bone, int64_t S,
                                             const int64_t *S_dev, int64_t ld, const void *table, int32_t table_dtype,
                                             int32_t L, int32_t F, int32_t log2T, double base_res, double growth,
                                             const float *aabb, float *grad_table, float *grad_xc, uint32_t flags,
                                             void *ws, size_t ws_bytes, ia355_stream_t stream) {
  if (S < 0 || ld < S || L <= 0 || L > 16 || F != 2 || log2T < 1 || log2T > 30) return IA355_ERR_INVALID_ARG;
  if (S > 0 && (!grad_feat || !xc)) return IA355_ERR_INVALID_ARG;
  if (grad_xc && !table) return IA355_ERR_INVALID_ARG;
  if (grad_xc && ((reinterpret_cast<uintptr_t>(table) & 15) != 0 || log2T < 2)) return IA355_ERR_INVALID_ARG;
  if (grad_xc && S > 0 && (!ws || ws_bytes < ia355_hashgrid_encode_bwd_workspace_size(S, L)))
    return IA355_ERR_WORKSPACE;
  if (table_dtype != IA355_F32 && table_dtype != IA355_F16) return IA355_ERR_INVALID_ARG;
  const uint32_t known = IA355_OVERWRITE | IA355_TABLE_COARSE | IA355_TABLE_FINE;
  if (flags & ~known) return IA355_ERR_INVALID_ARG;
  Levels lv;
  Box box;
  if (make_levels(L, log2T, base_res, growth, &lv) || make_box(aabb, &box)) return IA355_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  const bool dev = S_dev != nullptr;
  const int overwrite = (flags & IA355_OVERWRITE) != 0;
  // Run aggregation pays while a cell spans several ray steps (coarse dense
  // levels, which come first as the resolution grows with the level); finer
  // levels use the 16-lanes-per-item mapping.  The two groups touch disjoint
  // slices of the table, so a caller may run them on two streams.
  int ndense = 0;
  while (ndense < L && lv.dense[ndense] && lv.res[ndense] <= kAggMaxRes) ++ndense;
  const bool coarse = !(flags & IA355_TABLE_FINE) || (flags & IA355_TABLE_COARSE);
  const bool fine = !(flags & IA355_TABLE_COARSE) || (flags & IA355_TABLE_FINE);
  const int l0 = coarse ? 0 : ndense, l1 = fine ? L : ndense;
  const size_t level_floats = 2 * ((size_t)1 << log2T);
  if (grad_table && overwrite && l1 > l0) {
    const int32_t st = ia355_zero(grad_table + level_floats * l0, sizeof(float) * level_floats * (l1 - l0), stream);
    if (st != IA355_OK) return st;
  }
  if (grad_table && S > 0) {
    // The atomics do not return values, so a few waves per CU keep the
    // memory-side atomic units busy; bounded grids (grid-stride) leave CUs
    // to kernels on other streams (the position gradient and the IFT run
    // beside the table gradient).
    if (coarse && ndense > 0)
      table_grad_dense_kernel<<<stride_grid(ceil_div(S, kDgBlock) * ndense, true, kTgDenseMaxGrid), kDgBlock, 0, s>>>(
          grad_feat, xc, bone, S, S_dev, ld, ndense, log2T, lv, box, grad_table);
    if (fine && ndense < L)
      table_grad_kernel<<<stride_grid(ceil_div((int64_t)(L - ndense) * S * 16, kTgBlock), true, kTgMaxGrid), kTgBlock,
                          0, s>>>(grad_feat, xc, bone, S, S_dev, ld, ndense, L, log2T, lv, box, grad_table);
  }
  if (grad_xc && S > 0) {
    float *part = (float *)ws;
    const int per_xcd = (L + kXcd - 1) / kXcd;
    const int lv_lane = per_xcd >= 2 ? 2 : 1;
    const int ngroup = (per_xcd + lv_lane - 1) / lv_lane;
    int64_t nslot = ceil_div(S, kBwdBlock);
    if (dev && nslot > 1024) nslot = 1024;
    const int64_t blocks = nslot * ngroup * kXcd;
    if (blocks > 0x7fffffffLL) return IA355_ERR_INVALID_ARG;
    if (table_dtype == IA355_F32)
      launch_xgrad<float>(lv_lane, (unsigned)blocks, s, grad_feat, xc, bone, S, S_dev, ld, table, L, log2T, lv, box,
                          part, ngroup);
    else
      launch_xgrad<__half>(lv_lane, (unsigned)blocks, s, grad_feat, xc, bone, S, S_dev, ld, table, L, log2T, lv, box,
                           part, ngroup);
    xgrad_sum_kernel<<<stride_grid(ceil_div(S, kBwdBlock), dev, 1024), kBwdBlock, 0, s>>>(part, S, S_dev, L, ld,
                                                                                           grad_xc);
  }
  return launch_status();
}

extern "C" size_t ia355_hashgrid_table_grad_workspace_size(int64_t S, int32_t L, int32_t log2T) {
  BinGeom g;
  if (L <= 0 || L > 16 || !bin_geom(L, S, log2T, &g)) return 0;
  return bin_ws(g, nullptr).bytes;
}

extern "C" int32_t ia355_hashgrid_table_grad(const float *grad_feat, const float *xc, const int16_t *bone, int64_t S,
                                             const int64_t *S_dev, int64_t ld, int32_t L, int32_t F, int32_t log2T,
                                             double base_res, double growth, const float *aabb, float *grad_table,
                                             uint32_t flags, void *ws, size_t ws_bytes, ia355_stream_t stream) {
  const uint32_t known =
      IA355_OVERWRITE | IA355_TABLE_COARSE | IA355_TABLE_FINE | IA355_TABLE_PLAN | IA355_TABLE_REUSE_PLAN;
  if (flags & ~known) return IA355_ERR_INVALID_ARG;
  const bool plan_only = (flags & IA355_TABLE_PLAN) != 0, reuse = (flags & IA355_TABLE_REUSE_PLAN) != 0;
  if (plan_only && reuse) return IA355_ERR_INVALID_ARG;
  if (S < 0 || ld < S || L <= 0 || L > 16 || F != 2 || log2T < 2 || log2T > 30) return IA355_ERR_INVALID_ARG;
  if (S > 0 && !xc) return IA355_ERR_INVALID_ARG;
  if (!plan_only && (!grad_table || (S > 0 && !grad_feat))) return IA355_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(grad_table) & 15) != 0) return IA355_ERR_INVALID_ARG;  // float4 tile stores
  Levels lv;
  Box box;
  if (make_levels(L, log2T, base_res, growth, &lv) || make_box(aabb, &box)) return IA355_ERR_INVALID_ARG;
  BinGeom full;
  if (!bin_geom(L, S, log2T, &full)) return IA355_ERR_INVALID_ARG;
  if (!ws || ws_bytes < bin_ws(full, nullptr).bytes) return IA355_ERR_WORKSPACE;
  int ndense = 0;
  while (ndense < L && lv.dense[ndense] && lv.res[ndense] <= kAggMaxRes) ++ndense;
  const bool coarse = !(flags & IA355_TABLE_FINE) || (flags & IA355_TABLE_COARSE);
  const bool fine = !(flags & IA355_TABLE_COARSE) || (flags & IA355_TABLE_FINE);
  const int l0 = coarse ? 0 : ndense, l1 = fine ? L : ndense;
  if (l1 <= l0) return IA355_OK;
  const int overwrite = (flags & IA355_OVERWRITE) != 0;
  hipStream_t s = as_stream(stream);
  if (S == 0) {
    if (plan_only || !overwrite) return IA355_OK;
    const size_t level_floats = 2 * ((size_t)1 << log2T);
    return ia355_zero(grad_table + level_floats * l0, sizeof(float) * level_floats * (l1 - l0), stream);
  }
  BinGeom g;
  bin_geom(l1 - l0, S, log2T, &g);  // fewer levels than `full`: fits its workspace
  const BinWs w = bin_ws(g, ws);
  const size_t cnt_lds = sizeof(uint32_t) * (size_t)g.nbins;
  if (!reuse) {  // passes 1-3 read only the positions, the bones and the count
    bin_count_kernel<<<g.P, kBinBlock, cnt_lds, s>>>(xc, bone, S, S_dev, ld, l0, l1 - l0, log2T, g.tb, lv, box,
                                                     w.hist);
    bin_hist_scan_kernel<<<g.nchunk, 1024, 0, s>>>(w.hist, g.H, g.P, g.nbins, w.csum);
    bin_plan_kernel<<<1, 1024, 0, s>>>(w.hist, w.csum, g.nchunk, g.nbins, g.P, w.chunk_first, w.chunk_info);
    if (plan_only) return launch_status();
  }
  bin_scatter_kernel<<<g.P, kBinBlock, cnt_lds, s>>>(grad_feat, xc, bone, S, S_dev, ld, l0, l1 - l0, log2T, g.tb, lv,
                                                     box, w.hist, w.csum, w.rec, (uint32_t)g.rmax);
  if (overwrite)
    bin_clear_split_kernel<<<g.nbins < 1024 ? g.nbins : 1024, 256, 0, s>>>(w.chunk_first, g.nbins, l0, log2T, g.tb,
                                                                           grad_table);
  const unsigned acc_grid = (unsigned)(g.qmax < kAccMaxGrid ? g.qmax : kAccMaxGrid);
  bin_accum_kernel<<<acc_grid, kAccBlock, sizeof(unsigned long long) * 2 * ((size_t)1 << g.tb), s>>>(
      w.rec, w.chunk_first, w.chunk_info, g.nbins, (uint32_t)g.qmax, (uint32_t)g.rmax, l0, log2T, g.tb, overwrite,
      grad_table);
  return launch_status();
}
