// Slice binning: the shared part of the scatter-add kernels that replace
// global FP32 atomics by LDS accumulation.
//
// A scatter target (a hash level's table, the skinning grid's moment array)
// is cut into slices that fit one workgroup's LDS.  A bin kernel (specific
// to each target) writes, for each chunk of samples, its records grouped by
// slice and the per-chunk slice offsets offs[t][chunk][0..nsl] (exclusive
// prefix, offs[..][nsl] = records of the chunk).  The kernels here turn the
// offsets into a work plan: records per slice, and a flat list of items
// (table, slice, group, groups) where a slice with many records is split
// into groups of chunks.  The accumulate kernel (again target specific)
// sums one item's records in LDS and adds the slice to the target:
// plain read-modify-write when the slice has one group, atomics otherwise.
#pragma once
#include "common.h"

namespace ia355 {
namespace {

constexpr int kMaxGroups = 64;
constexpr int kPlanBlock = 1024;

// Exclusive scan of one int per thread over a block of NW waves; *total gets
// the block sum.  sh: NW ints of shared memory.  Every thread must call it.
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int *total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int inc = wave_incl_scan(v);
  if (lane == kWave - 1) sh[wid] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int t = sh[i];
    base += i < wid ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// Records per slice, summed over the chunks: one thread per (table, slice).
__global__ void slice_total_kernel(const int32_t *__restrict__ offs, int ntab, int64_t chunks, int nsl,
                                   int32_t *__restrict__ tot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ntab * nsl) return;
  const int t = (int)(i / nsl), s = (int)(i % nsl);
  int acc = 0;
  for (int64_t c = 0; c < chunks; ++c) {
    const int32_t *row = offs + ((int64_t)t * chunks + c) * (nsl + 1);
    acc += row[s + 1] - row[s];
  }
  tot[i] = acc;
}

__device__ __forceinline__ int slice_groups(int tot, int64_t chunks, int rec_per_group) {
  if (tot == 0) return 0;
  int g = (tot + rec_per_group - 1) / rec_per_group;
  if (g > kMaxGroups) g = kMaxGroups;
  if (g > chunks) g = (int)chunks;
  return g;
}

// One workgroup of kPlanBlock threads: groups per slice, their prefix, and
// the flat item list (table, slice, group, groups).  Item count is at most
// ntab * nsl + total_records / rec_per_group.
__global__ void __launch_bounds__(kPlanBlock) plan_kernel(const int32_t *__restrict__ tot, int ntab, int64_t chunks,
                                                         int nsl, int rec_per_group, int4 *__restrict__ items,
                                                         int32_t *__restrict__ n_items) {
  __shared__ int red[kPlanBlock / kWave];
  const int nall = ntab * nsl;
  const int per = (nall + kPlanBlock - 1) / kPlanBlock;
  const int i0 = threadIdx.x * per;
  int mine = 0;
  for (int i = 0; i < per; ++i)
    if (i0 + i < nall) mine += slice_groups(tot[i0 + i], chunks, rec_per_group);
  int total;
  int base = block_excl_scan<kPlanBlock / kWave>(mine, red, &total);
  for (int i = 0; i < per; ++i)
    if (i0 + i < nall) {
      const int G = slice_groups(tot[i0 + i], chunks, rec_per_group);
      for (int g = 0; g < G; ++g) items[base++] = make_int4((i0 + i) / nsl, (i0 + i) % nsl, g, G);
    }
  if (threadIdx.x == 0) *n_items = total;
}

// Chunk range [c0, c1) of group g of G over `chunks` chunks (non-empty when
// G <= chunks, which slice_groups guarantees).
__device__ __forceinline__ void group_chunks(int g, int G, int64_t chunks, int64_t *c0, int64_t *c1) {
  *c0 = (int64_t)g * chunks / G;
  *c1 = (int64_t)(g + 1) * chunks / G;
}

// Maps record r of a batch of nb chunks (starts sp[], run bases sb[]) to its
// index in the record array: the last chunk whose run starts at or before r.
__device__ __forceinline__ int64_t batch_record(int r, int nb, const int *sp, const int64_t *sb) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sp[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return sb[lo] + (r - sp[lo]);
}

}  // namespace
}  // namespace ia355
