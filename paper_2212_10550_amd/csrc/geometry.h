// Small 3x3 / rigid-transform helpers shared by the deform and root
// initialiser kernels (internal).
#pragma once
#include "common.h"

namespace ia355 {

// Inverse by the adjugate; returns the determinant.
__device__ __forceinline__ float inv3(const float A[3][3], float Ai[3][3]) {
  const float c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const float c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const float c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const float det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  const float id = 1.0f / det;
  Ai[0][0] = c00 * id;
  Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
  Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
  Ai[1][0] = c01 * id;
  Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
  Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
  Ai[2][0] = c02 * id;
  Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
  Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
  return det;
}

// Per-bone inverse transforms [M^-1 | -M^-1 t] (12 floats) and a
// non-singular flag, staged into LDS by the first threads of the block.
__device__ __forceinline__ void stage_bone_inverses(const float *__restrict__ B, int nb, float *sBinv, int *sBok) {
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    float M[3][3], Mi[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[i][j] = B[12 * b + 4 * i + j];
    const float det = inv3(M, Mi);
    sBok[b] = fabsf(det) >= 1e-12f;
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) sBinv[12 * b + 4 * i + j] = Mi[i][j];
      sBinv[12 * b + 4 * i + 3] = -(Mi[i][0] * B[12 * b + 3] + Mi[i][1] * B[12 * b + 7] + Mi[i][2] * B[12 * b + 11]);
    }
  }
}

}  // namespace ia355
