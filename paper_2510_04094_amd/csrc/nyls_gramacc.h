// Register-blocked FP64 Gram accumulation over LDS tiles, for one workgroup:
//   G += sum_rows w_row * q_row q_row^T   (q_row: gp columns, gp a multiple of 4)
// Each thread owns 4 x 4 blocks of the upper triangle; when there are few blocks the
// rows are split over thread groups, and group partials are summed in a fixed order.
#pragma once
#include "nyls_internal.h"

namespace nyls_gram {

constexpr int MAXB = 3;  // 4x4 blocks per thread (gp <= 132 -> at most 561 blocks)

struct Acc {
  int nb, nblk, ngrp, grp, nmine;
  int blk[MAXB], bi[MAXB], bj[MAXB];
  double c[MAXB][16];
};

__device__ inline void setup(Acc& A, int gp) {
  const int tid = threadIdx.x;
  A.nb = gp >> 2;
  A.nblk = A.nb * (A.nb + 1) / 2;
  A.ngrp = A.nblk >= NYLS_BLOCK ? 1 : NYLS_BLOCK / A.nblk;
  A.grp = A.ngrp > 1 ? tid / A.nblk : 0;
  A.nmine = 0;
#pragma unroll
  for (int k = 0; k < MAXB; ++k) { A.blk[k] = 0; A.bi[k] = 0; A.bj[k] = 0; }
  if (A.ngrp > 1) {
    if (A.grp < A.ngrp) { A.blk[0] = tid - A.grp * A.nblk; A.nmine = 1; }
  } else {
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = tid + k * NYLS_BLOCK;
      if (b < A.nblk) { A.blk[k] = b; A.nmine = k + 1; }
    }
  }
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    if (k < A.nmine) {
      int b = A.blk[k], row = 0;
      while (b >= A.nb - row) { b -= A.nb - row; ++row; }
      A.bi[k] = row;
      A.bj[k] = row + b;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) A.c[k][e] = 0.0;
  }
}

// Accumulate rows 0..nrows-1 of Q (row stride ldq) with weights w (nullptr: 1).
__device__ inline void accumulate(Acc& A, const double* Q, int ldq, const double* w, int nrows) {
  for (int row = A.grp; row < nrows; row += A.ngrp) {
    const double* q = Q + row * ldq;
    const double wr = w ? w[row] : 1.0;
    if (wr == 0.0) continue;
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      if (k >= A.nmine) break;
      const double* ra = q + 4 * A.bi[k];
      const double* rb = q + 4 * A.bj[k];
      const double a0 = wr * ra[0], a1 = wr * ra[1], a2 = wr * ra[2], a3 = wr * ra[3];
      const double b0 = rb[0], b1 = rb[1], b2 = rb[2], b3 = rb[3];
      double* c = A.c[k];
      c[0] += a0 * b0; c[1] += a0 * b1; c[2] += a0 * b2; c[3] += a0 * b3;
      c[4] += a1 * b0; c[5] += a1 * b1; c[6] += a1 * b2; c[7] += a1 * b3;
      c[8] += a2 * b0; c[9] += a2 * b1; c[10] += a2 * b2; c[11] += a2 * b3;
      c[12] += a3 * b0; c[13] += a3 * b1; c[14] += a3 * b2; c[15] += a3 * b3;
    }
  }
}

// Reduce the groups into red (LDS, >= nblk*16 doubles) and write the full symmetric
// g x g result to out (row stride ldo).  Ends with a barrier.
__device__ inline void finish(Acc& A, double* red, double* out, int g, int ldo) {
  const int tid = threadIdx.x;
  __syncthreads();
  for (int gi = 0; gi < A.ngrp; ++gi) {
    if (A.grp == gi) {
#pragma unroll
      for (int k = 0; k < MAXB; ++k) {
        if (k >= A.nmine) break;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          double* dst = red + A.blk[k] * 16 + e;
          *dst = (gi == 0) ? A.c[k][e] : *dst + A.c[k][e];
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < g * g; e += NYLS_BLOCK) {
    int a = e / g, b = e - a * g;
    if (a > b) { const int t = a; a = b; b = t; }
    const int ia = a >> 2, ib = b >> 2;
    const int blk = ia * A.nb - ia * (ia - 1) / 2 + (ib - ia);
    out[(e / g) * ldo + (e % g)] = red[blk * 16 + (a & 3) * 4 + (b & 3)];
  }
  __syncthreads();
}

__host__ __device__ inline int red_doubles(int gp) {
  const int nb = gp >> 2;
  return nb * (nb + 1) / 2 * 16;
}

}  // namespace nyls_gram
