// Small dense FP64 linear algebra for one workgroup (LDS-resident matrices, N <= 133).
#pragma once
#include "nyls_internal.h"

// In-place LU with partial pivoting of A (N x N, row stride lda, in LDS).
// piv[k] receives the row swapped into position k.  Returns (block-uniform) 1 when a
// zero pivot was met (elimination of that column skipped).  Uses red[0..2*NYLS_BLOCK/64).
__device__ inline int nyls_lu(double* A, int lda, int N, int* piv, double* red) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int singular = 0;
  for (int k = 0; k < N; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i < N; i += 64) {
        const double a = fabs(A[i * lda + k]);
        if (a > best) { best = a; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) piv[k] = bi;
    }
    __syncthreads();
    const int pr = piv[k];
    if (pr != k)
      for (int j = tid; j < N; j += NYLS_BLOCK) {
        const double t = A[k * lda + j];
        A[k * lda + j] = A[pr * lda + j];
        A[pr * lda + j] = t;
      }
    __syncthreads();
    const double pv = A[k * lda + k];
    if (pv == 0.0 || !(pv == pv)) {
      singular = 1;
      continue;
    }
    const double inv = 1.0 / pv;
    for (int i = k + 1 + tid; i < N; i += NYLS_BLOCK) A[i * lda + k] *= inv;
    __syncthreads();
    const int rows = N - k - 1, cols = N - k - 1;
    for (int e = tid; e < rows * cols; e += NYLS_BLOCK) {
      const int i = k + 1 + e / cols, j = k + 1 + e % cols;
      A[i * lda + j] -= A[i * lda + k] * A[k * lda + j];
    }
    __syncthreads();
  }
  (void)red;
  return singular;
}

// Solve A x = b with the factors of nyls_lu; b (length N, LDS) is overwritten by x.
__device__ inline void nyls_lu_solve(const double* A, int lda, int N, const int* piv, double* b) {
  const int tid = threadIdx.x;
  if (tid == 0)
    for (int k = 0; k < N; ++k) {
      const int pr = piv[k];
      if (pr != k) { const double t = b[k]; b[k] = b[pr]; b[pr] = t; }
    }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const double bk = b[k];
    for (int i = k + 1 + tid; i < N; i += NYLS_BLOCK) b[i] -= A[i * lda + k] * bk;
    __syncthreads();
  }
  for (int k = N - 1; k >= 0; --k) {
    if (tid == 0) b[k] /= A[k * lda + k];
    __syncthreads();
    const double xk = b[k];
    for (int i = tid; i < k; i += NYLS_BLOCK) b[i] -= A[i * lda + k] * xk;
    __syncthreads();
  }
}

// ---- single-wavefront variants (blockDim.x == 64): no barriers needed beyond LDS order ----

// Broadcast lane l's value (l uniform across the wave).
__device__ inline double nyls_rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double nyls_wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double nyls_wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Solve A x = b with LU factors (row stride lda, any address space); b in LDS.
__device__ inline void nyls_lu_solve_w(const double* A, int lda, int N, const int* piv, double* b) {
  const int lane = threadIdx.x;
  if (lane == 0)
    for (int k = 0; k < N; ++k) {
      const int pr = piv[k];
      if (pr != k) { const double t = b[k]; b[k] = b[pr]; b[pr] = t; }
    }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const double bk = b[k];
    for (int i = k + 1 + lane; i < N; i += 64) b[i] -= A[i * lda + k] * bk;
    __syncthreads();
  }
  for (int k = N - 1; k >= 0; --k) {
    if (lane == 0) b[k] /= A[k * lda + k];
    __syncthreads();
    const double xk = b[k];
    for (int i = lane; i < k; i += 64) b[i] -= A[i * lda + k] * xk;
    __syncthreads();
  }
}
