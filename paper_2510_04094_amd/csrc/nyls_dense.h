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

// Value of a double from another lane of the same row of 16 (DPP control CTRL, e.g. 0x120 + n
// = row_ror:n), moved as two 32-bit halves and reassembled bit for bit.  (Passing a double
// straight to the DPP builtin inside an overloaded call such as fmax lets the compiler read
// the moved bits as an integer value.)
template <int CTRL>
__device__ inline double nyls_dpp_f64(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wavefront, bitwise equal in every lane: rotations by 8, 4, 2 and 1 within each
// row of 16 lanes (DPP row_ror; the two lanes of every exchange add the same two values),
// then the lane-swap exchanges across rows.  No LDS round trip.
__device__ inline double nyls_wave_sum_dpp(double v) {
  v += nyls_dpp_f64<0x128>(v);
  v += nyls_dpp_f64<0x124>(v);
  v += nyls_dpp_f64<0x122>(v);
  v += nyls_dpp_f64<0x121>(v);
  double a, b;
  nyls_pair_xor16(v, a, b);
  nyls_pair_xor32(a + b, a, b);
  return a + b;
}

// Maximum over the wavefront (NaN entries ignored unless all are NaN), equal in every lane.
__device__ inline double nyls_wave_max_dpp(double v) {
  v = fmax(v, nyls_dpp_f64<0x128>(v));
  v = fmax(v, nyls_dpp_f64<0x124>(v));
  v = fmax(v, nyls_dpp_f64<0x122>(v));
  v = fmax(v, nyls_dpp_f64<0x121>(v));
  double a, b;
  nyls_pair_xor16(v, a, b);
  nyls_pair_xor32(fmax(a, b), a, b);
  return fmax(a, b);
}

// Row-per-lane updates in LDS over columns j0 <= j < m, in unguarded chunks of 8, then 4,
// then single columns: a chunk's loads (the lane's own row and the broadcast vectors) are
// all issued before its stores, so each chunk waits for LDS once instead of once per column.
// sum_j r[j] a[j] (two partial sums)
template <int C>
__device__ inline void nyls_dot_chunk(const double* r, const double* a, int j, double& s0,
                                     double& s1) {
  double x[C], y[C];
#pragma unroll
  for (int u = 0; u < C; ++u) { x[u] = r[j + u]; y[u] = a[j + u]; }
#pragma unroll
  for (int u = 0; u < C; ++u) {
    if (u & 1) s1 = fma(x[u], y[u], s1);
    else s0 = fma(x[u], y[u], s0);
  }
}
__device__ inline double nyls_row_dot(const double* r, const double* a, int j0, int m) {
  double s0 = 0.0, s1 = 0.0;
  int j = j0;
  for (; j + 8 <= m; j += 8) nyls_dot_chunk<8>(r, a, j, s0, s1);
  if (j + 4 <= m) { nyls_dot_chunk<4>(r, a, j, s0, s1); j += 4; }
  for (; j < m; ++j) s0 = fma(r[j], a[j], s0);
  return s0 + s1;
}
// r[j] -= v a[j] + w b[j]
template <int C>
__device__ inline void nyls_rank2_chunk(double* r, double v, const double* a, double w,
                                       const double* b, int j) {
  double x[C], y[C], z[C];
#pragma unroll
  for (int u = 0; u < C; ++u) { x[u] = r[j + u]; y[u] = a[j + u]; z[u] = b[j + u]; }
#pragma unroll
  for (int u = 0; u < C; ++u) r[j + u] = x[u] - (v * y[u] + w * z[u]);
}
__device__ inline void nyls_row_rank2(double* r, double v, const double* a, double w,
                                     const double* b, int j0, int m) {
  int j = j0;
  for (; j + 8 <= m; j += 8) nyls_rank2_chunk<8>(r, v, a, w, b, j);
  if (j + 4 <= m) { nyls_rank2_chunk<4>(r, v, a, w, b, j); j += 4; }
  for (; j < m; ++j) r[j] -= v * a[j] + w * b[j];
}
// r[j] -= v a[j]
template <int C>
__device__ inline void nyls_rank1_chunk(double* r, double v, const double* a, int j) {
  double x[C], y[C];
#pragma unroll
  for (int u = 0; u < C; ++u) { x[u] = r[j + u]; y[u] = a[j + u]; }
#pragma unroll
  for (int u = 0; u < C; ++u) r[j + u] = x[u] - v * y[u];
}
__device__ inline void nyls_row_rank1(double* r, double v, const double* a, int j0, int m) {
  int j = j0;
  for (; j + 8 <= m; j += 8) nyls_rank1_chunk<8>(r, v, a, j);
  if (j + 4 <= m) { nyls_rank1_chunk<4>(r, v, a, j); j += 4; }
  for (; j < m; ++j) r[j] -= v * a[j];
}
// sum_i a[i] Q[i][col] over rows j0 <= i < m (column access, stride lda)
template <int C>
__device__ inline void nyls_col_chunk(const double* a, const double* q, int lda, int i, double& s0,
                                     double& s1) {
  double x[C], y[C];
#pragma unroll
  for (int u = 0; u < C; ++u) { x[u] = a[i + u]; y[u] = q[(i + u) * lda]; }
#pragma unroll
  for (int u = 0; u < C; ++u) {
    if (u & 1) s1 = fma(x[u], y[u], s1);
    else s0 = fma(x[u], y[u], s0);
  }
}
__device__ inline double nyls_col_dot(const double* a, const double* q, int lda, int j0, int m) {
  double s0 = 0.0, s1 = 0.0;
  int i = j0;
  for (; i + 8 <= m; i += 8) nyls_col_chunk<8>(a, q, lda, i, s0, s1);
  if (i + 4 <= m) { nyls_col_chunk<4>(a, q, lda, i, s0, s1); i += 4; }
  for (; i < m; ++i) s0 = fma(a[i], q[i * lda], s0);
  return s0 + s1;
}


// One-wavefront LU with partial pivoting of the N x N matrix A (N <= 64, row stride lda, in
// LDS; all 64 lanes of the wavefront call it), followed by the solve of A x = b (b in LDS,
// overwritten by x).  Lane i owns row i and rows are never moved: the row chosen as pivot
// at step k (largest |a_ik| among the rows not yet chosen, lowest index on ties) is recorded
// in perm[k], and piv[k] receives the equivalent row interchange (the position swapped
// into position k), so that rows perm[0..N) of A, in that order, are the factors nyls_lu
// leaves in place.  The elimination arithmetic is nyls_lu's: l_i = a_ik (1 / a_kk), then
// a_ij - l_i a_kj.  The pivot search is a wave maximum and a ballot, the interchange
// sequence is tracked in registers, and the row updates run in chunks, so no step waits on
// a workgroup barrier.  Returns (wave-uniform) 1 when a zero or non-finite pivot was met
// (that column's elimination is skipped).
__device__ inline int nyls_lu_wave(double* A, int lda, int N, double* b, int* piv, int* perm) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < N;
  double* Ar = A + (row ? lane : 0) * lda;  // lanes past N only read row 0
  int pos = row ? -1 : 64;  // step at which this row became the pivot (-1: not yet)
  int cur = lane;           // original row now at position `lane` of the interchanged order
  int singular = 0;
  double a = Ar[0];         // this row's entry in the current column
  for (int k = 0; k < N; ++k) {
    const bool cand = pos < 0;
    const double mag = cand ? fabs(a) : -1.0;
    const double mx = nyls_wave_max_dpp(mag);
    unsigned long long bal = __ballot(cand && mag == mx);
    if (bal == 0) bal = __ballot(cand);  // every candidate is NaN
    const int p = __ffsll((long long)bal) - 1;
    const int q = __ffsll((long long)__ballot(cur == p)) - 1;  // >= k
    const int ck = __builtin_amdgcn_readlane(cur, k);
    if (lane == q) cur = ck;
    if (lane == k) cur = p;
    if (lane == 0) {
      piv[k] = q;
      perm[k] = p;
    }
    if (lane == p) pos = k;
    const double pv = nyls_rdlane(a, p);
    if (pv == 0.0 || !(pv == pv)) {
      singular = 1;
    } else {
      const double inv = 1.0 / pv;
      if (cand && lane != p) {
        const double l = a * inv;
        Ar[k] = l;
        nyls_row_rank1(Ar, l, A + p * lda, k + 1, N);
      }
    }
    nyls_wave_lds_sync();
    a = k + 1 < N ? Ar[k + 1] : 0.0;
  }
  // forward substitution, column by column: y_t sits in the row chosen at step t
  const int pl = row ? perm[lane] : 0;  // pivot row of step `lane`
  double c = row ? b[lane] : 0.0;
  for (int t = 0; t < N; ++t) {
    const double yt = nyls_rdlane(c, __builtin_amdgcn_readlane(pl, t));
    if (row && pos > t) c -= Ar[t] * yt;
  }
  // back substitution: x_t = y_t / u_tt, then the rows of earlier steps subtract it
  const double dg = row ? Ar[pos] : 1.0;
  for (int t = N - 1; t >= 0; --t) {
    const int pt = __builtin_amdgcn_readlane(pl, t);
    const double xt = nyls_rdlane(c, pt) / nyls_rdlane(dg, pt);
    if (row && pos < t) c -= Ar[t] * xt;
    if (lane == pt) c = xt;
  }
  if (row) b[pos] = c;
  nyls_wave_lds_sync();
  return singular;
}

// Solve A x = b with the factors nyls_lu / nyls_lu_wave leave (rows in pivot order, row
// stride N, any address space; piv: the row interchanges, any address space), N <= 64, by
// one wavefront: lane k holds entry k.  The interchanges are composed into a permutation in
// registers and b (LDS, overwritten by x) is gathered once; each substitution step
// broadcasts the solved entry with a lane read, and every lane walks its own factor row in
// chunks of eight entries loaded together (prefetching the next chunk as well measured no
// faster and costs 16 VGPRs).  Same operations in the same order as nyls_lu_solve_w.
__device__ inline void nyls_lu_solve_wave(const double* A, int N, const int* piv, double* b) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < N;
  const double* Ar = A + (size_t)(row ? lane : 0) * N;  // lanes past N read row 0 only
  const int pv = row ? piv[lane] : lane;
  int cur = lane;  // the entry of b that ends up at position `lane`
  for (int k = 0; k < N; ++k) {
    const int q = __builtin_amdgcn_readlane(pv, k);
    const int ck = __builtin_amdgcn_readlane(cur, k), cq = __builtin_amdgcn_readlane(cur, q);
    if (lane == k) cur = cq;
    if (lane == q) cur = ck;
  }
  double c = row ? b[cur] : 0.0;
  double a8[8];
  auto load8 = [&](int t0, double (&v)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = Ar[t0 + u < N ? t0 + u : N - 1];
  };
  // forward: unit lower factor
  for (int t0 = 0; t0 < N; t0 += 8) {
    load8(t0, a8);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u;
      if (t < N) {
        const double yt = nyls_rdlane(c, t);
        if (row && lane > t) c -= a8[u] * yt;
      }
    }
  }
  // back substitution: x_t = y_t / u_tt, then the entries above subtract it
  const double dg = row ? Ar[lane] : 1.0;
  const int tl = (N - 1) & ~7;  // first column of the last chunk
  for (int t0 = tl; t0 >= 0; t0 -= 8) {
    load8(t0, a8);
#pragma unroll
    for (int u = 7; u >= 0; --u) {
      const int t = t0 + u;
      if (t < N) {
        const double xt = nyls_rdlane(c, t) / nyls_rdlane(dg, t);
        if (row && lane < t) c -= a8[u] * xt;
        if (lane == t) c = xt;
      }
    }
  }
  if (row) b[lane] = c;
  nyls_wave_lds_sync();
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
