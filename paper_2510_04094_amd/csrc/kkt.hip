// Lemma 1 KKT system in feature coordinates (Sec. 3.1), one workgroup per instance:
//
//   [ I + gamma W^T S W   gamma W^T u   H ] [omega]   [gamma W^T z]
//   [ gamma u^T W         gamma s_cc    d ] [  b  ] = [gamma s_cr ]
//   [ H^T                 d^T           0 ] [ lam ]   [     v     ]
//
// from the Gram S~ = [[S, u, z], [u^T, s_cc, s_cr], ...] of the Gram kernel (kernel space:
// W^T S W; eigenbasis, rows rotated by U^T: Lambda^{-1/2} S Lambda^{-1/2}), W from the
// basis kernel, condition rows h_j = W^T k^(d_j)(t_{i_j}) and delta_j = [d_j = 0].
// Directions dropped by the eigenvalue cut-off get identity rows (their omega is 0).  The
// system is optionally written out, then LU-factorised with partial pivoting in LDS; the
// factors stay in the workspace for refinement and the adjoint, and the solution x and
// alpha = W omega are stored.
//
// Kernel-space Gram with m + 2 <= 128: the whole (omega, b) block and the right-hand side come
// from one product K~ = W~^T S~ W~ on the matrix cores, with W~ = diag(W[:, :r], 1, 1)
// zero-padded to 16 NT x 16 NT (NT = 4 or 8 column blocks): K~[:m+1, :m+1] is the (omega, b)
// block before scaling by gamma and K~[:m+1, m+1] the right-hand side.  Wave J of the
// workgroup takes column blocks J, J + 4: it forms T = S~ W~[:, 16J:16J+16] with
// v_mfma_f64_16x16x4f64 and keeps it in its accumulators, which are then exactly the B
// operands of W~^T T (register v of tile I holds rows 16 I + 4 v + lane / 16), so T never
// leaves the registers.
#include "nyls_dense.h"

namespace {

typedef double nyls_d4 __attribute__((ext_vector_type(4)));

// W~[s][k] of the padded transform (see above).
__device__ inline double wext(const double* W, int m, int r, int g, int s, int k) {
  if (s < m) return (k < r) ? W[s * m + k] : 0.0;
  return (s == k && s < g) ? 1.0 : 0.0;
}

// Writes gamma K~ (+ identity on the landmark diagonal) into K[a][b], a, b <= m, and
// gamma K~[a][m + 1] into rhs[a], a <= m, for g = m + 2 <= 16 NT.  256 threads; wave J takes
// column blocks J, J + 4, ... in turn (NT <= 8).
template <int NT, class Out>
__device__ inline void kkt_transform_mfma(const double* __restrict__ S, const double* __restrict__ W,
                                          int m, int r, double gam, Out out) {
  const int g = m + 2;
  const int lane = threadIdx.x & 63;
  const int row = lane & 15, kq = lane >> 4;
  // NT <= 4: one column block per wavefront (no loop, which keeps k_kkt's registers low)
  const int J0 = threadIdx.x >> 6, JS = NT <= NYLS_BLOCK / 64 ? NT : NYLS_BLOCK / 64;
  for (int J = J0; J < NT && 16 * J < g; J += JS) {
    nyls_d4 t[NT];
#pragma unroll
    for (int I = 0; I < NT; ++I) t[I] = nyls_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) {
      const int s = 4 * ks + kq;
      const double bop = wext(W, m, r, g, s, 16 * J + row);
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        const int a = 16 * I + row;
        const double aop = (a < g && s < g) ? S[a * g + s] : 0.0;
        t[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, t[I], 0, 0, 0);
      }
    }
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      if (16 * I >= g) break;
      nyls_d4 k4 = nyls_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4 * NT; ++ks) {
        const double aop = wext(W, m, r, g, 4 * ks + kq, 16 * I + row);
        k4 = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, t[ks >> 2][ks & 3], k4, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + 4 * v + kq, b = 16 * J + row;
        if (a <= m && b <= m + 1) out(a, b, gam * k4[v] + ((a == b && a < m) ? 1.0 : 0.0));
      }
    }
  }
}

// LU with partial pivoting of the N x N row-major matrix A in global memory (lda = N) by the
// 256 threads of a workgroup, for the wide bases: thread j updates columns j, j + 256, ...
// (coalesced across the threads), and each column loop issues eight loads before its stores.
// The pivot is the first largest |entry| of the column, the multipliers are kept in LDS
// (lcol, N doubles); pivots and arithmetic are those of nyls_lu.  redv / redi: four doubles
// and four ints of LDS.
__device__ inline int lu_global(double* A, int N, int* piv, double* lcol, double* redv, int* redi) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int singular = 0;
  for (int k = 0; k < N; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < N; i += NYLS_BLOCK) {
      const double a = fabs(A[i * N + k]);
      if (a > best) { best = a; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) {
      redv[wave] = best;
      redi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = redv[0];
      int ix = redi[0];
      for (int w = 1; w < NYLS_BLOCK / 64; ++w)
        if (redv[w] > b || (redv[w] == b && redi[w] < ix)) { b = redv[w]; ix = redi[w]; }
      piv[k] = ix;
    }
    __syncthreads();
    const int pr = piv[k];
    if (pr != k)
      for (int j = tid; j < N; j += NYLS_BLOCK) {
        const double t = A[k * N + j];
        A[k * N + j] = A[pr * N + j];
        A[pr * N + j] = t;
      }
    __syncthreads();
    const double pv = A[k * N + k];
    if (pv == 0.0 || !(pv == pv)) {
      singular = 1;
      continue;
    }
    const double inv = 1.0 / pv;
    for (int i = k + 1 + tid; i < N; i += NYLS_BLOCK) {
      const double l = A[i * N + k] * inv;
      A[i * N + k] = l;
      lcol[i] = l;
    }
    __syncthreads();
    for (int j = k + 1 + tid; j < N; j += NYLS_BLOCK) {
      const double u = A[k * N + j];
      int i = k + 1;
      for (; i + 8 <= N; i += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = A[(i + q) * N + j];
#pragma unroll
        for (int q = 0; q < 8; ++q) A[(i + q) * N + j] = v[q] - lcol[i + q] * u;
      }
      for (; i < N; ++i) A[i * N + j] -= lcol[i] * u;
    }
    __syncthreads();
  }
  return singular;
}

__device__ inline int instance_of(const int32_t* order) {
  return order ? order[blockIdx.x] : (int)blockIdx.x;
}

// gamma K~ (+ identity) of the kernel-space instances with 64 < m + 2 <= 130 (nine column
// blocks cover m <= 128), into the instance's T scratch as rows a <= m, columns b <= m + 1
// (row stride m + 2), for k_kkt.  A kernel of its own: its nine accumulator tiles per
// wavefront would cost k_kkt's other instances their occupancy.
__global__ __launch_bounds__(NYLS_BLOCK) void k_kkt_mfma_wide(const nyls_desc* __restrict__ desc,
                                                         const int32_t* __restrict__ order,
                                                         double* __restrict__ wsbase, int single,
                                                         int eigbasis, int only) {
  const int inst = single >= 0 ? single : instance_of(order);
  const nyls_desc& d = desc[inst];
  const int m = d.m, g = m + 2;
  if (g <= 64 || m > NYLS_NARROW_MAX_M) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  if (only && !((int)ws[L.info + 1] & only)) return;
  (void)eigbasis;  // (the FP32 eigenbasis Gram covers m + 2 <= 64 only)
  if (ws[L.info + 4] != 0.0) return;
  const int r = (int)ws[L.info + 0];
  double* T = ws + L.tmp;
  kkt_transform_mfma<(NYLS_NARROW_MAX_M + 2 + 15) / 16>(ws + L.gram, ws + L.W, m, r, d.gamma,
                        [&](int a, int b, double v) { T[a * g + b] = v; });
}

// The same product for the wide bases (kernel-space Gram), in two element-parallel steps
// over the instance's workspace: step 0 forms P = S~ W~ (g x g, in the rotation-log region,
// free after the eigensolver), step 1 gamma W~^T P (+ identity) into T.  Grid (instance,
// element tiles of 256).
__global__ __launch_bounds__(NYLS_BLOCK) void k_kkt_wide_transform(const nyls_desc* __restrict__ desc,
                                                              double* __restrict__ wsbase, int step) {
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m, g = m + 2;
  if (m <= NYLS_NARROW_MAX_M) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  if (ws[L.info + 4] != 0.0) return;  // eigenbasis Gram: k_kkt scales it directly
  const int e = (int)blockIdx.y * NYLS_BLOCK + (int)threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double* W = ws + L.W;
  double* P = ws + L.log;
  if (step == 0) {
    if (e >= g * g) return;
    const int a = e / g, k = e - a * g;
    const double* S = ws + L.gram;
    double v = 0.0;
    if (k >= m) {
      v = S[a * g + k];
    } else if (k < r) {
      for (int s = 0; s < m; ++s) v += S[a * g + s] * W[s * m + k];
    }
    P[e] = v;
  } else {
    if (e >= (m + 1) * g) return;
    const int a = e / g, b = e - a * g;
    double v = 0.0;
    if (a == m) {
      v = P[m * g + b];
    } else if (a < r) {
      for (int s = 0; s < m; ++s) v += W[s * m + a] * P[s * g + b];
    }
    ws[L.tmp + e] = d.gamma * v + ((a == b && a < m) ? 1.0 : 0.0);
  }
}

// WIDE = false: bases up to m = glo, the matrix in LDS; WIDE = true: larger bases, the matrix
// assembled and factored in place in the workspace (glo = NYLS_NARROW_MAX_M: only the systems
// that would not fit the LDS; glo = 64 for batches with many 64 < m <= 128 instances, whose
// 85 KB of LDS would hold one workgroup per CU).  Each instantiation skips the other's
// instances.
template <bool WIDE>
__global__ __launch_bounds__(NYLS_BLOCK) void k_kkt(const nyls_desc* __restrict__ desc,
                                                    const int32_t* __restrict__ order,
                                                    double* __restrict__ wsbase,
                                                    double* __restrict__ kkt_out,
                                                    double* __restrict__ rhs_out, int kn,
                                                    int factor, int single, int eigbasis,
                                                    int only, int glo) {
  extern __shared__ double sm[];
  const int inst = single >= 0 ? single : instance_of(order);
  const nyls_desc& d = desc[inst];
  if ((d.m > glo) != WIDE) return;
  if (only && !((int)wsbase[d.ws + nyls_layout(d.m, d.p, 0).info + 1] & only)) return;
  const int m = d.m, p = d.p;
  // in LDS with an odd row stride (row-per-lane access is conflict-free), the factors copied
  // out afterwards; wide bases in place
  constexpr bool wide = WIDE;
  const int g = m + 2, N = m + 1 + p, lda = wide ? N : (N | 1);
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* S = ws + L.gram;
  const double* T = ws + L.tmp;  // gamma K~ from k_kkt_mfma_wide (m + 2 > 64)
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma;

  double* K = wide ? ws + L.lu : sm;     // [N][lda]
  double* rhs = wide ? sm : K + N * lda;  // [N]
  double* kc = rhs + (N + 1);           // [p][m] kernel-derivative vectors of the conditions
  double* red = kc + NYLS_MAX_P * NYLS_MAX_M;
  int* piv = reinterpret_cast<int*>(red + 16);  // [N + 1]
  int* perm = piv + (N + 1);                     // [N + 1]

  // Kernel-space Gram: the (omega, b) block and its rhs are W~^T S~ W~ from the matrix cores
  // (here for g <= 64, from k_kkt_mfma_wide in the T scratch otherwise); with the eigenbasis
  // Gram (rows rotated by U^T) the transform is the diagonal Lambda^{-1/2}.
  const double* lamv = ws + L.lam;
  // per-instance choice of the FP64 Gram (eigbasis: the FP32 Gram of NYLS_MIXED, which
  // bases with m + 2 > 64 do not take)
  if (!eigbasis || g > 64) eigbasis = ws[L.info + 4] != 0.0 ? 1 : 0;
  const bool mx = !eigbasis;
  if (mx && g <= 64)
    kkt_transform_mfma<4>(S, W, m, r, gam, [&](int a, int b, double v) {
      if (b <= m) K[a * lda + b] = v;
      else rhs[a] = v;
    });
  else if (mx)
    for (int e = tid; e < (m + 1) * (m + 2); e += NYLS_BLOCK) {
      const int a = e / (m + 2), b = e - a * (m + 2);
      if (b <= m) K[a * lda + b] = T[a * g + b];
      else rhs[a] = T[a * g + b];
    }
  // condition kernel vectors k^(d_j)(t_{i_j})
  const double inv_sigma = 1.0 / d.sigma;
  for (int e = tid; e < p * m; e += NYLS_BLOCK) {
    const int j = e / m, s = e - j * m;
    const double z = (nyls_grid_t(d, d.cond_i[j]) - nyls_grid_t(d, d.lidx[s])) * inv_sigma;
    double kd[NYLS_MAX_P + 1];
    nyls_kderiv(z, inv_sigma, kd);
    kc[j * NYLS_MAX_M + s] = nyls_pick(kd, d.cond_d[j]);
  }
  __syncthreads();
  // feature-space condition rows h_j = W^T k^(d_j)(t_{i_j}), each entry formed once and
  // written to the workspace for the later passes, then read back into kc in place of the
  // kernel vectors (once every thread has finished reading those)
  for (int e = tid; e < p * m; e += NYLS_BLOCK) {
    const int j = e / m, k = e - j * m;
    double hv = 0.0;
    if (k < r)
      for (int s = 0; s < m; ++s) hv += W[s * m + k] * kc[j * NYLS_MAX_M + s];
    ws[L.H + e] = hv;
  }
  __syncthreads();
  for (int e = tid; e < p * m; e += NYLS_BLOCK) kc[(e / m) * NYLS_MAX_M + e % m] = ws[L.H + e];
  __syncthreads();
  for (int e = tid; e < N * N; e += NYLS_BLOCK) {
    const int a = e / N, b = e - a * N;
    if (mx && a <= m && b <= m) continue;
    double val = 0.0;
    if (a < m && b < m) {
      if (a < r && b < r) {  // eigenbasis Gram (the kernel-space block came from the MFMA product)
        val = gam * (S[a * g + b] / sqrt(lamv[a] * lamv[b])) + (a == b ? 1.0 : 0.0);
      } else {
        val = (a == b) ? 1.0 : 0.0;
      }
    } else if (a < m || b < m) {
      const int k = a < m ? a : b, o = a < m ? b : a;  // k: feature index, o: b or lambda
      if (k < r) {
        if (o == m) {
          val = gam * (S[k * g + m] / sqrt(lamv[k]));  // eigenbasis (see above)
        } else {
          val = kc[(o - m - 1) * NYLS_MAX_M + k];  // h_j[k]
        }
      }
    } else if (a == m && b == m) {
      val = gam * S[m * g + m];
    } else if (a == m || b == m) {
      const int j = (a == m ? b : a) - m - 1;
      val = d.cond_d[j] == 0 ? 1.0 : 0.0;
    }
    K[a * lda + b] = val;
  }
  for (int a = (mx ? m + 1 : 0) + tid; a < N; a += NYLS_BLOCK) {
    double val;
    if (a < m) {
      double acc = 0.0;
      if (a < r) acc = S[a * g + m + 1] / sqrt(lamv[a]);  // eigenbasis (see above)
      val = gam * acc;
    } else if (a == m) {
      val = gam * S[m * g + m + 1];
    } else {
      val = d.v[a - m - 1];
    }
    rhs[a] = val;
  }
  __syncthreads();
  if (kkt_out) {
    double* ko = kkt_out + (size_t)inst * kn * kn;
    for (int e = tid; e < N * N; e += NYLS_BLOCK) ko[e] = K[(e / N) * lda + e % N];
    for (int a = tid; a < N; a += NYLS_BLOCK) rhs_out[(size_t)inst * kn + a] = rhs[a];
  }
  if (!factor) return;
  int sing;
  if (N <= 64) {
    // one wavefront factors and solves (rows stay in place, perm gives their order); the
    // other wavefronts wait at the barrier
    if (tid < 64) {
      const int s1 = nyls_lu_wave(K, lda, N, rhs, piv, perm);
      if (tid == 0) red[0] = (double)s1;
    }
    __syncthreads();
    sing = (int)red[0];
    for (int e = tid; e < N * N; e += NYLS_BLOCK) ws[L.lu + e] = K[perm[e / N] * lda + e % N];
  } else if (wide) {
    sing = lu_global(K, N, piv, kc, red, perm);
    nyls_lu_solve(K, lda, N, piv, rhs);
  } else {
    sing = nyls_lu(K, lda, N, piv, red);
    nyls_lu_solve(K, lda, N, piv, rhs);
    for (int e = tid; e < N * N; e += NYLS_BLOCK) ws[L.lu + e] = K[(e / N) * lda + e % N];
  }
  for (int a = tid; a < N; a += NYLS_BLOCK) {
    ws[L.piv + a] = (double)piv[a];
    ws[L.x + a] = rhs[a];
  }
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * rhs[k];
    ws[L.alpha + s] = acc;
  }
  if (tid == 0) {
    int bits = (int)ws[L.info + 1];
    if (sing) bits |= NYLS_S_SINGULAR;
    for (int a = 0; a < N; ++a)
      if (!(fabs(rhs[a]) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    ws[L.info + 1] = (double)bits;
  }
}

}  // namespace

// LDS of k_kkt: the matrix of the largest on-chip system (bases up to m = mn <= glo), or the
// vectors of a system factored in the workspace, whichever is larger.
size_t nyls_kkt_lds_bytes(int mn, int maxm, int maxp, int glo) {
  const int Nn = mn + 1 + maxp, Nw = maxm + 1 + maxp;
  const size_t narrow = mn > 0 ? (size_t)Nn * (Nn + 1) + (Nn + 1) : 0;
  const size_t wide = maxm > glo ? (size_t)(Nw + 1) : 0;
  const int Nmax = Nn > Nw ? Nn : Nw;
  return ((narrow > wide ? narrow : wide) + NYLS_MAX_P * NYLS_MAX_M + 16) * sizeof(double) +
         (size_t)2 * (Nmax + 1) * sizeof(int);
}

hipError_t nyls_launch_kkt(const nyls_plan_view& pv, double* ws, double* kkt_out, double* rhs_out,
                           int factor, hipStream_t st) {
  // many 64 < m <= 128 instances: factor them in the workspace (see k_kkt)
  const int glo = pv.n_big >= 32 ? 64 : NYLS_NARROW_MAX_M;
  const int mn = pv.maxm_narrow < glo ? pv.maxm_narrow : glo;
  const size_t lds = nyls_kkt_lds_bytes(mn, pv.maxm, pv.maxp, glo);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kkt<false>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kkt<true>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int kn = pv.maxm + 1 + NYLS_MAX_P;
  const int eb = (pv.mode == NYLS_MIXED && !pv.only) ? 1 : 0;
  if (pv.maxm_narrow + 2 > 64)  // (NYLS_MIXED too: those bases take the FP64 Gram)
    hipLaunchKernelGGL(k_kkt_mfma_wide, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, pv.d_order, ws,
                       -1, eb, pv.only);
  if (pv.maxm > NYLS_NARROW_MAX_M && !eb) {
    const int g = pv.maxm + 2;
    for (int step = 0; step < 2; ++step)
      hipLaunchKernelGGL(k_kkt_wide_transform, dim3(pv.batch, (g * g + NYLS_BLOCK - 1) / NYLS_BLOCK),
                         dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, step);
  }
  if (glo == NYLS_NARROW_MAX_M ? pv.maxm_narrow > 0 : pv.batch > pv.n_big)  // some m <= glo
    hipLaunchKernelGGL(k_kkt<false>, dim3(pv.batch), dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order, ws,
                       kkt_out, rhs_out, kn, factor, -1, eb, pv.only, glo);
  if (pv.maxm > glo)
    hipLaunchKernelGGL(k_kkt<true>, dim3(pv.batch), dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order, ws,
                       kkt_out, rhs_out, kn, factor, -1, eb, pv.only, glo);
  return hipGetLastError();
}
