// Reference-style FP64 solve of Lemma 1 from explicit feature matrices (Sec. 3.1 as
// written: Psi, Psi', ..., Psi^(p) materialised, the rows of A / gamma = (Psi^(p) -
// sum f_k Psi^(p-k))^T formed, the products by a library GEMM), one instance per launch
// sequence.  This is the plain per-instance GPU baseline; the fused batched kernels never
// materialise the feature matrices.
#include "nyls_dense.h"

namespace {

// rows[i] = (g_i, c_i, r_i) in feature space; zero rows at condition points.
__global__ __launch_bounds__(NYLS_BLOCK) void k_explicit_rows(const nyls_desc* __restrict__ desc,
                                                              const double* __restrict__ wsbase,
                                                              const double* __restrict__ phi,
                                                              double* __restrict__ rows, int maxm,
                                                              int inst) {
  const nyls_desc& d = desc[inst];
  const int m = d.m, p = d.p, n = d.n, g = m + 2, nd = p + 1;
  const int r = (int)wsbase[d.ws + nyls_layout(m, p, 0).info];
  for (int64_t e = (int64_t)blockIdx.x * NYLS_BLOCK + threadIdx.x; e < (int64_t)n * g;
       e += (int64_t)gridDim.x * NYLS_BLOCK) {
    const int i = (int)(e / g), k = (int)(e - (int64_t)i * g);
    double val = 0.0;
    if (!nyls_is_condition_point(d, i)) {
      if (k < m) {
        if (k < r) {
          const double* row = phi + (size_t)i * nd * maxm;
          val = row[p * maxm + k];
          for (int q = 1; q <= p; ++q) val -= d.f[(size_t)(q - 1) * n + i] * row[(p - q) * maxm + k];
        }
      } else if (k == m) {
        val = -d.f[(size_t)(p - 1) * n + i];
      } else {
        val = d.r[i];
      }
    }
    rows[e] = val;
  }
}

// KKT from the feature-space Gram C = rows^T rows (g x g), then LU and solve.
__global__ __launch_bounds__(NYLS_BLOCK) void k_explicit_kkt(
    const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, const double* __restrict__ phi,
    const double* __restrict__ C, int maxm, int inst) {
  extern __shared__ double sm[];
  const nyls_desc& d = desc[inst];
  const int m = d.m, p = d.p;
  const int g = m + 2, N = m + 1 + p, lda = N + 1, nd = p + 1;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma;
  double* K = sm;
  double* rhs = K + N * lda;
  double* red = rhs + N + 1;
  int* piv = reinterpret_cast<int*>(red + 16);
  for (int e = tid; e < N * N; e += NYLS_BLOCK) {
    const int a = e / N, b = e - a * N;
    double val = 0.0;
    const bool fa = a < m, fb = b < m;
    if (fa && fb) {
      val = (a < r && b < r) ? gam * C[a * g + b] + (a == b ? 1.0 : 0.0) : (a == b ? 1.0 : 0.0);
    } else if (fa || fb) {
      const int k = fa ? a : b, o = fa ? b : a;
      if (k < r) {
        if (o == m) {
          val = gam * C[k * g + m];
        } else {
          const int j = o - m - 1;
          val = phi[((size_t)d.cond_i[j] * nd + d.cond_d[j]) * maxm + k];
        }
      }
    } else if (a == m && b == m) {
      val = gam * C[m * g + m];
    } else if (a == m || b == m) {
      const int j = (a == m ? b : a) - m - 1;
      val = d.cond_d[j] == 0 ? 1.0 : 0.0;
    }
    K[a * lda + b] = val;
  }
  for (int a = tid; a < N; a += NYLS_BLOCK) {
    double val;
    if (a < m) val = a < r ? gam * C[a * g + m + 1] : 0.0;
    else if (a == m) val = gam * C[m * g + m + 1];
    else val = d.v[a - m - 1];
    rhs[a] = val;
  }
  for (int e = tid; e < p * m; e += NYLS_BLOCK) {
    const int j = e / m, k = e - j * m;
    ws[L.H + e] = k < r ? phi[((size_t)d.cond_i[j] * nd + d.cond_d[j]) * maxm + k] : 0.0;
  }
  __syncthreads();
  const int sing = nyls_lu(K, lda, N, piv, red);
  nyls_lu_solve(K, lda, N, piv, rhs);
  for (int e = tid; e < N * N; e += NYLS_BLOCK) ws[L.lu + e] = K[(e / N) * lda + e % N];
  for (int a = tid; a < N; a += NYLS_BLOCK) {
    ws[L.piv + a] = (double)piv[a];
    ws[L.x + a] = rhs[a];
  }
  const double* W = ws + L.W;
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * rhs[k];
    ws[L.alpha + s] = acc;
  }
  if (tid == 0 && sing) ws[L.info + 1] = (double)((int)ws[L.info + 1] | NYLS_S_SINGULAR);
}

}  // namespace

hipError_t nyls_launch_explicit_rows(const nyls_plan_view& pv, int inst, const double* ws,
                                     const double* phi, double* rows, int n, int m,
                                     hipStream_t st) {
  const int64_t tot = (int64_t)n * (m + 2);
  int64_t gx = (tot + NYLS_BLOCK - 1) / NYLS_BLOCK;
  gx = gx > 1024 ? 1024 : gx;
  hipLaunchKernelGGL(k_explicit_rows, dim3((unsigned)gx), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, phi,
                     rows, pv.maxm, inst);
  return hipGetLastError();
}

hipError_t nyls_launch_explicit_kkt(const nyls_plan_view& pv, int inst, double* ws,
                                    const double* phi, const double* C, hipStream_t st) {
  const int N = pv.maxm + 1 + pv.maxp;
  const size_t lds = ((size_t)N * (N + 1) + N + 1 + 16) * sizeof(double) + (N + 1) * sizeof(int);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_explicit_kkt),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_explicit_kkt, dim3(1), dim3(NYLS_BLOCK), lds, st, pv.d_desc, ws, phi, C,
                     pv.maxm, inst);
  return hipGetLastError();
}
