// Leverage-score landmark sampling (Sec. 4.1, "Sampling strategy analysis for Nystrom
// landmarks": equidistant, random and leverage-score sampling).  The paper gives no score
// formula; these kernels compute ridge leverage scores of the grid points in the feature
// space of the plan's own (pilot) basis,
//     l_i = phi(t_i)^T (Phi^T Phi + ridge I)^{-1} phi(t_i),   Phi = [phi(t_i)]_{i < n},
// and draw m distinct landmarks with probabilities proportional to l_i without replacement by
// exponential keys ln(u_i) / l_i (Efraimidis and Spirakis, 2006), the caller handing in the
// uniforms u_i.
//
//  k_lev_prepare   one workgroup per instance: G = Phi^T Phi + ridge I accumulated in feature
//                  space over every grid point (kernel values from the Gaussian recurrence in
//                  LDS tiles, rotated by W), and G^{-1} (r x r) into the workspace;
//  k_lev_scores    a workgroup per (instance, 32 points): phi_i = W^T k_i staged in LDS,
//                  l_i = phi_i^T G^{-1} phi_i;
//  k_lev_select    one workgroup per instance: the m (or m - 2 interior, with the end points)
//                  largest keys by m successive block-wide maxima over (key, -index), each
//                  round looking only below the previous maximum, then sorted.
#include "nyls_dense.h"
#include "nyls_gramacc.h"

namespace {

constexpr int TP = 32;  // points per Gram tile
constexpr int CH = 8;   // points per thread in the Gaussian recurrence
constexpr int SP = 32;  // points per score workgroup

__host__ __device__ inline int round4(int x) { return (x + 3) & ~3; }

__global__ __launch_bounds__(NYLS_BLOCK) void k_lev_prepare(const nyls_desc* __restrict__ desc,
                                                            double* __restrict__ wsbase,
                                                            double ridge_in) {
  extern __shared__ double sm[];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const int gp = round4(r > 0 ? r : 1);
  const double ridge = ridge_in > 0.0 ? ridge_in : 1.0 / d.gamma;
  const double inv_sigma = 1.0 / d.sigma;
  double* tl = sm;                  // [128]
  double* red = tl + NYLS_NARROW_MAX_M;    // [16]
  int* piv = reinterpret_cast<int*>(red + 16);  // [128]
  double* big = reinterpret_cast<double*>(piv + NYLS_NARROW_MAX_M);
  double* K = big;                  // [TP][maxm] kernel values of a tile
  double* Q = K + TP * NYLS_NARROW_MAX_M;  // [TP][gp] features of a tile (also the reduction buffer)
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  __syncthreads();
  // G = Phi^T Phi accumulated in feature space: a kernel-space sum mapped through W twice
  // would carry its rounding amplified by lambda_1 / lambda_r
  nyls_gram::Acc A;
  nyls_gram::setup(A, gp);
  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma,
                            [&](int pt, int s, double, double ev) { K[pt * NYLS_NARROW_MAX_M + s] = ev; });
    __syncthreads();
    for (int e = tid; e < TP * gp; e += NYLS_BLOCK) {
      const int pt = e / gp, k = e - pt * gp;
      double acc = 0.0;
      if (k < r)
        for (int s = 0; s < m; ++s) acc += K[pt * NYLS_NARROW_MAX_M + s] * W[s * m + k];
      Q[e] = acc;
    }
    __syncthreads();
    nyls_gram::accumulate(A, Q, gp, nullptr, TP);
  }
  double* G = big;                 // [r][r + 1] after the tiles
  const int lg = r + 1;
  double* S = ws + L.gram;         // r x r (row stride r)
  nyls_gram::finish(A, Q, S, r, r);
  for (int e = tid; e < r * r; e += NYLS_BLOCK) {
    const int k = e / r, l = e - k * r;
    G[k * lg + l] = S[e] + (k == l ? ridge : 0.0);
  }
  __syncthreads();
  nyls_lu(G, lg, r, piv, red);
  // G^{-1}, column by column, into the U region (r x r, row stride r): l_i = phi_i^T G^{-1}
  // phi_i with phi_i = W^T k_i formed per point by the score kernel
  double* Gi = ws + L.U;
  double* X = G + r * lg;          // [r]
  for (int c = 0; c < r; ++c) {
    for (int k = tid; k < r; k += NYLS_BLOCK) X[k] = (k == c) ? 1.0 : 0.0;
    __syncthreads();
    nyls_lu_solve(G, lg, r, piv, X);
    for (int k = tid; k < r; k += NYLS_BLOCK) Gi[k * r + c] = X[k];
    __syncthreads();
  }
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_lev_scores(const nyls_desc* __restrict__ desc,
                                                           const double* __restrict__ wsbase,
                                                           double* __restrict__ scores) {
  __shared__ double kt[SP][NYLS_NARROW_MAX_M + 1];  // k_i, then phi_i = W^T k_i
  __shared__ double ph[SP][NYLS_NARROW_MAX_M + 1];
  __shared__ double part[NYLS_BLOCK];
  __shared__ double tl[NYLS_NARROW_MAX_M];
  const nyls_desc& d = desc[blockIdx.y];
  const int m = d.m, n = d.n;
  const int i0 = blockIdx.x * SP;
  if (i0 >= n) return;  // the grid is sized for the longest instance
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  const double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* Gi = ws + L.U;
  const int r = (int)ws[L.info + 0];
  const int tid = threadIdx.x;
  const double inv_sigma = 1.0 / d.sigma;
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  __syncthreads();
  for (int e = tid; e < SP * m; e += NYLS_BLOCK) {
    const int pt = e / m, s = e - pt * m;
    const int i = i0 + pt;
    const double z = i < n ? (nyls_grid_t(d, i) - tl[s]) * inv_sigma : 0.0;
    kt[pt][s] = i < n ? exp(-z * z) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < SP * r; e += NYLS_BLOCK) {
    const int pt = e / r, k = e - pt * r;
    double acc = 0.0;
    for (int s = 0; s < m; ++s) acc += kt[pt][s] * W[s * m + k];
    ph[pt][k] = acc;
  }
  __syncthreads();
  // thread (pt, q): rows a = q, q + 8, ... of G^{-1} applied to phi_pt
  constexpr int NQ = NYLS_BLOCK / SP;
  const int pt = tid & (SP - 1), q = tid / SP;
  double acc = 0.0;
  for (int a = q; a < r; a += NQ) {
    double y = 0.0;
    for (int b = 0; b < r; ++b) y += Gi[a * r + b] * ph[pt][b];
    acc += ph[pt][a] * y;
  }
  part[tid] = acc;
  __syncthreads();
  if (q == 0 && i0 + pt < n) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) sum += part[pt + k * SP];
    scores[d.goff + i0 + pt] = sum;
  }
}

// (key, index) order: larger key first, then smaller index (a stable descending sort).
__device__ inline bool lev_before(double ka, int ia, double kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_lev_select(const nyls_desc* __restrict__ desc,
                                                           const double* __restrict__ scores,
                                                           const double* __restrict__ u, int ends,
                                                           int32_t* __restrict__ lidx, int maxm) {
  __shared__ double bk[NYLS_BLOCK / 64];
  __shared__ int bi[NYLS_BLOCK / 64];
  __shared__ int chosen[NYLS_NARROW_MAX_M];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lo = ends ? 1 : 0, hi = ends ? n - 1 : n;
  const int want = ends ? m - 2 : m;
  const double* sc = scores + d.goff;
  const double* uu = u + d.goff;
  double pk = HUGE_VAL;  // previous maximum (key, index)
  int pidx = -1;
  for (int j = 0; j < want; ++j) {
    double best = -HUGE_VAL;
    int bidx = 0x7fffffff;
    for (int i = lo + tid; i < hi; i += NYLS_BLOCK) {
      const double s = sc[i];
      const double key = s > 0.0 ? log(uu[i]) / s : -HUGE_VAL;
      if (lev_before(pk, pidx, key, i) && lev_before(key, i, best, bidx)) {
        best = key;
        bidx = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bidx, o);
      if (lev_before(ob, oi, best, bidx)) {
        best = ob;
        bidx = oi;
      }
    }
    if (lane == 0) {
      bk[wv] = best;
      bi[wv] = bidx;
    }
    __syncthreads();
    best = bk[0];
    bidx = bi[0];
    for (int w = 1; w < NYLS_BLOCK / 64; ++w)
      if (lev_before(bk[w], bi[w], best, bidx)) {
        best = bk[w];
        bidx = bi[w];
      }
    if (tid == 0) chosen[j] = bidx;
    pk = best;
    pidx = bidx;
    __syncthreads();
  }
  if (tid == 0) {
    int cnt = want;
    if (ends) {
      chosen[cnt++] = 0;
      chosen[cnt++] = n - 1;
    }
    for (int a = 1; a < cnt; ++a) {  // insertion sort, m <= 128
      const int v = chosen[a];
      int b = a - 1;
      while (b >= 0 && chosen[b] > v) {
        chosen[b + 1] = chosen[b];
        --b;
      }
      chosen[b + 1] = v;
    }
  }
  __syncthreads();
  for (int k = tid; k < maxm; k += NYLS_BLOCK) lidx[(size_t)inst * maxm + k] = k < m ? chosen[k] : -1;
}

size_t prepare_lds_bytes(int maxm) {
  const int gp = round4(maxm);
  size_t q = (size_t)TP * gp;
  const size_t redd = nyls_gram::red_doubles(gp);
  if (redd > q) q = redd;
  size_t tile = (size_t)TP * NYLS_NARROW_MAX_M + q;
  const size_t g = (size_t)maxm * (maxm + 1) + maxm;
  if (g > tile) tile = g;
  return (NYLS_NARROW_MAX_M + 16) * sizeof(double) + NYLS_NARROW_MAX_M * sizeof(int) + tile * sizeof(double);
}

}  // namespace

struct nyls_plan;
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl);

extern "C" int nyls_leverage_scores(const nyls_plan* pl, double ridge, double* scores, void* ws,
                                    hipStream_t stream) {
  if (!pl || !scores || !ws) return NYLS_E_NULL;
  if (!(ridge >= 0.0) || !(ridge < HUGE_VAL)) return NYLS_E_ARG;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  double* w = static_cast<double*>(ws);
  hipError_t e = nyls_launch_eig(pv, w, -1, stream);
  if (e != hipSuccess) return NYLS_E_HIP;
  const size_t lds = prepare_lds_bytes(pv.maxm);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lev_prepare),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return NYLS_E_HIP;
  hipLaunchKernelGGL(k_lev_prepare, dim3(pv.batch), dim3(NYLS_BLOCK), lds, stream, pv.d_desc, w, ridge);
  const dim3 grid((pv.maxn + SP - 1) / SP, pv.batch);
  hipLaunchKernelGGL(k_lev_scores, grid, dim3(NYLS_BLOCK), 0, stream, pv.d_desc, w, scores);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}

extern "C" int nyls_leverage_sample(const nyls_plan* pl, const double* scores, const double* u,
                                    int32_t ends, int32_t* lidx, hipStream_t stream) {
  if (!pl || !scores || !u || !lidx) return NYLS_E_NULL;
  // with `ends` the other m - 2 landmarks come from the n - 2 interior points (m <= n)
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  hipLaunchKernelGGL(k_lev_select, dim3(pv.batch), dim3(NYLS_BLOCK), 0, stream, pv.d_desc, scores, u,
                     ends ? 1 : 0, lidx, pv.maxm);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}
