// Explicit feature map and prediction at caller times (App. A.2 eq32, Sec. 3):
//   phi^(d)(t) = W^T k_m^(d)(t),   y_hat^(d)(t) = alpha^T k_m^(d)(t) + [d = 0] b.
// Grid: (instance, tile of evaluation points).  A tile's kernel-derivative values are
// built once in LDS and contracted with W (read from the workspace, L2-resident).
#include <algorithm>

#include "nyls_internal.h"

namespace {

// evaluation points per workgroup (8 for wide bases, whose kernel values would not fit)
__host__ __device__ inline int tile_points(int maxm) { return maxm > NYLS_NARROW_MAX_M ? 8 : 16; }

__global__ __launch_bounds__(NYLS_BLOCK) void k_features(
    const nyls_desc* __restrict__ desc, const double* __restrict__ wsbase,
    const double* __restrict__ t_eval, const int64_t* __restrict__ eval_off, int dmax,
    double* __restrict__ phi, double* __restrict__ eigval, int32_t* __restrict__ rank_out,
    int maxm, int single) {
  extern __shared__ double sm[];
  const int inst = single >= 0 ? single : (int)blockIdx.y;
  const nyls_desc& d = desc[inst];
  const int m = d.m;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  const double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;
  // t_eval == nullptr: evaluate on the instance's own grid points 0..n-1
  const bool on_grid = (t_eval == nullptr);
  const int64_t e0 = on_grid ? 0 : eval_off[inst], e1 = on_grid ? d.n : eval_off[inst + 1];
  if (blockIdx.x == 0) {
    if (eigval)
      for (int k = tid; k < maxm; k += NYLS_BLOCK) eigval[(size_t)inst * maxm + k] = k < m ? ws[L.lam + k] : 0.0;
    if (rank_out && tid == 0) rank_out[inst] = (int32_t)ws[L.info + 0];
  }
  const int nd = dmax + 1;
  const int TE = tile_points(maxm);
  double* kd = sm;                 // [TE][nd][m]
  double* tl = kd + TE * nd * maxm;
  const double inv_sigma = 1.0 / d.sigma;
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  const double* W = ws + L.W;
  for (int64_t base = e0 + (int64_t)blockIdx.x * TE; base < e1; base += (int64_t)gridDim.x * TE) {
  const int cnt = (int)((e1 - base) < TE ? (e1 - base) : TE);
  __syncthreads();
  for (int e = tid; e < cnt * m; e += NYLS_BLOCK) {
    const int pt = e / m, s = e - pt * m;
    const double te = on_grid ? nyls_grid_t(d, (int)(base + pt)) : t_eval[base + pt];
    const double z = (te - tl[s]) * inv_sigma;
    double v[NYLS_MAX_P + 1];
    nyls_kderiv(z, inv_sigma, v);
#pragma unroll
    for (int q = 0; q <= NYLS_MAX_P; ++q)
      if (q < nd) kd[(pt * nd + q) * m + s] = v[q];
  }
  __syncthreads();
  for (int e = tid; e < cnt * nd * maxm; e += NYLS_BLOCK) {
    const int k = e % maxm, row = e / maxm;  // row = pt * nd + q
    double acc = 0.0;
    if (k < m) {
      const double* kr = kd + row * m;
      for (int s = 0; s < m; ++s) acc += W[s * m + k] * kr[s];
    }
    phi[(base * nd + row) * maxm + k] = acc;
  }
  }
}

__global__ __launch_bounds__(64) void k_predict(
    const nyls_desc* __restrict__ desc, const double* __restrict__ wsbase,
    const double* __restrict__ t_eval, const int64_t* __restrict__ eval_off, int dd,
    double* __restrict__ out) {
  __shared__ double tl[NYLS_MAX_M], al[NYLS_MAX_M];
  const int inst = blockIdx.y;
  const nyls_desc& d = desc[inst];
  const int m = d.m;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  const double* ws = wsbase + d.ws;
  const int64_t e0 = eval_off[inst], e1 = eval_off[inst + 1];
  if (e0 + (int64_t)blockIdx.x * 64 >= e1) return;
  for (int s = threadIdx.x; s < m; s += 64) {
    tl[s] = nyls_grid_t(d, d.lidx[s]);
    al[s] = ws[L.alpha + s];
  }
  __syncthreads();
  const double inv_sigma = 1.0 / d.sigma;
  const double bias = dd == 0 ? ws[L.x + m] : 0.0;
  for (int64_t e = e0 + (int64_t)blockIdx.x * 64 + threadIdx.x; e < e1; e += (int64_t)gridDim.x * 64) {
    const double t = t_eval[e];
    double acc = 0.0;
    for (int s = 0; s < m; ++s) {
      const double z = (t - tl[s]) * inv_sigma;
      double v[NYLS_MAX_P + 1];
      nyls_kderiv(z, inv_sigma, v);
      acc += al[s] * nyls_pick(v, dd);
    }
    out[e] = acc + bias;
  }
}

}  // namespace

hipError_t nyls_launch_features(const nyls_plan_view& pv, const double* ws, const double* t_eval,
                                const int64_t* eval_off, int dmax, double* phi, double* eigval,
                                int32_t* rank, int64_t max_eval, int single, hipStream_t st) {
  const int TE = tile_points(pv.maxm);
  const size_t lds = ((size_t)TE * (dmax + 1) * pv.maxm + NYLS_MAX_M) * sizeof(double);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_features),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  // grid-stride over each instance's points; the grid is sized for about n evaluations
  // per instance (max_eval caps it)
  int64_t gx = (std::min<int64_t>(max_eval, pv.maxn) + TE - 1) / TE;
  gx = gx < 1 ? 1 : (gx > 64 ? 64 : gx);
  dim3 grid((unsigned)gx, single >= 0 ? 1 : pv.batch);
  hipLaunchKernelGGL(k_features, grid, dim3(NYLS_BLOCK), lds, st, pv.d_desc, ws, t_eval, eval_off,
                     dmax, phi, eigval, rank, pv.maxm, single);
  return hipGetLastError();
}

hipError_t nyls_launch_predict(const nyls_plan_view& pv, const double* ws, const double* t_eval,
                               const int64_t* eval_off, int d, double* out, int64_t max_eval,
                               hipStream_t st) {
  // grid-stride over each instance's times: four one-wave blocks per instance (blocks past the
  // instance's count exit at once); max_eval, when known, caps it lower
  int64_t gx = (max_eval + 63) / 64;
  gx = gx < 1 ? 1 : (gx > 4 ? 4 : gx);
  dim3 grid((unsigned)gx, pv.batch);
  hipLaunchKernelGGL(k_predict, grid, dim3(64), 0, st, pv.d_desc, ws, t_eval, eval_off, d, out);
  return hipGetLastError();
}
