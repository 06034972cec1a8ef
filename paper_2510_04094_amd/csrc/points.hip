// Per-grid-point FP64 passes after the KKT solve, one wavefront per instance:
//
//  * iterative refinement: with the current (omega, b, lambda) and alpha = W omega, the
//    exact FP64 residual of the Lemma 1 system is formed without the Gram, from one pass
//    over the points:
//        rho_i = r_i - p_i^T alpha - c_i b,
//        R_omega = gamma W^T sum_i rho_i p_i - omega - H lambda,
//        R_b     = gamma sum_i c_i rho_i - delta^T lambda,
//        R_v     = v - H^T omega - delta b,
//    and the correction solves the stored factorisation (assembled from an FP32 or a
//    kernel-space FP64 Gram, which lose accuracy when K_mm is ill-conditioned);
//  * output: y_hat(t_i) = alpha^T k_m(t_i) + b on the whole grid (Sec. 3.1 model).
// Each pass also writes y_hat for the current solution, so once a correction is below
// 1e-11 max|y_hat| the iteration stops and no separate output pass runs.
//
// Layout of the work: lane s owns landmark s (and s + 64 when m > 64) and walks the grid
// in chunks of CP points with the Gaussian recurrence, so kernel values never leave
// registers; the per-point weights of the ODE operator are broadcast from the lane that
// loaded them; per-point dot products over the landmarks go through a small LDS tile and
// a 4-way lane split; sum_i rho_i p_i stays in each landmark's lane.  A single wavefront
// needs no workgroup barriers, and the small LDS footprint lets many instances share a CU.
#include "nyls_dense.h"

namespace {

constexpr int CP = 16;  // points per chunk
constexpr int NK = NYLS_MAX_M + 1 + NYLS_MAX_P;

__device__ inline int instance_of(const int32_t* order, int single) {
  return single >= 0 ? single : (order ? order[blockIdx.x] : (int)blockIdx.x);
}

template <int ML>
__global__ __launch_bounds__(64) void k_points(
    const nyls_desc* __restrict__ desc, const int32_t* __restrict__ order,
    double* __restrict__ wsbase, int refine, double* __restrict__ yhat,
    double* __restrict__ omega_out, double* __restrict__ bias_out, double* __restrict__ lambda_out,
    int32_t* __restrict__ status, int maxm, int single) {
  __shared__ double T1[CP][64 * ML];  // p_i[s] alpha_s
  __shared__ double T0[CP][64 * ML];  // k_s(t_i) alpha_s
  __shared__ double Rv[NK], xv[NK], zs[NYLS_MAX_M];
  __shared__ int piv[NK];

  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  const int m = d.m, p = d.p, n = d.n;
  const int N = m + 1 + p;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* LU = ws + L.lu;
  const int lane = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma, inv_sigma = 1.0 / d.sigma;
  const double a = d.dt * inv_sigma, q2 = exp(-2.0 * a * a);
  double* yo = yhat + d.goff;

  int ls[ML];
  double tls[ML], alv[ML];
  bool lv[ML];
#pragma unroll
  for (int u = 0; u < ML; ++u) {
    const int s = lane + 64 * u;
    lv[u] = s < m;
    ls[u] = lv[u] ? d.lidx[s] : 0;
    tls[u] = lv[u] ? nyls_grid_t(d, ls[u]) : 0.0;
    alv[u] = lv[u] ? ws[L.alpha + s] : 0.0;
  }
  for (int e = lane; e < N; e += 64) {
    xv[e] = ws[L.x + e];
    piv[e] = (int)ws[L.piv + e];
  }
  __syncthreads();

  // One pass over the grid.  Always writes y_hat for the current (alpha, b); when
  // `refining` also forms rho_i and accumulates sum_i rho_i p_i (zacc, per landmark lane)
  // and sum_i c_i rho_i (sacc).
  auto pass = [&](bool refining, double b, double (&zacc)[ML], double& sacc, double& ymax) {
    for (int i0 = 0; i0 < n; i0 += CP) {
      const int pi = i0 + lane;
      const bool okj = lane < CP && pi < n && !nyls_is_condition_point(d, pi);
      double wj[NYLS_MAX_P + 1];
      nyls_opweights(p, [&](int k) { return okj ? d.f[(size_t)(k - 1) * n + pi] : 0.0; }, wj);
      const double cj = okj ? -d.f[(size_t)(p - 1) * n + pi] : 0.0;
      const double rj = okj ? d.r[pi] : 0.0;
      double pv[ML][CP];
#pragma unroll
      for (int u = 0; u < ML; ++u) {
        nyls_wave_gauss<CP>(d, i0, ls[u], tls[u], a, q2, inv_sigma, [&](int jj, double z, double e) {
          double pvv = 0.0;
          if (refining) {
            double kd[NYLS_MAX_P + 1];
            nyls_kderiv_e(z, e, inv_sigma, kd);
#pragma unroll
            for (int q = 0; q <= NYLS_MAX_P; ++q) pvv += nyls_rdlane(wj[q], jj) * kd[q];
          }
          pvv = lv[u] ? pvv : 0.0;
          pv[u][jj] = pvv;
          T1[jj][lane + 64 * u] = pvv * alv[u];
          T0[jj][lane + 64 * u] = lv[u] ? e * alv[u] : 0.0;
        });
      }
      __syncthreads();
      const int pl = lane % CP, part = lane / CP;
      double s1 = 0.0, s0 = 0.0;
#pragma unroll
      for (int c = part; c < 64 * ML; c += 64 / CP) {
        s1 += T1[pl][c];
        s0 += T0[pl][c];
      }
      s1 += __shfl_xor(s1, 16);
      s1 += __shfl_xor(s1, 32);
      s0 += __shfl_xor(s0, 16);
      s0 += __shfl_xor(s0, 32);
      __syncthreads();
      double rho = 0.0;
      if (lane < CP && pi < n) {
        yo[pi] = s0 + b;
        ymax = fmax(ymax, fabs(s0 + b));
        if (refining && okj) {
          rho = rj - s1 - cj * b;
          sacc += cj * rho;
        }
      }
      if (refining) {
#pragma unroll
        for (int jj = 0; jj < CP; ++jj) {
          const double rr = nyls_rdlane(rho, jj);
#pragma unroll
          for (int u = 0; u < ML; ++u) zacc[u] += rr * pv[u][jj];
        }
      }
    }
  };

  double corr = 0.0, ymax = 0.0;
  bool need_output = true;
  for (int step = 0; step < refine; ++step) {
    double zacc[ML], sacc = 0.0;
    ymax = 0.0;
#pragma unroll
    for (int u = 0; u < ML; ++u) zacc[u] = 0.0;
    pass(true, xv[m], zacc, sacc, ymax);
#pragma unroll
    for (int u = 0; u < ML; ++u)
      if (lv[u]) zs[lane + 64 * u] = zacc[u];
    const double ssum = nyls_wave_sum(sacc);
    ymax = nyls_wave_max(ymax);
    __syncthreads();
    for (int e = lane; e < N; e += 64) {
      double val = 0.0;
      if (e < m) {
        if (e < r) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + e] * zs[s];
          val = gam * acc - xv[e];
          for (int j = 0; j < p; ++j) val -= ws[L.H + j * m + e] * xv[m + 1 + j];
        }
      } else if (e == m) {
        val = gam * ssum;
        for (int j = 0; j < p; ++j) val -= (d.cond_d[j] == 0 ? 1.0 : 0.0) * xv[m + 1 + j];
      } else {
        const int j = e - m - 1;
        val = d.v[j] - (d.cond_d[j] == 0 ? xv[m] : 0.0);
        for (int k = 0; k < r; ++k) val -= ws[L.H + j * m + k] * xv[k];
      }
      Rv[e] = val;
    }
    __syncthreads();
    nyls_lu_solve_w(LU, N, N, piv, Rv);
    for (int e = lane; e < N; e += 64) xv[e] += Rv[e];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < ML; ++u) {
      const int s = lane + 64 * u;
      if (lv[u]) {
        double acc = 0.0;
        for (int k = 0; k < r; ++k) acc += W[s * m + k] * xv[k];
        alv[u] = acc;
      }
    }
    // The change of y_hat(t) is phi(t)^T d_omega + d_b, and |phi(t)|_2^2 is the Nystrom
    // approximation of k(t, t) = 1, which never exceeds it: |d_y_hat| <= |d_omega|_2 + |d_b|.
    double dsq = 0.0;
    for (int k = lane; k < r; k += 64) dsq += Rv[k] * Rv[k];
    corr = sqrt(nyls_wave_sum(dsq)) + fabs(Rv[m]);
    if (corr <= 1e-11 * ymax) {  // y_hat written by this pass is final to rounding level
      need_output = false;
      break;
    }
  }
  if (need_output) {
    double zacc[ML], sacc = 0.0, ym = 0.0;
    pass(false, xv[m], zacc, sacc, ym);
  }

  for (int e = lane; e < N; e += 64) ws[L.x + e] = xv[e];
#pragma unroll
  for (int u = 0; u < ML; ++u)
    if (lv[u]) ws[L.alpha + lane + 64 * u] = alv[u];
  if (omega_out)
    for (int k = lane; k < maxm; k += 64) omega_out[(size_t)inst * maxm + k] = k < m ? xv[k] : 0.0;
  if (lambda_out && lane < NYLS_MAX_P)
    lambda_out[(size_t)inst * NYLS_MAX_P + lane] = lane < p ? xv[m + 1 + lane] : 0.0;
  if (lane == 0) {
    if (bias_out) bias_out[inst] = xv[m];
    int bits = (int)ws[L.info + 1];
    if (!(fabs(xv[m]) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    if (refine > 0 && need_output && corr > 1e-8 * ymax) bits |= NYLS_S_REFINE_NOCONV;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 3] = corr;
    if (status) status[inst] = bits;
  }
}

}  // namespace

hipError_t nyls_launch_points(const nyls_plan_view& pv, double* ws, int refine, double* yhat,
                              double* omega, double* bias, double* lambda, int32_t* status,
                              int single, hipStream_t st) {
  const dim3 grid(single >= 0 ? 1 : pv.batch);
  if (pv.maxm <= 64)
    hipLaunchKernelGGL(k_points<1>, grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws, refine, yhat,
                       omega, bias, lambda, status, pv.maxm, single);
  else
    hipLaunchKernelGGL(k_points<2>, grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws, refine, yhat,
                       omega, bias, lambda, status, pv.maxm, single);
  return hipGetLastError();
}
