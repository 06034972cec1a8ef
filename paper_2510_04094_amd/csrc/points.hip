// Per-grid-point FP64 passes after the KKT solve, one workgroup per instance:
//
//  * iterative refinement (mixed precision): with the current (omega, b, lambda) and
//    alpha = W omega, the exact FP64 residual of the Lemma 1 system is formed without
//    the Gram, from one pass over the points:
//        rho_i = r_i - p_i^T alpha - c_i b,
//        R_omega = gamma W^T sum_i rho_i p_i - omega - H lambda,
//        R_b     = gamma sum_i c_i rho_i - delta^T lambda,
//        R_v     = v - H^T omega - delta b,
//    and the correction solves the stored factorisation (assembled from the FP32 or the
//    kernel-space FP64 Gram, both of which lose accuracy when K_mm is ill-conditioned);
//    steps repeat until the correction is at rounding level or `refine` steps are done;
//  * output: y_hat(t_i) = alpha^T k_m(t_i) + b on the whole grid (Sec. 3.1 model).
#include "nyls_dense.h"

namespace {

constexpr int TP = 32;  // points per refinement tile
constexpr int TPG = NYLS_BLOCK / TP;  // threads per point in the dot products

__device__ inline int instance_of(const int32_t* order, int single) {
  return single >= 0 ? single : (order ? order[blockIdx.x] : (int)blockIdx.x);
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_points(
    const nyls_desc* __restrict__ desc, const int32_t* __restrict__ order,
    double* __restrict__ wsbase, int refine, double* __restrict__ yhat,
    double* __restrict__ omega_out, double* __restrict__ bias_out, double* __restrict__ lambda_out,
    int32_t* __restrict__ status, int maxm, int single) {
  extern __shared__ double sm[];
  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  const int m = d.m, p = d.p, n = d.n;
  const int N = m + 1 + p;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma, inv_sigma = 1.0 / d.sigma;

  const double* LU = ws + L.lu;            // factors stay in global memory (L2-resident)
  double* Pt = sm;                         // [TP][m]
  double* rho = Pt + TP * maxm;            // [TP]
  double* fr = rho + TP;                   // [TP][p+1]
  double* al = fr + TP * (NYLS_MAX_P + 1); // [m] alpha
  double* tl = al + NYLS_MAX_M;            // [m] landmark times
  double* z = tl + NYLS_MAX_M;             // [m] reduced sum rho_i p_i
  double* R = z + NYLS_MAX_M;              // [N]
  double* x = R + (NYLS_MAX_M + 1 + NYLS_MAX_P);  // [N]
  double* red = x + (NYLS_MAX_M + 1 + NYLS_MAX_P);  // [16]
  double* zpart = red + 16;                // [NYLS_BLOCK]
  int* piv = reinterpret_cast<int*>(zpart + NYLS_BLOCK);
  int* okp = piv + (NYLS_MAX_M + 1 + NYLS_MAX_P);

  for (int s = tid; s < m; s += NYLS_BLOCK) {
    tl[s] = nyls_grid_t(d, d.lidx[s]);
    al[s] = ws[L.alpha + s];
  }
  for (int a = tid; a < N; a += NYLS_BLOCK) x[a] = ws[L.x + a];
  if (refine > 0)
    for (int a = tid; a < N; a += NYLS_BLOCK) piv[a] = (int)ws[L.piv + a];
  __syncthreads();

  const int ngc = NYLS_BLOCK / m;  // accumulation groups over points
  const int cs = tid % m, cg = tid / m;
  double corr = 0.0;
  for (int step = 0; step < refine; ++step) {
    const double b = x[m];
    double zacc = 0.0, sacc = 0.0;
    for (int i0 = 0; i0 < n; i0 += TP) {
      __syncthreads();
      for (int e = tid; e < TP; e += NYLS_BLOCK) {
        const int i = i0 + e;
        const bool ok = i < n && !nyls_is_condition_point(d, i);
        okp[e] = ok;
        for (int k = 0; k < p; ++k) fr[e * (NYLS_MAX_P + 1) + k] = ok ? d.f[(size_t)k * n + i] : 0.0;
        fr[e * (NYLS_MAX_P + 1) + p] = ok ? d.r[i] : 0.0;
      }
      __syncthreads();
      for (int e = tid; e < TP * m; e += NYLS_BLOCK) {
        const int pt = e / m, s = e - pt * m;
        double val = 0.0;
        if (okp[pt]) {
          const double* fp = fr + pt * (NYLS_MAX_P + 1);
          const double zz = (nyls_grid_t(d, i0 + pt) - tl[s]) * inv_sigma;
          double kd[NYLS_MAX_P + 1], w[NYLS_MAX_P + 1];
          nyls_kderiv(zz, inv_sigma, kd);
          nyls_opweights(p, [&](int k) { return fp[k - 1]; }, w);
          val = nyls_dot5(w, kd);
        }
        Pt[pt * m + s] = val;
      }
      __syncthreads();
      {
        const int pt = tid / TPG, sub = tid % TPG;
        double acc = 0.0;
        for (int s = sub; s < m; s += TPG) acc += Pt[pt * m + s] * al[s];
        for (int o = TPG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (sub == 0) {
          const double* fp = fr + pt * (NYLS_MAX_P + 1);
          const double c = -fp[p - 1];
          const double rv = okp[pt] ? fp[p] - acc - c * b : 0.0;
          rho[pt] = rv;
          sacc += c * rv;
        }
      }
      __syncthreads();
      if (cg < ngc)
        for (int pt = cg; pt < TP; pt += ngc) zacc += rho[pt] * Pt[pt * m + cs];
    }
    zpart[tid] = (cg < ngc) ? zacc : 0.0;
    const double ssum = nyls_block_sum(sacc, red);
    __syncthreads();
    for (int s = tid; s < m; s += NYLS_BLOCK) {
      double acc = 0.0;
      for (int gi = 0; gi < ngc; ++gi) acc += zpart[gi * m + s];
      z[s] = acc;
    }
    __syncthreads();
    for (int a = tid; a < N; a += NYLS_BLOCK) {
      double val = 0.0;
      if (a < m) {
        if (a < r) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + a] * z[s];
          val = gam * acc - x[a];
          for (int j = 0; j < p; ++j) val -= ws[L.H + j * m + a] * x[m + 1 + j];
        }
      } else if (a == m) {
        val = gam * ssum;
        for (int j = 0; j < p; ++j) val -= (d.cond_d[j] == 0 ? 1.0 : 0.0) * x[m + 1 + j];
      } else {
        const int j = a - m - 1;
        val = d.v[j] - (d.cond_d[j] == 0 ? x[m] : 0.0);
        for (int k = 0; k < r; ++k) val -= ws[L.H + j * m + k] * x[k];
      }
      R[a] = val;
    }
    __syncthreads();
    nyls_lu_solve(LU, N, N, piv, R);
    for (int a = tid; a < N; a += NYLS_BLOCK) x[a] += R[a];
    __syncthreads();
    // correction size bound |delta y_hat|_inf <= |W delta omega|_1 + |delta b| (|k_s| <= 1)
    double part = 0.0;
    for (int s = tid; s < m; s += NYLS_BLOCK) {
      double acc = 0.0, dacc = 0.0;
      for (int k = 0; k < r; ++k) { acc += W[s * m + k] * x[k]; dacc += W[s * m + k] * R[k]; }
      al[s] = acc;
      part += fabs(dacc);
    }
    corr = nyls_block_sum(part, red) + fabs(R[m]);
    // stop once the correction is at rounding level relative to the solution size
    double asz = 0.0;
    for (int s = tid; s < m; s += NYLS_BLOCK) asz += fabs(al[s]);
    asz = nyls_block_sum(asz, red) + fabs(x[m]);
    __syncthreads();
    if (corr <= 1e-13 * asz) break;
  }

  // Output pass: y_hat on every grid point.
  const double b = x[m];
  double* yo = yhat + d.goff;
  for (int i = tid; i < n; i += NYLS_BLOCK) {
    const double ti = nyls_grid_t(d, i);
    double acc = 0.0;
    for (int s = 0; s < m; ++s) {
      const double zz = (ti - tl[s]) * inv_sigma;
      acc += al[s] * exp(-zz * zz);
    }
    yo[i] = acc + b;
  }
  for (int a = tid; a < N; a += NYLS_BLOCK) ws[L.x + a] = x[a];
  for (int s = tid; s < m; s += NYLS_BLOCK) ws[L.alpha + s] = al[s];
  if (omega_out)
    for (int k = tid; k < maxm; k += NYLS_BLOCK) omega_out[(size_t)inst * maxm + k] = k < m ? x[k] : 0.0;
  if (lambda_out)
    for (int j = tid; j < NYLS_MAX_P; j += NYLS_BLOCK) lambda_out[(size_t)inst * NYLS_MAX_P + j] = j < p ? x[m + 1 + j] : 0.0;
  if (tid == 0) {
    if (bias_out) bias_out[inst] = b;
    int bits = (int)ws[L.info + 1];
    if (!(fabs(b) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 3] = corr;
    if (status) status[inst] = bits;
  }
}

}  // namespace

size_t nyls_points_lds_bytes(int maxm, int maxp) {
  (void)maxp;
  const int NK = NYLS_MAX_M + 1 + NYLS_MAX_P;
  return ((size_t)TP * maxm + TP + TP * (NYLS_MAX_P + 1) + 3 * NYLS_MAX_M + 2 * NK + 16 +
          NYLS_BLOCK) * sizeof(double) + (size_t)(NK + TP) * sizeof(int);
}

hipError_t nyls_launch_points(const nyls_plan_view& pv, double* ws, int refine, double* yhat,
                              double* omega, double* bias, double* lambda, int32_t* status,
                              int single, hipStream_t st) {
  const size_t lds = nyls_points_lds_bytes(pv.maxm, pv.maxp);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_points),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_points, dim3(single >= 0 ? 1 : pv.batch), dim3(NYLS_BLOCK), lds, st,
                     pv.d_desc, pv.d_order, ws, refine, yhat, omega, bias, lambda, status, pv.maxm,
                     single);
  return hipGetLastError();
}
