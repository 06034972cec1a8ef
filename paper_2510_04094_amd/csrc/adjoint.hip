// Adjoint of the Lemma 1 solve (Sec. 3.1): gradients of a loss l(y_hat(s_j)) with respect
// to the ODE data f_k(t_i), r(t_i), the condition values v_j, gamma and sigma, reusing the
// factorisation nyls_solve left in the workspace.  One workgroup per instance.
//
// With x = (omega, b, lambda) solving A x = rhs (A symmetric), alpha = W omega and the ODE
// residual e_i = p_i^T alpha + c_i b - r_i:
//   1. x_bar = (W^T kbar, sum_j g_j, 0), kbar = sum_j g_j k_m(s_j);  mu = A^{-1} x_bar
//      (plus FP64 iterative refinement of mu: the stored factors are of the FP32 or the
//      kernel-space FP64 Gram, which lose accuracy for ill-conditioned K_mm);
//   2. beta = W mu_omega, nu_i = beta^T p_i + c_i mu_b,
//      yh^(q)_i = alpha^T k^(q)_i + [q=0] b,  zh^(q)_i = beta^T k^(q)_i + [q=0] mu_b;
//   3. dl/df_k(t_i) = gamma (e_i zh^(p-k)_i + nu_i yh^(p-k)_i), dl/dr(t_i) = gamma nu_i,
//      dl/dv_j = mu_lambda_j, dl/dgamma = -sum_i nu_i e_i;
//   4. dl/dsigma = (terms through k^(q)(.) at fixed W, closed-form d/dsigma of the kernel
//      derivatives) + (the K_mm term): the problem depends on W only via Q = W W^T =
//      f(K_mm), f(l) = 1/l above the cut-off, so with dl/dW = g1 omega^T - g2 mu_omega^T
//      (g1 = kbar - gamma sum nu_i p_i - H_k mu_lambda, g2 = gamma sum e_i p_i + H_k lambda)
//      the spectral (Daleckii-Krein) derivative gives
//      sum_{l < r} [ sum_{k < r} F_kl Qb_kl D_kl + 2 sum_{k >= r} F_kl Qb_kl D_kl ],
//      Qb_kl = sqrt(lam_l)/2 ((U^T g1)_k omega_l - (U^T g2)_k mu_l),  D = U^T dK_mm/dsigma U,
//      F_kl = -1/(lam_k lam_l) (k < r), 1/(lam_l (lam_l - lam_k)) (k >= r).
#include "nyls_dense.h"

namespace {

constexpr int TP = 16;
constexpr int CH = 8;                 // points per thread in the Gaussian recurrence
constexpr int TPG = NYLS_BLOCK / TP;  // threads per point in the dot products

// d/dsigma of the q-th kernel derivative:
// (-1)^(q+1) sigma^(-q-1) e^{-z^2} (q H_q(z) - z H_{q+1}(z)), all q = 0..NYLS_MAX_P.
__device__ inline void kderiv_dsigma_e(double z, double e, double inv_sigma,
                                       double (&ds)[NYLS_MAX_P + 1]) {
  double hm = 1.0, h = 2.0 * z;     // H_q, H_{q+1} with q = 0
  double sc = -inv_sigma;           // (-1)^(q+1) sigma^(-q-1)
#pragma unroll
  for (int q = 0; q <= NYLS_MAX_P; ++q) {
    ds[q] = sc * e * (q * hm - z * h);
    const double hn = 2.0 * z * h - 2.0 * (q + 1) * hm;
    hm = h;
    h = hn;
    sc *= -inv_sigma;
  }
}

__device__ inline void kderiv_dsigma(double z, double inv_sigma, double (&ds)[NYLS_MAX_P + 1]) {
  kderiv_dsigma_e(z, exp(-z * z), inv_sigma, ds);
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_backward(
    const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, int refine,
    const double* __restrict__ t_obs, const int64_t* __restrict__ obs_off,
    const double* __restrict__ gobs, double* __restrict__ dl_df, double* __restrict__ dl_dr,
    double* __restrict__ dl_dv, double* __restrict__ dl_dsigma, double* __restrict__ dl_dgamma,
    int64_t total, int maxm) {
  extern __shared__ double sm[];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, p = d.p, n = d.n;
  const int N = m + 1 + p;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* U = ws + L.U;
  const double* lamv = ws + L.lam;
  const double* LU = ws + L.lu;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma, sig = d.sigma, inv_sigma = 1.0 / sig;

  double* tl = sm;                      // [128] landmark times
  double* al = tl + NYLS_MAX_M;         // [128] alpha
  double* be = al + NYLS_MAX_M;         // [128] beta = W mu_omega
  double* kb = be + NYLS_MAX_M;         // [128] kbar, later g1
  double* ae = kb + NYLS_MAX_M;         // [128] sum e_i p_i, later g2
  double* an = ae + NYLS_MAX_M;         // [128] sum nu_i p_i
  double* hk = an + NYLS_MAX_M;         // [4][128] kernel-space condition vectors
  double* xv = hk + NYLS_MAX_P * NYLS_MAX_M;  // [136] x
  double* mu = xv + 136;                // [136]
  double* R = mu + 136;                 // [136]
  double* ug = R + 136;                 // [2][128] U^T g1, U^T g2
  double* part = ug + 2 * NYLS_MAX_M;   // [2][256]
  double* red = part + 2 * NYLS_BLOCK;  // [16]
  double* pd = red + 16;                // [TP][8] per-point scalars
  double* wq = pd + TP * 8;             // [TP][NYLS_MAX_P+1] operator weights per point
  int* piv = reinterpret_cast<int*>(wq + TP * (NYLS_MAX_P + 1));  // [136]
  double* big = reinterpret_cast<double*>(piv + 136);
  double* P = big;                      // [TP][m]   p_i
  double* DP = P + TP * maxm;           // [TP][m]   d p_i / d sigma
  double* KQ = DP + TP * maxm;          // [p][TP][m] k^(q)_i, q < p

  for (int s = tid; s < m; s += NYLS_BLOCK) {
    tl[s] = nyls_grid_t(d, d.lidx[s]);
    al[s] = ws[L.alpha + s];
  }
  for (int a = tid; a < N; a += NYLS_BLOCK) {
    xv[a] = ws[L.x + a];
    piv[a] = (int)ws[L.piv + a];
  }
  __syncthreads();
  const double b = xv[m];

  // 1. observations: kbar, sum g, and the direct sigma term sum g_j alpha^T dk(s_j)/dsigma
  const int64_t j0 = obs_off[inst], j1 = obs_off[inst + 1];
  double t1 = 0.0, gsum = 0.0;
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
      const double z = (t_obs[j] - tl[s]) * inv_sigma;
      acc += gobs[j] * exp(-z * z);
    }
    kb[s] = acc;
  }
  for (int64_t j = j0 + tid; j < j1; j += NYLS_BLOCK) {
    gsum += gobs[j];
    double acc = 0.0;
    for (int s = 0; s < m; ++s) {
      const double z = (t_obs[j] - tl[s]) * inv_sigma;
      acc += al[s] * (2.0 * z * z * inv_sigma) * exp(-z * z);  // dK/dsigma = K 2 z^2 / sigma
    }
    t1 += gobs[j] * acc;
  }
  // condition vectors k^(d_j)(t_{i_j}) (kernel space)
  for (int e = tid; e < p * m; e += NYLS_BLOCK) {
    const int j = e / m, s = e - j * m;
    const double z = (nyls_grid_t(d, d.cond_i[j]) - tl[s]) * inv_sigma;
    double kd[NYLS_MAX_P + 1];
    nyls_kderiv(z, inv_sigma, kd);
    hk[j * NYLS_MAX_M + s] = nyls_pick(kd, d.cond_d[j]);
  }
  gsum = nyls_block_sum(gsum, red);
  t1 = nyls_block_sum(t1, red);
  __syncthreads();
  // 2. x_bar and mu = A^{-1} x_bar
  for (int a = tid; a < N; a += NYLS_BLOCK) {
    double val = 0.0;
    if (a < r) {
      for (int s = 0; s < m; ++s) val += W[s * m + a] * kb[s];
    } else if (a == m) {
      val = gsum;
    }
    R[a] = val;
    mu[a] = val;
  }
  __syncthreads();
  nyls_lu_solve(LU, N, N, piv, mu);

  const int ngc = NYLS_BLOCK / m, cs = tid % m, cg = tid / m;
  // 2b. refinement of mu: residual x_bar - A mu from one FP64 pass over the points
  for (int step = 0; step <= refine; ++step) {
    for (int s = tid; s < m; s += NYLS_BLOCK) {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc += W[s * m + k] * mu[k];
      be[s] = acc;
    }
    __syncthreads();
    if (step == refine) break;
    const double mub = mu[m];
    double nacc = 0.0, cacc = 0.0;
    for (int i0 = 0; i0 < n; i0 += TP) {
      __syncthreads();
      for (int e = tid; e < TP; e += NYLS_BLOCK) {
        const int i = i0 + e;
        const bool ok = i < n && !nyls_is_condition_point(d, i);
        double w[NYLS_MAX_P + 1];
        nyls_opweights(p, [&](int k) { return ok ? d.f[(size_t)(k - 1) * n + i] : 0.0; }, w);
#pragma unroll
        for (int q = 0; q <= NYLS_MAX_P; ++q) wq[e * (NYLS_MAX_P + 1) + q] = w[q];
      }
      __syncthreads();
      nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double zz, double ev) {
        double kd[NYLS_MAX_P + 1];
        nyls_kderiv_e(zz, ev, inv_sigma, kd);
        const double* w = wq + pt * (NYLS_MAX_P + 1);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q <= NYLS_MAX_P; ++q) v += w[q] * kd[q];
        P[pt * m + s] = v;
      });
      __syncthreads();
      {
        const int pt = tid / TPG, sub = tid % TPG;
        const int i = i0 + pt;
        double acc = 0.0;
        for (int s = sub; s < m; s += TPG) acc += P[pt * m + s] * be[s];
        for (int o = TPG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (sub == 0) {
          double nu = 0.0;
          if (i < n && !nyls_is_condition_point(d, i)) {
            const double c = -d.f[(size_t)(p - 1) * n + i];
            nu = acc + c * mub;
            cacc += c * nu;
          }
          pd[pt * 8] = nu;
        }
      }
      __syncthreads();
      if (cg < ngc)
        for (int pt = cg; pt < TP; pt += ngc) nacc += pd[pt * 8] * P[pt * m + cs];
    }
    part[tid] = cg < ngc ? nacc : 0.0;
    const double csum = nyls_block_sum(cacc, red);
    __syncthreads();
    for (int s = tid; s < m; s += NYLS_BLOCK) {
      double acc = 0.0;
      for (int gi = 0; gi < ngc; ++gi) acc += part[gi * m + s];
      an[s] = acc;
    }
    __syncthreads();
    // R = x_bar - A mu (A mu: mu_w + gamma W^T sum nu p + H mu_l ; gamma sum c nu + d^T mu_l ;
    //                         H^T mu_w + d mu_b)
    for (int a = tid; a < N; a += NYLS_BLOCK) {
      double amu;
      if (a < m) {
        amu = mu[a];
        if (a < r) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + a] * an[s];
          amu += gam * acc;
          for (int j = 0; j < p; ++j) amu += ws[L.H + j * m + a] * mu[m + 1 + j];
        }
      } else if (a == m) {
        amu = gam * csum;
        for (int j = 0; j < p; ++j) amu += (d.cond_d[j] == 0 ? 1.0 : 0.0) * mu[m + 1 + j];
      } else {
        const int j = a - m - 1;
        amu = d.cond_d[j] == 0 ? mu[m] : 0.0;
        for (int k = 0; k < r; ++k) amu += ws[L.H + j * m + k] * mu[k];
      }
      double xb = 0.0;
      if (a < r) { for (int s = 0; s < m; ++s) xb += W[s * m + a] * kb[s]; }
      else if (a == m) xb = gsum;
      part[NYLS_BLOCK + a] = xb - amu;
    }
    __syncthreads();
    for (int a = tid; a < N; a += NYLS_BLOCK) R[a] = part[NYLS_BLOCK + a];
    __syncthreads();
    nyls_lu_solve(LU, N, N, piv, R);
    double dn = 0.0, xn = 0.0;
    for (int a = tid; a < N; a += NYLS_BLOCK) {
      mu[a] += R[a];
      dn = fmax(dn, fabs(R[a]));
      xn = fmax(xn, fabs(mu[a]));
    }
    for (int o = 32; o > 0; o >>= 1) {
      dn = fmax(dn, __shfl_xor(dn, o));
      xn = fmax(xn, __shfl_xor(xn, o));
    }
    __syncthreads();
    if ((tid & 63) == 0) { part[tid >> 6] = dn; part[8 + (tid >> 6)] = xn; }
    __syncthreads();
    dn = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
    xn = fmax(fmax(part[8], part[9]), fmax(part[10], part[11]));
    __syncthreads();
    if (dn <= 1e-13 * xn) refine = step + 1;  // converged: the next iteration only forms beta
  }
  const double mub = mu[m];

  // 3. gradient pass over the points
  double sum_nu_e = 0.0, t2 = 0.0, aeacc = 0.0, anacc = 0.0;
  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    for (int e = tid; e < TP; e += NYLS_BLOCK) {
      const int i = i0 + e;
      double w[NYLS_MAX_P + 1];
      nyls_opweights(p, [&](int k) { return i < n ? d.f[(size_t)(k - 1) * n + i] : 0.0; }, w);
#pragma unroll
      for (int q = 0; q <= NYLS_MAX_P; ++q) wq[e * (NYLS_MAX_P + 1) + q] = w[q];
    }
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double zz, double ev) {
      double kd[NYLS_MAX_P + 1], ds[NYLS_MAX_P + 1];
      nyls_kderiv_e(zz, ev, inv_sigma, kd);
      kderiv_dsigma_e(zz, ev, inv_sigma, ds);
      const double* w = wq + pt * (NYLS_MAX_P + 1);
      double pv = 0.0, dpv = 0.0;
#pragma unroll
      for (int q = 0; q <= NYLS_MAX_P; ++q) {
        pv += w[q] * kd[q];
        dpv += w[q] * ds[q];
      }
      P[pt * m + s] = pv;
      DP[pt * m + s] = dpv;
#pragma unroll
      for (int q = 0; q < NYLS_MAX_P; ++q)
        if (q < p) KQ[(q * TP + pt) * m + s] = kd[q];
    });
    __syncthreads();
    {
      const int pt = tid / TPG, sub = tid % TPG;
      const int i = i0 + pt;
      double ap = 0.0, bp = 0.0, adp = 0.0, bdp = 0.0;
      double ak[NYLS_MAX_P], bk[NYLS_MAX_P];
#pragma unroll
      for (int q = 0; q < NYLS_MAX_P; ++q) { ak[q] = 0.0; bk[q] = 0.0; }
      for (int s = sub; s < m; s += TPG) {
        const double pv = P[pt * m + s], dpv = DP[pt * m + s];
        ap += al[s] * pv;
        bp += be[s] * pv;
        adp += al[s] * dpv;
        bdp += be[s] * dpv;
#pragma unroll
        for (int q = 0; q < NYLS_MAX_P; ++q)
          if (q < p) {
            const double kv = KQ[(q * TP + pt) * m + s];
            ak[q] += al[s] * kv;
            bk[q] += be[s] * kv;
          }
      }
      for (int o = TPG / 2; o > 0; o >>= 1) {
        ap += __shfl_xor(ap, o);
        bp += __shfl_xor(bp, o);
        adp += __shfl_xor(adp, o);
        bdp += __shfl_xor(bdp, o);
#pragma unroll
        for (int q = 0; q < NYLS_MAX_P; ++q) {
          ak[q] += __shfl_xor(ak[q], o);
          bk[q] += __shfl_xor(bk[q], o);
        }
      }
      if (sub == 0 && i < n) {
        const bool ok = !nyls_is_condition_point(d, i);
        double e = 0.0, nu = 0.0;
        if (ok) {
          const double c = -d.f[(size_t)(p - 1) * n + i];
          e = ap + c * b - d.r[i];
          nu = bp + c * mub;
          sum_nu_e += nu * e;
          t2 += e * bdp + nu * adp;
        }
        pd[pt * 8 + 0] = e;
        pd[pt * 8 + 1] = nu;
        if (dl_dr) dl_dr[d.goff + i] = ok ? gam * nu : 0.0;
        if (dl_df) {
#pragma unroll
          for (int k = 1; k <= NYLS_MAX_P; ++k) {
            if (k > p) break;
            const int q = p - k;
            double yq = 0.0, zq = 0.0;
#pragma unroll
            for (int qq = 0; qq < NYLS_MAX_P; ++qq)
              if (qq == q) { yq = ak[qq]; zq = bk[qq]; }
            if (q == 0) { yq += b; zq += mub; }
            dl_df[(size_t)(k - 1) * total + d.goff + i] = ok ? gam * (e * zq + nu * yq) : 0.0;
          }
        }
      } else if (sub == 0) {
        pd[pt * 8 + 0] = 0.0;
        pd[pt * 8 + 1] = 0.0;
      }
    }
    __syncthreads();
    if (cg < ngc)
      for (int pt = cg; pt < TP; pt += ngc) {
        aeacc += pd[pt * 8 + 0] * P[pt * m + cs];
        anacc += pd[pt * 8 + 1] * P[pt * m + cs];
      }
  }
  part[tid] = cg < ngc ? aeacc : 0.0;
  part[NYLS_BLOCK + tid] = cg < ngc ? anacc : 0.0;
  sum_nu_e = nyls_block_sum(sum_nu_e, red);
  t2 = nyls_block_sum(t2, red);
  __syncthreads();
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double a1 = 0.0, a2 = 0.0;
    for (int gi = 0; gi < ngc; ++gi) {
      a1 += part[gi * m + s];
      a2 += part[NYLS_BLOCK + gi * m + s];
    }
    ae[s] = a1;
    an[s] = a2;
  }
  __syncthreads();

  // 4. sigma: condition-row term, then the K_mm term
  double t3 = 0.0;
  for (int e = tid; e < p * m; e += NYLS_BLOCK) {
    const int j = e / m, s = e - j * m;
    const double z = (nyls_grid_t(d, d.cond_i[j]) - tl[s]) * inv_sigma;
    double ds[NYLS_MAX_P + 1];
    kderiv_dsigma(z, inv_sigma, ds);
    t3 += (xv[m + 1 + j] * be[s] + mu[m + 1 + j] * al[s]) * nyls_pick(ds, d.cond_d[j]);
  }
  t3 = nyls_block_sum(t3, red);
  // g1 = kbar - gamma sum nu p - H_k mu_lambda ; g2 = gamma sum e p + H_k lambda
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double g1 = kb[s] - gam * an[s], g2 = gam * ae[s];
    for (int j = 0; j < p; ++j) {
      g1 -= hk[j * NYLS_MAX_M + s] * mu[m + 1 + j];
      g2 += hk[j * NYLS_MAX_M + s] * xv[m + 1 + j];
    }
    kb[s] = g1;
    ae[s] = g2;
  }
  __syncthreads();
  for (int k = tid; k < m; k += NYLS_BLOCK) {
    double u1 = 0.0, u2 = 0.0;
    for (int s = 0; s < m; ++s) {
      u1 += U[s * m + k] * kb[s];
      u2 += U[s * m + k] * ae[s];
    }
    ug[k] = u1;
    ug[NYLS_MAX_M + k] = u2;
  }
  __syncthreads();
  // E = dK/dsigma U[:, :r] (global scratch), then D_kl = U[:, k]^T E[:, l]
  double* E = ws + L.tmp;
  for (int e = tid; e < m * r; e += NYLS_BLOCK) {
    const int a = e / r, l = e - a * r;
    double acc = 0.0;
    for (int s = 0; s < m; ++s) {
      const double z = (tl[a] - tl[s]) * inv_sigma;
      acc += (2.0 * z * z * inv_sigma) * exp(-z * z) * U[s * m + l];
    }
    E[a * m + l] = acc;
  }
  __syncthreads();
  double tk = 0.0;
  for (int e = tid; e < m * r; e += NYLS_BLOCK) {
    const int k = e / r, l = e - k * r;
    double dkl = 0.0;
    for (int a = 0; a < m; ++a) dkl += U[a * m + k] * E[a * m + l];
    const double ll = lamv[l], lk = lamv[k];
    const double qb = 0.5 * sqrt(ll) * (ug[k] * xv[l] - ug[NYLS_MAX_M + k] * mu[l]);
    const double fkl = (k < r) ? -1.0 / (lk * ll) : 1.0 / (ll * (ll - lk));
    tk += (k < r ? 1.0 : 2.0) * fkl * qb * dkl;
  }
  tk = nyls_block_sum(tk, red);
  if (tid == 0) {
    if (dl_dgamma) dl_dgamma[inst] = -sum_nu_e;
    if (dl_dsigma) dl_dsigma[inst] = t1 - gam * t2 - t3 + tk;
  }
  if (dl_dv)
    for (int j = tid; j < NYLS_MAX_P; j += NYLS_BLOCK) dl_dv[inst * NYLS_MAX_P + j] = j < p ? mu[m + 1 + j] : 0.0;
  for (int a = tid; a < N; a += NYLS_BLOCK) ws[L.mu + a] = mu[a];
}

size_t backward_lds_bytes(int maxm, int maxp) {
  const size_t common = (6 * NYLS_MAX_M + NYLS_MAX_P * NYLS_MAX_M + 3 * 136 + 2 * NYLS_MAX_M +
                         2 * NYLS_BLOCK + 16 + TP * 8 + TP * (NYLS_MAX_P + 1)) * sizeof(double) +
                        136 * sizeof(int);
  const size_t tiles = (size_t)(2 + maxp) * TP * maxm * sizeof(double);
  return common + tiles;
}

}  // namespace

struct nyls_plan;
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl);

extern "C" int nyls_backward(const nyls_plan* pl, const double* t_obs, const int64_t* obs_off,
                             const double* dl_dyobs, double* dl_df, double* dl_dr, double* dl_dv,
                             double* dl_dsigma, double* dl_dgamma, void* ws, hipStream_t stream) {
  if (!pl || !t_obs || !obs_off || !dl_dyobs || !ws) return NYLS_E_NULL;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.mode == NYLS_FP64_EXPLICIT) return NYLS_E_MODE;
  const int refine = 3;  // at most; stops once the correction is at rounding level
  const size_t lds = backward_lds_bytes(pv.maxm, pv.maxp);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_backward),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  nyls_prof_begin(NYLS_K_BACKWARD, stream);
  hipLaunchKernelGGL(k_backward, dim3(pv.batch), dim3(NYLS_BLOCK), lds, stream, pv.d_desc,
                     static_cast<double*>(ws), refine, t_obs, obs_off, dl_dyobs, dl_df, dl_dr, dl_dv,
                     dl_dsigma, dl_dgamma, pv.total, pv.maxm);
  nyls_prof_end(NYLS_K_BACKWARD, stream);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}
