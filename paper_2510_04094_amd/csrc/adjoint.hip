// Adjoint of the Lemma 1 solve (Sec. 3.1): gradients of a loss l(y_hat(s_j)) with respect
// to the ODE data f_k(t_i), r(t_i), the condition values v_j, gamma and sigma, reusing the
// factorisation nyls_solve left in the workspace.
//
// With x = (omega, b, lambda) solving A x = rhs (A symmetric), alpha = W omega and the ODE
// residual e_i = p_i^T alpha + c_i b - r_i:
//   1. x_bar = (W^T kbar, sum_j g_j, 0), kbar = sum_j g_j k_m(s_j);  mu = A^{-1} x_bar
//      (plus FP64 iterative refinement of mu: the stored factors are of the FP32 or the
//      kernel-space FP64 Gram, which lose accuracy for ill-conditioned K_mm);
//   2. beta = W mu_omega, nu_i = beta^T p_i + c_i mu_b,
//      yh^(q)_i = alpha^T k^(q)_i + [q=0] b,  zh^(q)_i = beta^T k^(q)_i + [q=0] mu_b;
//   3. dl/df_k(t_i) = gamma (e_i zh^(p-k)_i + nu_i yh^(p-k)_i), dl/dr(t_i) = gamma nu_i,
//      dl/dv_j = mu_lambda_j, dl/dgamma = -sum_i nu_i e_i = mu_omega^T omega / gamma
//      (the KKT rows give gamma G^T e = -(omega + H lambda), gamma c^T e = -delta^T lambda
//      and H^T mu_omega + delta mu_b = 0; the sum over the points cancels by orders of
//      magnitude at large gamma, the product of the two solution vectors does not);
//   4. dl/dsigma = (terms through k^(q)(.) at fixed W, closed-form d/dsigma of the kernel
//      derivatives) + (the K_mm term): the problem depends on W only via Q = W W^T =
//      f(K_mm), f(l) = 1/l above the cut-off, so with dl/dW = g1 omega^T - g2 mu_omega^T
//      (g1 = kbar - gamma sum nu_i p_i - H_k mu_lambda, g2 = gamma sum e_i p_i + H_k lambda)
//      the spectral (Daleckii-Krein) derivative gives
//      sum_{l < r} [ sum_{k < r} F_kl Qb_kl D_kl + 2 sum_{k >= r} F_kl Qb_kl D_kl ],
//      Qb_kl = sqrt(lam_l)/2 ((U^T g1)_k omega_l - (U^T g2)_k mu_l),  D = U^T dK_mm/dsigma U,
//      F_kl = -1/(lam_k lam_l) (k < r), 1/(lam_l (lam_l - lam_k)) (k >= r).
//
// One wavefront per instance with the lane layout of nyls_walk.h (the refinement pass of
// the forward solve has the same structure).  The gradient pass forms, per (point, landmark)
// pair, p_i, d p_i / d sigma and k^(q)_i (q < p) from the Hermite factors, reduces their
// dot products with alpha and beta over the landmarks, and keeps sum_i e_i p_i and
// sum_i nu_i p_i in registers.  d/dsigma of the q-th kernel derivative h_q e is
// -e (q h_q / sigma + z h_{q+1}) (h_q as in nyls_hfac, z = (t - t_s) / sigma = -sigma g / 2).
#include "nyls_dense.h"
#include "nyls_walk.h"

namespace {

template <int NB, int P, bool EX>
__global__ __launch_bounds__(64) void k_backward(
    const nyls_desc* __restrict__ desc, const int32_t* __restrict__ order,
    double* __restrict__ wsbase, int refine, const double* __restrict__ t_obs,
    const int64_t* __restrict__ obs_off, const double* __restrict__ gobs,
    double* __restrict__ dl_df, double* __restrict__ dl_dr, double* __restrict__ dl_dv,
    double* __restrict__ dl_dsigma, double* __restrict__ dl_dgamma, int64_t total) {
  constexpr int ML = 16 * NB;   // landmark slots
  constexpr int Q = 4 + 2 * P;  // dot products per point in the gradient pass
  constexpr int NKL = ML + 1 + P;
  // LDS: the gradient pass's reduction tile (Q quantities x 16 points) shares its space with
  // the small per-instance vectors, which the mu refinement uses next to tile rows 0..15
  // (one quantity) and which are parked in the workspace while the gradient pass runs.  This
  // keeps the workgroup under a quarter of the 160 KiB of LDS per compute unit, so LDS does
  // not limit the number of resident wavefronts below what the registers allow.
  constexpr int TILE = Q * 16 * NYLS_WALK_PAD;
  constexpr int VOFF = 16 * NYLS_WALK_PAD;
  constexpr int VLEN = 6 * ML + P * ML + 4 * NKL;
  __shared__ __align__(16) double lds[TILE > VOFF + VLEN ? TILE : VOFF + VLEN];
  __shared__ double bc[2 * 16];
  __shared__ int piv[NKL];
  double* const tile = lds;
  double* const tl = lds + VOFF;
  double* const kb = tl + ML;
  double* const ae = kb + ML;
  double* const an = ae + ML;
  double* const ug1 = an + ML;
  double* const ug2 = ug1 + ML;
  double* const hkv = ug2 + ML;  // hkv[j * ML + s]: k^(d_j)(t_{i_j}) at landmark s
  double* const xv = hkv + P * ML;
  double* const mu = xv + NKL;
  double* const R = mu + NKL;
  double* const xb = R + NKL;

  const int inst = order ? order[blockIdx.x] : (int)blockIdx.x;
  const nyls_desc& d = desc[inst];
  if (d.p != P || d.rec != (EX ? 0 : 1) || nyls_slot_blocks(d.m) != NB || (d.flags & NYLS_DF_SPLIT))
    return;  // another launch handles this instance (split instances: adjoint_split.hip)
  const int m = d.m, n = d.n;
  const int N = m + 1 + P;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* U = ws + L.U;
  const double* lamv = ws + L.lam;
  const double* LU = ws + L.lu;
  const double* Hc = ws + L.H;
  const int lane = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma;

  nyls_walk<NB, EX> wk;
  wk.init(d, lane);
  nyls_cpts cpt;
  cpt.init(d);
  const int sl = wk.sl, ph = wk.ph;
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  nyls_oppoly<P> op;
  op.init(inv_s2);
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);

  for (int s = lane; s < m; s += 64) tl[s] = nyls_grid_t(d, d.lidx[s]);
  for (int a = lane; a < N; a += 64) {
    xv[a] = ws[L.x + a];
    piv[a] = (int)ws[L.piv + a];
  }
  double alv[NB], bev[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) alv[b] = wk.lv[b] ? ws[L.alpha + 16 * b + sl] : 0.0;
  __syncthreads();
  const double bias = xv[m];

  // 1. observations (phase ph takes every fourth one): kbar, sum g, and the direct sigma
  //    term sum_j g_j alpha^T dk(s_j)/dsigma, dK/dsigma = K 2 z^2 / sigma
  const int64_t j0 = obs_off[inst], j1 = obs_off[inst + 1];
  double t1 = 0.0, gsum = 0.0;
  {
    double kba[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) kba[b] = 0.0;
    for (int64_t j = j0 + ph; j < j1; j += 4) {
      const double tj = t_obs[j], gj = gobs[j];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (!wk.lv[b]) continue;
        const double z = (tj - tl[16 * b + sl]) * inv_sigma;
        const double e = exp(-z * z);
        kba[b] += gj * e;
        t1 += gj * alv[b] * (2.0 * z * z * inv_sigma) * e;
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const double v = nyls_walk_fold(kba[b]);
      if (ph == 0 && wk.lv[b]) kb[16 * b + sl] = v;
    }
    for (int64_t j = j0 + lane; j < j1; j += 64) gsum += gobs[j];
    t1 = nyls_wave_sum(t1);
    gsum = nyls_wave_sum(gsum);
  }
  // condition vectors k^(d_j)(t_{i_j}) (kernel space)
  for (int e = lane; e < P * m; e += 64) {
    const int j = e / m, s = e - j * m;
    const double z = (nyls_grid_t(d, d.cond_i[j]) - tl[s]) * inv_sigma;
    double h[P + 2];
    nyls_hfac<P>(-2.0 * inv_sigma * z, inv_s2, h);
    double hv = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q)
      if (q == d.cond_d[j]) hv = h[q];
    hkv[j * ML + s] = hv * exp(-z * z);
  }
  __syncthreads();

  // 2. x_bar and mu = A^{-1} x_bar
  for (int a = lane; a < N; a += 64) {
    double val = 0.0;
    if (a < r) {
      for (int s = 0; s < m; ++s) val += W[s * m + a] * kb[s];
    } else if (a == m) {
      val = gsum;
    }
    xb[a] = val;
    mu[a] = val;
  }
  __syncthreads();
  if (N <= 64) nyls_lu_solve_wave(LU, N, piv, mu);
  else nyls_lu_solve_w(LU, N, N, piv, mu);
  auto beta_from_mu = [&]() {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int s = 16 * b + sl;
      double acc = 0.0;
      if (wk.lv[b])
        for (int k = 0; k < r; ++k) acc += W[s * m + k] * mu[k];
      bev[b] = acc;
    }
  };
  beta_from_mu();

  // 2b. refinement of mu: the residual x_bar - A mu from one FP64 pass over the points
  //     (nu_i = p_i^T beta + c_i mu_b, A mu = (mu_w + gamma W^T sum nu p + H mu_l,
  //     gamma sum c nu + delta^T mu_l, H^T mu_w + delta mu_b)).  Stops when the correction
  //     is below 1e-8 of mu (omega and b parts; three orders below what the 1e-5 gradient
  //     accuracy needs) or stops halving (the FP64 residual of this system has a floor of
  //     about 1e-9 .. 1e-7 of mu for ill-conditioned K_mm, which further passes do not lower).
  double dprev = 0.0;
  int passes = 0;
  for (int step = 0; step < refine; ++step) {
    ++passes;
    const double mub = mu[m];
    double zacc[NB], sacc = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) zacc[b] = 0.0;
    struct stage {
      double f[P][4];
      double c;
    };
    auto load = [&](int i0, stage& st) {
#pragma unroll
      for (int k = 0; k < P; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) st.f[k][j] = nyls_bload(fr, (k * n + i0 + 4 * j + ph) * 8);
      st.c = -nyls_bload(fr, ((P - 1) * n + i0 + (lane & 15)) * 8);
    };
    auto body = [&](int i0, const stage& st) {
      wk.advance(d, i0);
      double cj[4][P];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double f[P];
#pragma unroll
        for (int k = 0; k < P; ++k) f[k] = st.f[k][j];
        op.coef(f, cj[j]);
      }
      double pe[NB][4];
      double acc = 0.0;
      wk.chunk(
          d, i0,
          [&](int b, int j, double g, double e) {
            pe[b][j] = e * nyls_horner<P>(g, cj[j]);
            acc += bev[b] * pe[b][j];
          },
          [&](int j) {
            nyls_walk_put(tile, lane, 0, j, acc);
            acc = 0.0;
          });
      double tot[1];
      nyls_walk_sum<1>(tile, lane, tot);
      const int ip = i0 + (lane & 15);
      const bool okp = ip < n && !cpt.has(ip);
      const double nu = okp ? tot[0] + st.c * mub : 0.0;
      if (lane < 16) sacc += st.c * nu;
      const double w1[1] = {nu};
      double nj[1][4];
      nyls_walk_bcast<1>(w1, bc, lane, nj);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) zacc[b] += nj[0][j] * pe[b][j];
    };
    stage sa, sb;
    load(0, sa);
    for (int i0 = 0; i0 < n; i0 += 32) {
      load(i0 + 16, sb);
      body(i0, sa);
      if (i0 + 16 >= n) break;
      load(i0 + 32, sa);
      body(i0 + 16, sb);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const double v = nyls_walk_fold(zacc[b]);
      if (ph == 0 && wk.lv[b]) an[16 * b + sl] = v;
    }
    const double csum = nyls_wave_sum(sacc);
    __syncthreads();
    for (int a = lane; a < N; a += 64) {
      double amu;
      if (a < m) {
        amu = mu[a];
        if (a < r) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + a] * an[s];
          amu += gam * acc;
          for (int j = 0; j < P; ++j) amu += Hc[j * m + a] * mu[m + 1 + j];
        }
      } else if (a == m) {
        amu = gam * csum;
        for (int j = 0; j < P; ++j) amu += (d.cond_d[j] == 0 ? 1.0 : 0.0) * mu[m + 1 + j];
      } else {
        const int j = a - m - 1;
        amu = d.cond_d[j] == 0 ? mu[m] : 0.0;
        for (int k = 0; k < r; ++k) amu += Hc[j * m + k] * mu[k];
      }
      R[a] = xb[a] - amu;
    }
    __syncthreads();
    if (N <= 64) nyls_lu_solve_wave(LU, N, piv, R);
    else nyls_lu_solve_w(LU, N, N, piv, R);
    double dsq = 0.0, xsq = 0.0;
    for (int k = lane; k < r; k += 64) {
      dsq += R[k] * R[k];
      xsq += mu[k] * mu[k];
    }
    const double dn = sqrt(nyls_wave_sum(dsq)) + fabs(R[m]);
    const double xn = sqrt(nyls_wave_sum(xsq)) + fabs(mu[m]);
    for (int a = lane; a < N; a += 64) mu[a] += R[a];
    __syncthreads();
    beta_from_mu();
    // Stop once this correction, or the next one predicted from the contraction seen so
    // far (this correction over the previous one, or over mu itself for the first), is
    // below 1e-8 |mu|, or once the corrections stop halving.
    const bool stalled = step > 0 && dn > 0.5 * dprev;
    const double pred = dn * (dn / (step > 0 ? dprev : xn));
    dprev = dn;
    if (dn <= 1e-8 * xn || pred <= 1e-8 * xn || stalled) break;
  }
  const double mub = mu[m];

  // park kb, hk and mu in the workspace (x stays there) while the tile covers them
  for (int s = lane; s < m; s += 64) {
    ws[L.beta + s] = kb[s];
    for (int j = 0; j < P; ++j) ws[L.acc + j * m + s] = hkv[j * ML + s];
  }
  for (int a = lane; a < N; a += 64) ws[L.mu + a] = mu[a];
  __syncthreads();

  // 3. gradient pass
  double aeacc[NB], anacc[NB], t2 = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) aeacc[b] = anacc[b] = 0.0;
  {
    struct stage {
      double f[P][4];
      double r, c;
    };
    auto load = [&](int i0, stage& st) {
#pragma unroll
      for (int k = 0; k < P; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) st.f[k][j] = nyls_bload(fr, (k * n + i0 + 4 * j + ph) * 8);
      const int ip = i0 + (lane & 15);
      st.r = nyls_bload(rr, ip * 8);
      st.c = -nyls_bload(fr, ((P - 1) * n + ip) * 8);
    };
    const double half_sigma = 0.5 * d.sigma;
    auto body = [&](int i0, const stage& st) {
      wk.advance(d, i0);
      // per point: p_i = e poly(g), d p_i / d sigma = e (sigma / 2) D(g); the coefficients
      // of point j are formed when its first slot is emitted (one point's set is live)
      double cj[P], dj[P + 2];
      double pe[NB][4];
      double acc[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) acc[q] = 0.0;
      wk.chunk(
          d, i0,
          [&](int b, int j, double g, double e) {
            if (b == 0) {
              double f[P];
#pragma unroll
              for (int k = 0; k < P; ++k) f[k] = st.f[k][j];
              op.coef(f, cj);
              op.dcoef(f, dj);
            }
            double h[P + 2];
            nyls_hfac<P>(g, inv_s2, h);  // only h_q, q < P, are used
            const double pv = e * nyls_horner<P>(g, cj);
            const double dpv = e * nyls_horner<P + 2>(g, dj);  // without the sigma / 2
            pe[b][j] = pv;
            acc[0] += alv[b] * pv;
            acc[1] += bev[b] * pv;
            acc[2] += alv[b] * dpv;
            acc[3] += bev[b] * dpv;
#pragma unroll
            for (int q = 0; q < P; ++q) {
              const double kq = e * h[q];
              acc[4 + q] += alv[b] * kq;
              acc[4 + P + q] += bev[b] * kq;
            }
          },
          [&](int j) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              nyls_walk_put(tile, lane, q, j, acc[q]);
              acc[q] = 0.0;
            }
          });
      double tot[Q];
      nyls_walk_sum<Q>(tile, lane, tot);
      const int ip = i0 + (lane & 15);
      const bool okp = ip < n && !cpt.has(ip);
      const double ei = okp ? tot[0] + st.c * bias - st.r : 0.0;
      const double nui = okp ? tot[1] + st.c * mub : 0.0;
      if (lane < 16 && ip < n) {
        t2 += half_sigma * (ei * tot[3] + nui * tot[2]);
        if (dl_dr) dl_dr[d.goff + ip] = gam * nui;
        if (dl_df) {
#pragma unroll
          for (int k = 1; k <= P; ++k) {
            const int q = P - k;
            const double yq = tot[4 + q] + (q == 0 ? bias : 0.0);
            const double zq = tot[4 + P + q] + (q == 0 ? mub : 0.0);
            dl_df[(size_t)(k - 1) * total + d.goff + ip] = gam * (ei * zq + nui * yq);
          }
        }
      }
      const double w2[2] = {ei, nui};
      double en[2][4];
      nyls_walk_bcast<2>(w2, bc, lane, en);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          aeacc[b] += en[0][j] * pe[b][j];
          anacc[b] += en[1][j] * pe[b][j];
        }
    };
    stage sa, sb;
    load(0, sa);
    for (int i0 = 0; i0 < n; i0 += 32) {
      load(i0 + 16, sb);
      body(i0, sa);
      if (i0 + 16 >= n) break;
      load(i0 + 32, sa);
      body(i0 + 16, sb);
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double va = nyls_walk_fold(aeacc[b]), vn = nyls_walk_fold(anacc[b]);
    if (ph == 0 && wk.lv[b]) {
      ae[16 * b + sl] = va;
      an[16 * b + sl] = vn;
    }
  }
  t2 = nyls_wave_sum(t2);
  __syncthreads();
  for (int s = lane; s < m; s += 64) {
    tl[s] = nyls_grid_t(d, d.lidx[s]);
    kb[s] = ws[L.beta + s];
    for (int j = 0; j < P; ++j) hkv[j * ML + s] = ws[L.acc + j * m + s];
  }
  for (int a = lane; a < N; a += 64) {
    xv[a] = ws[L.x + a];
    mu[a] = ws[L.mu + a];
  }
  __syncthreads();

  // 4. sigma: condition-row term (phase-0 lanes own the landmarks), then the K_mm term
  double t3 = 0.0;
  if (ph == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (!wk.lv[b]) continue;
      const int s = 16 * b + sl;
      for (int j = 0; j < P; ++j) {
        const double z = (nyls_grid_t(d, d.cond_i[j]) - tl[s]) * inv_sigma;
        const double e = exp(-z * z);
        double h[P + 2];
        nyls_hfac<P>(-2.0 * inv_sigma * z, inv_s2, h);
        double ds = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q)
          if (q == d.cond_d[j]) ds = -e * (q * inv_sigma * h[q] + z * h[q + 1]);
        t3 += (xv[m + 1 + j] * bev[b] + mu[m + 1 + j] * alv[b]) * ds;
      }
    }
  }
  t3 = nyls_wave_sum(t3);
  // g1 = kbar - gamma sum nu p - H_k mu_lambda ; g2 = gamma sum e p + H_k lambda
  for (int s = lane; s < m; s += 64) {
    double g1 = kb[s] - gam * an[s], g2 = gam * ae[s];
    for (int j = 0; j < P; ++j) {
      g1 -= hkv[j * ML + s] * mu[m + 1 + j];
      g2 += hkv[j * ML + s] * xv[m + 1 + j];
    }
    kb[s] = g1;
    ae[s] = g2;
  }
  __syncthreads();
  for (int k = lane; k < m; k += 64) {
    double u1 = 0.0, u2 = 0.0;
    for (int s = 0; s < m; ++s) {
      u1 += U[s * m + k] * kb[s];
      u2 += U[s * m + k] * ae[s];
    }
    ug1[k] = u1;
    ug2[k] = u2;
  }
  // dK_mm/dsigma into the (no longer needed) Gram block, then E = dK U[:, :r] into tmp
  double* dK = ws + L.gram;
  double* E = ws + L.tmp;
  for (int e = lane; e < m * m; e += 64) {
    const int a = e / m, s = e - a * m;
    const double z = (tl[a] - tl[s]) * inv_sigma;
    dK[e] = (2.0 * z * z * inv_sigma) * exp(-z * z);
  }
  __syncthreads();
  for (int e = lane; e < m * r; e += 64) {
    const int a = e / r, l = e - a * r;
    double acc = 0.0;
    for (int s = 0; s < m; ++s) acc += dK[a * m + s] * U[s * m + l];
    E[a * m + l] = acc;
  }
  __syncthreads();
  double tk = 0.0;
  for (int e = lane; e < m * r; e += 64) {
    const int k = e / r, l = e - k * r;
    double dkl = 0.0;
    for (int a = 0; a < m; ++a) dkl += U[a * m + k] * E[a * m + l];
    const double ll = lamv[l], lk = lamv[k];
    const double qb = 0.5 * sqrt(ll) * (ug1[k] * xv[l] - ug2[k] * mu[l]);
    const double fkl = (k < r) ? -1.0 / (lk * ll) : 1.0 / (ll * (ll - lk));
    tk += (k < r ? 1.0 : 2.0) * fkl * qb * dkl;
  }
  tk = nyls_wave_sum(tk);
  double mw = 0.0;
  for (int k = lane; k < r; k += 64) mw += mu[k] * xv[k];
  mw = nyls_wave_sum(mw);
  if (lane == 0) {
    ws[L.info + 6] = (double)passes;
    if (dl_dgamma) dl_dgamma[inst] = mw / gam;
    if (dl_dsigma) dl_dsigma[inst] = t1 - gam * t2 - t3 + tk;
  }
  if (dl_dv && lane < NYLS_MAX_P) dl_dv[inst * NYLS_MAX_P + lane] = lane < P ? mu[m + 1 + lane] : 0.0;
  for (int a = lane; a < N; a += 64) ws[L.mu + a] = mu[a];
}

template <int NB, bool EX>
void launch_nbx(const nyls_plan_view& pv, double* ws, int refine, const double* t_obs,
                const int64_t* obs_off, const double* g, double* dl_df, double* dl_dr,
                double* dl_dv, double* dl_ds, double* dl_dg, hipStream_t st) {
  const dim3 grid(pv.batch), block(64);
  if (pv.p_mask & 2)
    hipLaunchKernelGGL((k_backward<NB, 1, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws,
                       refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, pv.total);
  if (pv.p_mask & 4)
    hipLaunchKernelGGL((k_backward<NB, 2, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws,
                       refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, pv.total);
  if (pv.p_mask & 8)
    hipLaunchKernelGGL((k_backward<NB, 3, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws,
                       refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, pv.total);
  if (pv.p_mask & 16)
    hipLaunchKernelGGL((k_backward<NB, 4, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws,
                       refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, pv.total);
}

template <int NB>
void launch_nb(const nyls_plan_view& pv, double* ws, int refine, const double* t_obs,
               const int64_t* obs_off, const double* g, double* dl_df, double* dl_dr,
               double* dl_dv, double* dl_ds, double* dl_dg, hipStream_t st) {
  if (pv.rec_mask & 2)
    launch_nbx<NB, false>(pv, ws, refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, st);
  if (pv.rec_mask & 1)
    launch_nbx<NB, true>(pv, ws, refine, t_obs, obs_off, g, dl_df, dl_dr, dl_dv, dl_ds, dl_dg, st);
}

}  // namespace

struct nyls_plan;
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl);
hipError_t nyls_launch_backward_split(const nyls_plan_view& pv, double* ws, int refine,
                                      const double* t_obs, const int64_t* obs_off, const double* g,
                                      double* dl_df, double* dl_dr, double* dl_dv, double* dl_ds,
                                      double* dl_dg, hipStream_t st);

extern "C" int nyls_backward(const nyls_plan* pl, const double* t_obs, const int64_t* obs_off,
                             const double* dl_dyobs, double* dl_df, double* dl_dr, double* dl_dv,
                             double* dl_dsigma, double* dl_dgamma, void* ws, hipStream_t stream) {
  if (!pl || !t_obs || !obs_off || !dl_dyobs || !ws) return NYLS_E_NULL;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.mode == NYLS_FP64_EXPLICIT) return NYLS_E_MODE;
  const int refine = 3;  // at most; stops once the correction is at rounding level
  double* w = static_cast<double*>(ws);
  nyls_prof_begin(NYLS_K_BACKWARD, stream);
  if (pv.nb_mask & 4)
    launch_nb<2>(pv, w, refine, t_obs, obs_off, dl_dyobs, dl_df, dl_dr, dl_dv, dl_dsigma, dl_dgamma, stream);
  if (pv.nb_mask & 16)
    launch_nb<4>(pv, w, refine, t_obs, obs_off, dl_dyobs, dl_df, dl_dr, dl_dv, dl_dsigma, dl_dgamma, stream);
  if (pv.nb_mask & 256)
    launch_nb<8>(pv, w, refine, t_obs, obs_off, dl_dyobs, dl_df, dl_dr, dl_dv, dl_dsigma, dl_dgamma, stream);
  if (pv.n_split)
    (void)nyls_launch_backward_split(pv, w, refine, t_obs, obs_off, dl_dyobs, dl_df, dl_dr, dl_dv,
                                     dl_dsigma, dl_dgamma, stream);
  nyls_prof_end(NYLS_K_BACKWARD, stream);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}
