// Adjoint of instances split over point chunks (NYLS_DF_SPLIT): the computation of k_backward
// (adjoint.hip, Sec. 3.1 Lemma 1 transposed) cut at its passes over the grid, so that each pass
// runs one workgroup per chunk of d.chunk grid points and one wavefront per instance adds the
// chunks' partial sums in chunk order (results do not depend on scheduling):
//   k_bws_setup       observations (kbar, sum g, the direct sigma term), condition vectors,
//                     x_bar and mu = A^{-1} x_bar from the stored factors;
//   k_bws_mu_pass     per chunk: nu_i = beta^T p_i + c_i mu_b, sums of nu_i p_i and c_i nu_i;
//   k_bws_mu_combine  the refinement step of mu (residual x_bar - A mu, solve, stopping rule);
//   k_bws_grad_pass   per chunk: the gradient pass (dl/df, dl/dr at its points; sums of e_i p_i,
//                     nu_i p_i and the sigma terms);
//   k_bws_final       the sigma terms through K_mm, dl/dgamma, dl/dv.
// Workspace of a split instance during nyls_backward (regions the solve no longer needs):
//   L.beta [m] kbar;  L.acc [P m] condition vectors;  L.mu [N] mu;  L.tmp [N] x_bar, then the
//   state (L.tmp + N ..); per chunk the mu-pass sums in the pass-partial area and the
//   gradient-pass sums in the Gram-partial area of the split solve.
#include "nyls_dense.h"
#include "nyls_walk.h"

namespace {

constexpr int NK = NYLS_MAX_M + 1 + NYLS_MAX_P;
enum { BS_DONE = 0, BS_DPREV, BS_PASSES, BS_T1, BS_GSUM, BS_COUNT };

template <int P>
__device__ inline bool takes(const nyls_desc& d) {
  return (d.flags & NYLS_DF_SPLIT) && d.p == P;
}

// beta = W mu for this lane's landmark slots (s0 + 16 b + sl)
template <int NB>
__device__ inline void beta_slots(const double* W, const double* mu, int m, int r, int s0, int sl,
                                  const bool (&lv)[NB], double (&bev)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int s = s0 + 16 * b + sl;
    double acc = 0.0;
    if (lv[b])
      for (int k = 0; k < r; ++k) acc += W[s * m + k] * mu[k];
    bev[b] = acc;
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_bws_setup(const nyls_desc* __restrict__ desc,
                                                  double* __restrict__ wsbase,
                                                  const double* __restrict__ t_obs,
                                                  const int64_t* __restrict__ obs_off,
                                                  const double* __restrict__ gobs) {
  __shared__ double tl[NYLS_MAX_M], kb[NYLS_MAX_M], mu[NK];
  __shared__ int piv[NK];
  const int inst = (int)blockIdx.x;
  const nyls_desc& d = desc[inst];
  if (!takes<P>(d)) return;
  const int m = d.m, N = m + 1 + P, lane = threadIdx.x;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const int r = (int)ws[L.info + 0];
  const double inv_sigma = 1.0 / d.sigma, inv_s2 = inv_sigma * inv_sigma;
  for (int s = lane; s < m; s += 64) tl[s] = nyls_grid_t(d, d.lidx[s]);
  for (int a = lane; a < N; a += 64) piv[a] = (int)ws[L.piv + a];
  __syncthreads();
  // observations: kbar_s = sum_j g_j k(s_j, t_s), sum g, sum_j g_j alpha^T dk(s_j)/dsigma
  const int64_t j0 = obs_off[inst], j1 = obs_off[inst + 1];
  double t1 = 0.0, gsum = 0.0;
  for (int s = lane; s < m; s += 64) {
    const double al = ws[L.alpha + s];
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
      const double z = (t_obs[j] - tl[s]) * inv_sigma;
      const double e = exp(-z * z);
      acc += gobs[j] * e;
      t1 += gobs[j] * al * (2.0 * z * z * inv_sigma) * e;
    }
    kb[s] = acc;
    ws[L.beta + s] = acc;
  }
  for (int64_t j = j0 + lane; j < j1; j += 64) gsum += gobs[j];
  t1 = nyls_wave_sum(t1);
  gsum = nyls_wave_sum(gsum);
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
    ws[L.acc + e] = hv * exp(-z * z);
  }
  __syncthreads();
  // x_bar and mu = A^{-1} x_bar
  for (int a = lane; a < N; a += 64) {
    double val = 0.0;
    if (a < r) {
      for (int s = 0; s < m; ++s) val += W[s * m + a] * kb[s];
    } else if (a == m) {
      val = gsum;
    }
    ws[L.tmp + a] = val;
    mu[a] = val;
  }
  __syncthreads();
  nyls_lu_solve_w(ws + L.lu, N, N, piv, mu);
  for (int a = lane; a < N; a += 64) ws[L.mu + a] = mu[a];
  if (lane == 0) {
    double* st = ws + L.tmp + N;
    st[BS_DONE] = 0.0;
    st[BS_DPREV] = 0.0;
    st[BS_PASSES] = 0.0;
    st[BS_T1] = t1;
    st[BS_GSUM] = gsum;
  }
}

// G = 2: wide bases, two wavefronts per chunk (one per half of the landmark slots), the
// per-point sums joined through LDS as in the forward passes.
template <int NB, int P, bool EX, int G = 1>
__global__ __launch_bounds__(64 * G) void k_bws_mu_pass(const nyls_desc* __restrict__ desc,
                                                        double* __restrict__ wsbase) {
  __shared__ __align__(16) double tiles[G][16 * NYLS_WALK_PAD];
  __shared__ double bcs[G][16];
  __shared__ double xw[G > 1 ? 2 * G * 16 : 1];
  const nyls_desc& d = desc[blockIdx.x];
  if (!takes<P>(d) || d.rec != (EX ? 0 : 1) || nyls_slot_blocks(d.m) != NB * G) return;
  const int c = (int)blockIdx.y;
  if (c >= d.nchunks) return;
  const int m = d.m, n = d.n, N = m + 1 + P;
  const int lane = threadIdx.x & 63, grp = G > 1 ? (int)(threadIdx.x >> 6) : 0;
  const int s0 = 16 * NB * grp;
  double* const tile = tiles[grp];
  double* const bc = bcs[grp];
  int parity = 0;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  if (ws[L.tmp + N + BS_DONE] != 0.0) return;
  const int r = (int)ws[L.info + 0];
  const int ibeg = c * d.chunk, iend = min(n, ibeg + d.chunk);
  nyls_walk<NB, EX> wk;
  wk.init(d, lane, s0);
  nyls_cpts cpt;
  cpt.init(d);
  const int ph = wk.ph;
  const double inv_s2 = wk.inv_sigma * wk.inv_sigma;
  nyls_oppoly<P> op;
  op.init(inv_s2);
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8);
  const double* mu = ws + L.mu;
  double bev[NB];
  beta_slots<NB>(ws + L.W, mu, m, r, s0, wk.sl, wk.lv, bev);
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
    if constexpr (G > 1) {
      nyls_walk_join<G, 1>(tot, xw, lane, grp, parity);
      parity ^= 1;
    }
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
  load(ibeg, sa);
  for (int i0 = ibeg; i0 < iend; i0 += 32) {
    load(i0 + 16, sb);
    body(i0, sa);
    if (i0 + 16 >= iend) break;
    load(i0 + 32, sa);
    body(i0 + 16, sb);
  }
  double* part = wsbase + d.part + nyls_split_pass(m, d.nchunks, c);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double v = nyls_walk_fold(zacc[b]);
    if (ph == 0 && wk.lv[b]) part[s0 + 16 * b + wk.sl] = v;
  }
  const double csum = nyls_wave_sum(sacc);
  if (lane == 0 && grp == 0) part[m] = csum;
}

// One refinement step of mu (step `step` of at most `refine`), as in k_backward: the residual
// x_bar - A mu from the chunk sums, the correction from the stored factors, and the stopping
// rule (correction below 1e-8 |mu|, predicted to be, or no longer halving).
template <int P>
__global__ __launch_bounds__(64) void k_bws_mu_combine(const nyls_desc* __restrict__ desc,
                                                       double* __restrict__ wsbase, int step,
                                                       int refine) {
  __shared__ double an[NYLS_MAX_M], mu[NK], R[NK];
  __shared__ int piv[NK];
  const nyls_desc& d = desc[blockIdx.x];
  if (!takes<P>(d)) return;
  const int m = d.m, N = m + 1 + P, nc = d.nchunks, lane = threadIdx.x;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  double* st = ws + L.tmp + N;
  if (st[BS_DONE] != 0.0) return;
  const int r = (int)ws[L.info + 0];
  const double* W = ws + L.W;
  const double* Hc = ws + L.H;
  const double* xb = ws + L.tmp;
  const double* part = wsbase + d.part;
  const double gam = d.gamma;
  for (int s = lane; s < m; s += 64) {
    double acc = 0.0;
    for (int cc = 0; cc < nc; ++cc) acc += part[nyls_split_pass(m, nc, cc) + s];
    an[s] = acc;
  }
  double csum = 0.0;
  if (lane == 0)
    for (int cc = 0; cc < nc; ++cc) csum += part[nyls_split_pass(m, nc, cc) + m];
  csum = nyls_rdlane(csum, 0);
  for (int a = lane; a < N; a += 64) {
    mu[a] = ws[L.mu + a];
    piv[a] = (int)ws[L.piv + a];
  }
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
  nyls_lu_solve_w(ws + L.lu, N, N, piv, R);
  double dsq = 0.0, xsq = 0.0;
  for (int k = lane; k < r; k += 64) {
    dsq += R[k] * R[k];
    xsq += mu[k] * mu[k];
  }
  const double dn = sqrt(nyls_wave_sum(dsq)) + fabs(R[m]);
  const double xn = sqrt(nyls_wave_sum(xsq)) + fabs(mu[m]);
  for (int a = lane; a < N; a += 64) ws[L.mu + a] = mu[a] + R[a];
  const double dprev = st[BS_DPREV];
  const bool stalled = step > 0 && dn > 0.5 * dprev;
  const double pred = dn * (dn / (step > 0 ? dprev : xn));
  const bool done = dn <= 1e-8 * xn || pred <= 1e-8 * xn || stalled || step + 1 >= refine;
  __syncthreads();
  if (lane == 0) {
    st[BS_DPREV] = dn;
    st[BS_PASSES] += 1.0;
    st[BS_DONE] = done ? 1.0 : 0.0;
  }
}

template <int NB, int P, bool EX, int G = 1>
__global__ __launch_bounds__(64 * G) void k_bws_grad_pass(const nyls_desc* __restrict__ desc,
                                                          double* __restrict__ wsbase,
                                                          double* __restrict__ dl_df,
                                                          double* __restrict__ dl_dr, int64_t total) {
  constexpr int Q = 4 + 2 * P;
  __shared__ __align__(16) double tiles[G][Q * 16 * NYLS_WALK_PAD];
  __shared__ double bcs[G][2 * 16];
  __shared__ double xw[G > 1 ? 2 * G * Q * 16 : 1];
  const nyls_desc& d = desc[blockIdx.x];
  if (!takes<P>(d) || d.rec != (EX ? 0 : 1) || nyls_slot_blocks(d.m) != NB * G) return;
  const int c = (int)blockIdx.y;
  if (c >= d.nchunks) return;
  const int m = d.m, n = d.n;
  const int lane = threadIdx.x & 63, grp = G > 1 ? (int)(threadIdx.x >> 6) : 0;
  const int s0 = 16 * NB * grp;
  const bool lead = grp == 0;  // writes dl/df, dl/dr and the scalar sum
  double* const tile = tiles[grp];
  double* const bc = bcs[grp];
  int parity = 0;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const int r = (int)ws[L.info + 0];
  const int ibeg = c * d.chunk, iend = min(n, ibeg + d.chunk);
  const double gam = d.gamma;
  nyls_walk<NB, EX> wk;
  wk.init(d, lane, s0);
  nyls_cpts cpt;
  cpt.init(d);
  const int ph = wk.ph;
  const double inv_s2 = wk.inv_sigma * wk.inv_sigma;
  nyls_oppoly<P> op;
  op.init(inv_s2);
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  const double* mu = ws + L.mu;
  double alv[NB], bev[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) alv[b] = wk.lv[b] ? ws[L.alpha + s0 + 16 * b + wk.sl] : 0.0;
  beta_slots<NB>(ws + L.W, mu, m, r, s0, wk.sl, wk.lv, bev);
  const double bias = ws[L.x + m], mub = mu[m];
  double aeacc[NB], anacc[NB], t2 = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) aeacc[b] = anacc[b] = 0.0;
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
          nyls_hfac<P>(g, inv_s2, h);
          const double pv = e * nyls_horner<P>(g, cj);
          const double dpv = e * nyls_horner<P + 2>(g, dj);
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
    if constexpr (G > 1) {
      nyls_walk_join<G, Q>(tot, xw, lane, grp, parity);
      parity ^= 1;
    }
    const int ip = i0 + (lane & 15);
    const bool okp = ip < n && !cpt.has(ip);
    const double ei = okp ? tot[0] + st.c * bias - st.r : 0.0;
    const double nui = okp ? tot[1] + st.c * mub : 0.0;
    if (lane < 16 && ip < n && lead) {
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
  load(ibeg, sa);
  for (int i0 = ibeg; i0 < iend; i0 += 32) {
    load(i0 + 16, sb);
    body(i0, sa);
    if (i0 + 16 >= iend) break;
    load(i0 + 32, sa);
    body(i0 + 16, sb);
  }
  double* part = wsbase + d.part + nyls_split_gram(m, c);  // [m] sum e p, [m] sum nu p, t2
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double va = nyls_walk_fold(aeacc[b]), vn = nyls_walk_fold(anacc[b]);
    if (ph == 0 && wk.lv[b]) {
      part[s0 + 16 * b + wk.sl] = va;
      part[m + s0 + 16 * b + wk.sl] = vn;
    }
  }
  t2 = nyls_wave_sum(t2);
  if (lane == 0 && lead) part[2 * m] = t2;
}

// C(i, j) = sum_k A(i, k) B(k, j), i < M, j < N, for the 256 threads of a workgroup: 64 x 64
// output tiles (4 x 4 per thread) over k-chunks of 16, both operands staged through LDS
// (ab: 2 * 16 * 65 doubles).  a(i, k) and b(k, j) read the operands; A_KFAST says that
// consecutive k of a row of A are adjacent in memory (else consecutive i are), which decides
// the order the tile is loaded in (B is read with consecutive j adjacent).  out(i, j, v)
// receives each result once.
template <bool A_KFAST, class FA, class FB, class FO>
__device__ inline void block_gemm(int M, int N, int K, FA a, FB b, FO out, double* ab) {
  constexpr int TS = 65;  // LDS row stride
  double* As = ab;           // [16][TS]: As[k][i]
  double* Bs = ab + 16 * TS;  // [16][TS]: Bs[k][j]
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  for (int i0 = 0; i0 < M; i0 += 64)
    for (int j0 = 0; j0 < N; j0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      for (int k0 = 0; k0 < K; k0 += 16) {
        __syncthreads();
        for (int e = tid; e < 16 * 64; e += NYLS_BLOCK) {
          const int ia = A_KFAST ? e >> 4 : e & 63, ka = A_KFAST ? e & 15 : e >> 6;
          As[ka * TS + ia] = (i0 + ia < M && k0 + ka < K) ? a(i0 + ia, k0 + ka) : 0.0;
          const int jb = e & 63, kb = e >> 6;
          Bs[kb * TS + jb] = (j0 + jb < N && k0 + kb < K) ? b(k0 + kb, j0 + jb) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = As[kk * TS + 4 * ti + u];
            bv[u] = Bs[kk * TS + 4 * tj + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 4 * ti + u, j = j0 + 4 * tj + v;
          if (i < M && j < N) out(i, j, acc[u][v]);
        }
    }
}

// The sigma terms through the conditions and K_mm, dl/dgamma and dl/dv, as in k_backward;
// 256 threads, the m^3 products of the K_mm term as LDS-tiled products.
template <int P>
__global__ __launch_bounds__(NYLS_BLOCK) void k_bws_final(const nyls_desc* __restrict__ desc,
                                                  double* __restrict__ wsbase,
                                                  double* __restrict__ dl_dv,
                                                  double* __restrict__ dl_dsigma,
                                                  double* __restrict__ dl_dgamma) {
  __shared__ double tl[NYLS_MAX_M], kb[NYLS_MAX_M], ae[NYLS_MAX_M], an[NYLS_MAX_M];
  __shared__ double ug1[NYLS_MAX_M], ug2[NYLS_MAX_M], xv[NK], mu[NK], red[16];
  __shared__ double ab[2 * 16 * 65];
  const int inst = (int)blockIdx.x;
  const nyls_desc& d = desc[inst];
  if (!takes<P>(d)) return;
  const int m = d.m, N = m + 1 + P, nc = d.nchunks, tid = threadIdx.x;
  constexpr int NT = NYLS_BLOCK;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* U = ws + L.U;
  const double* lamv = ws + L.lam;
  const double* hkv = ws + L.acc;  // [P][m]
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma, inv_sigma = 1.0 / d.sigma, inv_s2 = inv_sigma * inv_sigma;
  const double* part = wsbase + d.part;
  const double* st = ws + L.tmp + N;
  const double t1 = st[BS_T1];
  const double passes = st[BS_PASSES];
  for (int s = tid; s < m; s += NT) {
    double a1 = 0.0, a2 = 0.0;
    for (int cc = 0; cc < nc; ++cc) {
      a1 += part[nyls_split_gram(m, cc) + s];
      a2 += part[nyls_split_gram(m, cc) + m + s];
    }
    ae[s] = a1;
    an[s] = a2;
    tl[s] = nyls_grid_t(d, d.lidx[s]);
    kb[s] = ws[L.beta + s];
  }
  double t2 = 0.0;
  for (int cc = 0; cc < nc; ++cc) t2 += part[nyls_split_gram(m, cc) + 2 * m];
  for (int a = tid; a < N; a += NT) {
    xv[a] = ws[L.x + a];
    mu[a] = ws[L.mu + a];
  }
  __syncthreads();
  // sigma: condition-row term, one landmark per thread
  double t3 = 0.0;
  for (int s = tid; s < m; s += NT) {
    double al = 0.0, be = 0.0;
    for (int k = 0; k < r; ++k) {
      al += W[s * m + k] * xv[k];
      be += W[s * m + k] * mu[k];
    }
    for (int j = 0; j < P; ++j) {
      const double z = (nyls_grid_t(d, d.cond_i[j]) - tl[s]) * inv_sigma;
      const double e = exp(-z * z);
      double h[P + 2];
      nyls_hfac<P>(-2.0 * inv_sigma * z, inv_s2, h);
      double ds = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q)
        if (q == d.cond_d[j]) ds = -e * (q * inv_sigma * h[q] + z * h[q + 1]);
      t3 += (xv[m + 1 + j] * be + mu[m + 1 + j] * al) * ds;
    }
  }
  t3 = nyls_block_sum(t3, red);
  // g1 = kbar - gamma sum nu p - H_k mu_lambda ; g2 = gamma sum e p + H_k lambda
  for (int s = tid; s < m; s += NT) {
    double g1 = kb[s] - gam * an[s], g2 = gam * ae[s];
    for (int j = 0; j < P; ++j) {
      g1 -= hkv[j * m + s] * mu[m + 1 + j];
      g2 += hkv[j * m + s] * xv[m + 1 + j];
    }
    kb[s] = g1;
    ae[s] = g2;
  }
  __syncthreads();
  for (int k = tid; k < m; k += NT) {
    double u1 = 0.0, u2 = 0.0;
    for (int s = 0; s < m; ++s) {
      u1 += U[s * m + k] * kb[s];
      u2 += U[s * m + k] * ae[s];
    }
    ug1[k] = u1;
    ug2[k] = u2;
  }
  // dK_mm/dsigma into the Gram block, then E = dK U[:, :r] into tmp (x_bar and the state,
  // read above, are no longer needed)
  double* dK = ws + L.gram;
  double* E = ws + L.tmp;
  __syncthreads();
  for (int e = tid; e < m * m; e += NT) {
    const int a = e / m, s = e - a * m;
    const double z = (tl[a] - tl[s]) * inv_sigma;
    dK[e] = (2.0 * z * z * inv_sigma) * exp(-z * z);
  }
  block_gemm<true>(
      m, r, m, [&](int a, int s) { return dK[a * m + s]; }, [&](int s, int l) { return U[s * m + l]; },
      [&](int a, int l, double v) { E[a * m + l] = v; }, ab);
  __syncthreads();
  double tk = 0.0;  // sum over (k, l) of the weight times (U^T dK U)[k][l]
  block_gemm<false>(
      m, r, m, [&](int k, int a) { return U[a * m + k]; }, [&](int a, int l) { return E[a * m + l]; },
      [&](int k, int l, double dkl) {
        const double ll = lamv[l], lk = lamv[k];
        const double qb = 0.5 * sqrt(ll) * (ug1[k] * xv[l] - ug2[k] * mu[l]);
        const double fkl = (k < r) ? -1.0 / (lk * ll) : 1.0 / (ll * (ll - lk));
        tk += (k < r ? 1.0 : 2.0) * fkl * qb * dkl;
      },
      ab);
  tk = nyls_block_sum(tk, red);
  double mw = 0.0;
  for (int k = tid; k < r; k += NT) mw += mu[k] * xv[k];
  mw = nyls_block_sum(mw, red);
  if (tid == 0) {
    ws[L.info + 6] = passes;
    if (dl_dgamma) dl_dgamma[inst] = mw / gam;
    if (dl_dsigma) dl_dsigma[inst] = t1 - gam * t2 - t3 + tk;
  }
  if (dl_dv && tid < NYLS_MAX_P) dl_dv[inst * NYLS_MAX_P + tid] = tid < P ? mu[m + 1 + tid] : 0.0;
}

// NB: slot blocks of the instance class (16: wide bases, two wavefronts of eight blocks)
template <int NB, int P, bool EX>
void launch_passes_x(const nyls_plan_view& pv, double* ws, bool mu_pass, double* dl_df,
                     double* dl_dr, hipStream_t st) {
  constexpr int G = NB > 8 ? NB / 8 : 1, NW = NB / G;
  const dim3 grid(pv.batch, pv.max_chunks), block(64 * G);
  if (mu_pass)
    hipLaunchKernelGGL((k_bws_mu_pass<NW, P, EX, G>), grid, block, 0, st, pv.d_desc, ws);
  else
    hipLaunchKernelGGL((k_bws_grad_pass<NW, P, EX, G>), grid, block, 0, st, pv.d_desc, ws, dl_df,
                       dl_dr, pv.total);
}

template <int NB, int P>
void launch_passes_p(const nyls_plan_view& pv, double* ws, bool mu_pass, double* dl_df,
                     double* dl_dr, hipStream_t st) {
  if (!(pv.p_mask & (1u << P)) || !(pv.nb_mask & (1u << NB))) return;
  if (pv.rec_mask & 2) launch_passes_x<NB, P, false>(pv, ws, mu_pass, dl_df, dl_dr, st);
  if (pv.rec_mask & 1) launch_passes_x<NB, P, true>(pv, ws, mu_pass, dl_df, dl_dr, st);
}

template <int NB>
void launch_passes_nb(const nyls_plan_view& pv, double* ws, bool mu_pass, double* dl_df,
                      double* dl_dr, hipStream_t st) {
  launch_passes_p<NB, 1>(pv, ws, mu_pass, dl_df, dl_dr, st);
  launch_passes_p<NB, 2>(pv, ws, mu_pass, dl_df, dl_dr, st);
  launch_passes_p<NB, 3>(pv, ws, mu_pass, dl_df, dl_dr, st);
  launch_passes_p<NB, 4>(pv, ws, mu_pass, dl_df, dl_dr, st);
}

template <int P>
void launch_small(const nyls_plan_view& pv, double* ws, int which, int step, int refine,
                  const double* t_obs, const int64_t* obs_off, const double* g, double* dl_dv,
                  double* dl_ds, double* dl_dg, hipStream_t st) {
  if (!(pv.p_mask & (1u << P))) return;
  const dim3 grid(pv.batch);
  if (which == 0)
    hipLaunchKernelGGL(k_bws_setup<P>, grid, dim3(64), 0, st, pv.d_desc, ws, t_obs, obs_off, g);
  else if (which == 1)
    hipLaunchKernelGGL(k_bws_mu_combine<P>, grid, dim3(64), 0, st, pv.d_desc, ws, step, refine);
  else
    hipLaunchKernelGGL(k_bws_final<P>, grid, dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, dl_dv, dl_ds, dl_dg);
}

void launch_small_all(const nyls_plan_view& pv, double* ws, int which, int step, int refine,
                      const double* t_obs, const int64_t* obs_off, const double* g, double* dl_dv,
                      double* dl_ds, double* dl_dg, hipStream_t st) {
  launch_small<1>(pv, ws, which, step, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  launch_small<2>(pv, ws, which, step, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  launch_small<3>(pv, ws, which, step, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  launch_small<4>(pv, ws, which, step, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
}

}  // namespace

// The adjoint of the plan's split instances (the other instances are left to k_backward).
hipError_t nyls_launch_backward_split(const nyls_plan_view& pv, double* ws, int refine,
                                      const double* t_obs, const int64_t* obs_off, const double* g,
                                      double* dl_df, double* dl_dr, double* dl_dv, double* dl_ds,
                                      double* dl_dg, hipStream_t st) {
  if (!pv.n_split) return hipSuccess;
  launch_small_all(pv, ws, 0, 0, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  for (int step = 0; step < refine; ++step) {
    launch_passes_nb<2>(pv, ws, true, dl_df, dl_dr, st);
    launch_passes_nb<4>(pv, ws, true, dl_df, dl_dr, st);
    launch_passes_nb<8>(pv, ws, true, dl_df, dl_dr, st);
    launch_passes_nb<16>(pv, ws, true, dl_df, dl_dr, st);
    launch_small_all(pv, ws, 1, step, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  }
  launch_passes_nb<2>(pv, ws, false, dl_df, dl_dr, st);
  launch_passes_nb<4>(pv, ws, false, dl_df, dl_dr, st);
  launch_passes_nb<8>(pv, ws, false, dl_df, dl_dr, st);
  launch_passes_nb<16>(pv, ws, false, dl_df, dl_dr, st);
  launch_small_all(pv, ws, 2, 0, refine, t_obs, obs_off, g, dl_dv, dl_ds, dl_dg, st);
  return hipGetLastError();
}
