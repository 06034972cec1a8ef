// FP64 operator Gram of Lemma 1 (Sec. 3.1), one workgroup per instance.
//
// For every residual point i the kernel-space row
//     q_i = ( p_i[0..m-1], c_i, r_i ),  p_i = k_m^(p)(t_i) - sum_k f_k(t_i) k_m^(p-k)(t_i),
//     c_i = -f_p(t_i),
// is evaluated in registers/LDS (never written to HBM) and the symmetric Gram
//     S~ = sum_i q_i q_i^T   ((m+2) x (m+2): S, u = sum c_i p_i, z = sum r_i p_i, ...)
// is accumulated.  Points are processed in tiles of TP: the tile's rows are built in LDS,
// then each thread owns 4 x 4 output blocks of the upper triangle and accumulates them
// in registers; when few blocks exist the tile's points are split over thread groups.
// Group partials are summed in a fixed order, so the result is bitwise reproducible.
#include "nyls_internal.h"

namespace {

constexpr int TP = 64;      // points per tile
constexpr int CH = 16;      // points per thread in the Gaussian recurrence
constexpr int MAXB = 3;     // 4x4 blocks per thread (m <= 128 -> at most 561 blocks)

__device__ inline int instance_of(const int32_t* order) {
  return order ? order[blockIdx.x] : (int)blockIdx.x;
}

__device__ inline void block_coords(int blk, int nb, int& bi, int& bj) {
  int b = blk, row = 0;
  while (b >= nb - row) { b -= nb - row; ++row; }
  bi = row;
  bj = row + b;
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_gram64(const nyls_desc* __restrict__ desc,
                                                       const int32_t* __restrict__ order,
                                                       double* __restrict__ wsbase, int maxm,
                                                       int only) {
  extern __shared__ double sm[];
  const nyls_desc& d = desc[instance_of(order)];
  if (only && !((int)wsbase[d.ws + nyls_layout(d.m, d.p, 0).info + 1] & only)) return;
  const int m = d.m, p = d.p, n = d.n;
  const int g = m + 2;
  const int gp = (g + 3) & ~3;
  const int nb = gp >> 2;
  const int nblk = nb * (nb + 1) / 2;
  const int ngrp = nblk >= NYLS_BLOCK ? 1 : NYLS_BLOCK / nblk;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;

  const int gpmax = (maxm + 2 + 3) & ~3;
  double* Q = sm;                          // [TP][gp] tile rows (also the reduction buffer)
  double* fr = Q + (size_t)TP * gp;         // [TP][NYLS_MAX_P+1] operator weights per point
  double* tl = fr + TP * (NYLS_MAX_P + 1);  // [m] landmark times
  int* okp = reinterpret_cast<int*>(tl + NYLS_MAX_M);  // [TP] residual-point flag
  double* Q2 = reinterpret_cast<double*>(okp + TP) + (size_t)TP * (gpmax - gp);  // [TP][gp]
  double* Ub = Q2 + (size_t)TP * gp;        // [m][m] eigenvectors (only when maxm <= 64)

  // Ill-conditioned K_mm (retained eigenvalues below 1e-9 lambda_1): the kernel-space Gram
  // would lose most digits in W^T S W, so the rows are rotated by U^T first and the Gram is
  // accumulated in the eigenbasis (the KKT kernel then scales by Lambda^{-1/2}).
  const int rank = (int)ws[L.info + 0];
  const bool rotate = only || (rank > 0 && ws[L.lam + rank - 1] < 1e-9 * ws[L.lam]);
  const double* Ug = ws + L.U;
  const bool ulds = maxm <= 64;
  if (rotate && ulds)
    for (int e = tid; e < m * m; e += NYLS_BLOCK) Ub[e] = Ug[e];
  const double* Uu = ulds ? Ub : Ug;
  double* Qa = rotate ? Q2 : Q;             // rows the Gram accumulates

  const double inv_sigma = 1.0 / d.sigma;
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);

  // Thread -> (group, blocks)
  const int grp = (ngrp > 1) ? tid / nblk : 0;
  int myblk[MAXB] = {0, 0, 0}, bi[MAXB] = {0, 0, 0}, bj[MAXB] = {0, 0, 0}, nmine = 0;
  if (ngrp > 1) {
    if (grp < ngrp) { myblk[0] = tid - grp * nblk; nmine = 1; }
  } else {
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = tid + k * NYLS_BLOCK;
      if (b < nblk) { myblk[k] = b; nmine = k + 1; }
    }
  }
#pragma unroll
  for (int k = 0; k < MAXB; ++k)
    if (k < nmine) block_coords(myblk[k], nb, bi[k], bj[k]);
  double acc[MAXB][16];
#pragma unroll
  for (int k = 0; k < MAXB; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[k][e] = 0.0;

  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    // per-point operator weights w_q (L = d^p - sum f_k d^(p-k)), c_i, r_i, padding
    for (int e = tid; e < TP; e += NYLS_BLOCK) {
      const int i = i0 + e;
      const bool ok = i < n && !nyls_is_condition_point(d, i);
      okp[e] = ok;
      double w[NYLS_MAX_P + 1];
      nyls_opweights(p, [&](int k) { return ok ? d.f[(size_t)(k - 1) * n + i] : 0.0; }, w);
#pragma unroll
      for (int q = 0; q <= NYLS_MAX_P; ++q) fr[e * (NYLS_MAX_P + 1) + q] = w[q];
      Q[e * gp + m] = ok ? -d.f[(size_t)(p - 1) * n + i] : 0.0;
      Q[e * gp + m + 1] = ok ? d.r[i] : 0.0;
      for (int c = m + 2; c < gp; ++c) Q[e * gp + c] = 0.0;
    }
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double z, double ev) {
      double kd[NYLS_MAX_P + 1];
      nyls_kderiv_e(z, ev, inv_sigma, kd);
      const double* w = fr + pt * (NYLS_MAX_P + 1);
      double v = 0.0;
#pragma unroll
      for (int q = 0; q <= NYLS_MAX_P; ++q) v += w[q] * kd[q];
      Q[pt * gp + s] = v;
    });
    __syncthreads();
    if (rotate) {
      for (int e = tid; e < TP * gp; e += NYLS_BLOCK) {
        const int pt = e / gp, k = e - pt * gp;
        double v = Q[pt * gp + k];
        if (k < m) {
          v = 0.0;
          const double* q = Q + pt * gp;
          for (int s2 = 0; s2 < m; ++s2) v += q[s2] * Uu[s2 * m + k];
        }
        Q2[e] = v;
      }
      __syncthreads();
    }
    for (int pt = grp; pt < TP; pt += ngrp) {
      if (!okp[pt]) continue;
      const double* row = Qa + pt * gp;
#pragma unroll
      for (int k = 0; k < MAXB; ++k) {
        if (k >= nmine) break;
        const double* ra = row + 4 * bi[k];
        const double* rb = row + 4 * bj[k];
        const double a0 = ra[0], a1 = ra[1], a2 = ra[2], a3 = ra[3];
        const double b0 = rb[0], b1 = rb[1], b2 = rb[2], b3 = rb[3];
        double* c = acc[k];
        c[0] += a0 * b0; c[1] += a0 * b1; c[2] += a0 * b2; c[3] += a0 * b3;
        c[4] += a1 * b0; c[5] += a1 * b1; c[6] += a1 * b2; c[7] += a1 * b3;
        c[8] += a2 * b0; c[9] += a2 * b1; c[10] += a2 * b2; c[11] += a2 * b3;
        c[12] += a3 * b0; c[13] += a3 * b1; c[14] += a3 * b2; c[15] += a3 * b3;
      }
    }
  }
  __syncthreads();
  // Fixed-order reduction of the groups into Q[blk][16].
  for (int gi = 0; gi < ngrp; ++gi) {
    if (grp == gi) {
#pragma unroll
      for (int k = 0; k < MAXB; ++k) {
        if (k >= nmine) break;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          double* dst = Q + myblk[k] * 16 + e;
          *dst = (gi == 0) ? acc[k][e] : *dst + acc[k][e];
        }
      }
    }
    __syncthreads();
  }
  double* out = ws + L.gram;
  for (int e = tid; e < g * g; e += NYLS_BLOCK) {
    int a = e / g, b = e - a * g;
    if (a > b) { const int t = a; a = b; b = t; }
    const int ia = a >> 2, ib = b >> 2;
    const int blk = ia * nb - ia * (ia - 1) / 2 + (ib - ia);
    out[e] = Q[blk * 16 + (a & 3) * 4 + (b & 3)];
  }
  if (tid == 0) ws[L.info + 4] = rotate ? 1.0 : 0.0;
}

}  // namespace

size_t nyls_gram64_lds_bytes(int maxm) {
  const int gp = (maxm + 2 + 3) & ~3;
  const int nb = gp >> 2;
  const size_t tile = (size_t)TP * gp, red = (size_t)nb * (nb + 1) / 2 * 16;
  // the rotated-row tile Q2 sits after the point flags at an offset that is independent of
  // the instance's own tile width; the reduction buffer may run into fr / tl / okp only
  const size_t base = tile * sizeof(double) + TP * (NYLS_MAX_P + 1) * sizeof(double) +
                      NYLS_MAX_M * sizeof(double) + TP * sizeof(int);
  size_t total = base + tile * sizeof(double) + (maxm <= 64 ? (size_t)maxm * maxm * sizeof(double) : 0);
  if (red * sizeof(double) > total) total = red * sizeof(double);
  return total;
}

hipError_t nyls_launch_gram64(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  const size_t lds = nyls_gram64_lds_bytes(pv.maxm);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram64),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_gram64, dim3(pv.batch), dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order, ws,
                     pv.maxm, pv.only);
  return hipGetLastError();
}
