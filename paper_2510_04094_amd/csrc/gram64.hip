// FP64 operator Gram of Lemma 1 (Sec. 3.1).
//
// For every residual point i the kernel-space row
//     q_i = ( p_i[0..m-1], c_i, r_i ),  p_i = k_m^(p)(t_i) - sum_k f_k(t_i) k_m^(p-k)(t_i),
//     c_i = -f_p(t_i),
// is evaluated in registers (never written to HBM) and the symmetric Gram
//     S~ = sum_i q_i q_i^T   ((m+2) x (m+2): S, u = sum c_i p_i, z = sum r_i p_i, ...)
// is accumulated.
//
// k_gram64_mfma (kernel-space Gram, the common case): one wavefront per instance with the
// lane layout of nyls_walk.h, where lane (sl, ph) holds q_i[16 b + sl] for the points
// 4 j + ph of each 16-point chunk (columns m and m+1 carry c_i and r_i).  That is exactly the
// operand layout of v_mfma_f64_16x16x4f64 with the four points of one j as the k dimension
// (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k), so every tile pair (I <= J) of the
// Gram takes one FP64 MFMA per j: A = q[16 I + sl], B = q[16 J + sl], FP64 accumulation.
// Only the ceil((m+2)/16) blocks that carry data get tiles, and when the last of them holds at
// most four columns (m = 50: landmarks 48, 49, c_i, r_i) those columns are accumulated on the
// VALU instead of a mostly-empty MFMA tile row: each column value is broadcast along its
// 16-lane row (one DPP move) and multiplied into per-lane sums, which overlap with the
// matrix-core work of the full blocks.
//
// k_gram64 (ill-conditioned K_mm: retained eigenvalues below 1e-9 lambda_1, or the FP64
// re-solve of a mixed-precision instance): the rows are rotated by U^T first and the Gram is
// accumulated in the eigenbasis (the KKT kernel then scales by Lambda^{-1/2}).  It also takes
// the kernel-space Grams of m + 2 > 64, whose 36 MFMA tiles would not fit in registers.  256
// threads per instance: 64-point tiles of rows in LDS, 4 x 4 register blocks per thread,
// group partials summed in a fixed order.
#include "nyls_walk.h"

#include <type_traits>

namespace {

constexpr int CH = 16;      // points per thread in the Gaussian recurrence
constexpr int MAXB = 3;     // 4x4 blocks per thread (m <= 128 -> at most 561 blocks)
// Wide bases (m > NYLS_NARROW_MAX_M, split instances only): 32-point tiles (two 260-column
// tiles fit the LDS), and the up to 2145 blocks of the Gram are shared out over
// ceil(nblk / (3 * 256)) workgroups per chunk (grid z), each writing its blocks straight
// from registers; every one of them forms the chunk's rows.
constexpr int kWideBlocks = MAXB * NYLS_BLOCK;
constexpr int kG4Blocks = NYLS_GRAM4_MAX_G / 16;  // column blocks of the four-wave MFMA Gram

__device__ inline int instance_of(const int32_t* order) {
  return order ? order[blockIdx.x] : (int)blockIdx.x;
}

__device__ inline void block_coords(int blk, int nb, int& bi, int& bj) {
  int b = blk, row = 0;
  while (b >= nb - row) { b -= nb - row; ++row; }
  bi = row;
  bj = row + b;
}

// smode 0: instances without NYLS_DF_SPLIT, the whole grid, into the instance's Gram, in the
// basis the eigensolver's result calls for; smode 3 / 4: the same in two halves, kernel space
// for every instance (3, needs nothing from the eigensolver, so it can run beside it) and,
// after the eigensolver, rotated for the instances that need the eigenbasis (4);
// smode 1 / 2: split instances, chunk blockIdx.y of the grid, into its partial sum, in
// kernel space (1) or, for instances that need the eigenbasis, rotated (2).
// TP = 64: bases up to NYLS_NARROW_MAX_M; TP = 32: wide bases (see kWideBlocks).
template <int TP>
__global__ __launch_bounds__(NYLS_BLOCK) void k_gram64(const nyls_desc* __restrict__ desc,
                                                       const int32_t* __restrict__ order,
                                                       double* __restrict__ wsbase, int maxm,
                                                       int only, int smode) {
  constexpr bool WIDE = TP == 32;
  extern __shared__ double sm[];
  const nyls_desc& d = desc[instance_of(order)];
  const bool split = smode == 1 || smode == 2;
  if (((d.flags & NYLS_DF_SPLIT) != 0) != split) return;
  if ((d.m > NYLS_NARROW_MAX_M) != WIDE) return;
  const int chunk = (int)blockIdx.y;
  if (split && chunk >= d.nchunks) return;
  if (only && !((int)wsbase[d.ws + nyls_layout(d.m, d.p, 0).info + 1] & only)) return;
  const int m = d.m, p = d.p, n = d.n;
  const int g = m + 2;
  const int gp = (g + 3) & ~3;
  const int nb = gp >> 2;
  const int nblk = nb * (nb + 1) / 2;
  const int ngrp = (WIDE || nblk >= NYLS_BLOCK) ? 1 : NYLS_BLOCK / nblk;
  const int blk0 = WIDE ? (int)blockIdx.z * kWideBlocks : 0;  // first block of this workgroup
  if (blk0 >= nblk) return;
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
  // FP64 re-solves (only) take the eigenbasis, except unsplit bases with 64 < m + 2 <= 128:
  // those keep the kernel-space Gram of the four-wave MFMA kernel unless K_mm is
  // ill-conditioned (the FP64 mode's own rule), which this kernel would otherwise rotate on
  // the VALU.
  const int rank = (smode == 1 || smode == 3) ? 0 : (int)ws[L.info + 0];
  const bool g4 = !split && m + 2 > 64 && m + 2 <= 16 * kG4Blocks;
  const bool rotate = (only && !g4) || (rank > 0 && ws[L.lam + rank - 1] < 1e-9 * ws[L.lam]);
  if ((smode == 2 || smode == 4) && !rotate) return;  // the kernel-space Gram stands
  // m + 2 <= 64: the one-wave MFMA kernels take the instance unless its tuning asks for this
  // one, m + 2 <= 128 in kernel space the four-wave one (split instances always come here)
  if (!split && nyls_slot_blocks(m + 2) <= 4 && !(d.flags & NYLS_DF_GRAM_VALU)) return;
  if (!split && !rotate && m + 2 <= 16 * kG4Blocks && !(d.flags & NYLS_DF_GRAM_VALU)) return;
  const int ibeg = split ? chunk * d.chunk : 0;
  const int iend = split ? min(n, ibeg + d.chunk) : n;
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
      const int b = blk0 + tid + k * NYLS_BLOCK;
      if (b < nblk && (WIDE || b < kWideBlocks)) { myblk[k] = b; nmine = k + 1; }
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

  for (int i0 = ibeg; i0 < iend; i0 += TP) {
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
  double* out = split ? wsbase + d.part + nyls_split_gram(m, chunk) : ws + L.gram;
  if constexpr (WIDE) {
    // one thread per block: its entries and their mirror images, straight from registers
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      if (k >= nmine) break;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int a = 4 * bi[k] + (e >> 2), b = 4 * bj[k] + (e & 3);
        if (a < g && b < g) {
          out[a * g + b] = acc[k][e];
          out[b * g + a] = acc[k][e];
        }
      }
    }
    return;
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
  for (int e = tid; e < g * g; e += NYLS_BLOCK) {
    int a = e / g, b = e - a * g;
    if (a > b) { const int t = a; a = b; b = t; }
    const int ia = a >> 2, ib = b >> 2;
    const int blk = ia * nb - ia * (ia - 1) / 2 + (ib - ia);
    out[e] = Q[blk * 16 + (a & 3) * 4 + (b & 3)];
  }
  if (tid == 0 && !split) ws[L.info + 4] = rotate ? 1.0 : 0.0;
}

// Gram of a split instance: the sum of its chunk partials in chunk order (a fixed order,
// so the result does not depend on which workgroup finished first), and the basis it is in.
// Grid (instance, tiles of 256 Gram entries), one entry per thread.
__global__ __launch_bounds__(NYLS_BLOCK) void k_gram_split_sum(const nyls_desc* __restrict__ desc,
                                                               double* __restrict__ wsbase) {
  const nyls_desc& d = desc[blockIdx.x];
  if (!(d.flags & NYLS_DF_SPLIT)) return;
  const int m = d.m, g = m + 2;
  const int e = (int)blockIdx.y * NYLS_BLOCK + (int)threadIdx.x;
  if ((int)blockIdx.y * NYLS_BLOCK >= g * g) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const double* part = wsbase + d.part;
  if (e < g * g) {
    double acc = 0.0;
    for (int c = 0; c < d.nchunks; ++c) acc += part[nyls_split_gram(m, c) + e];
    ws[L.gram + e] = acc;
  }
  if (e == 0) {
    const int rank = (int)ws[L.info + 0];
    const bool rotate = rank > 0 && ws[L.lam + rank - 1] < 1e-9 * ws[L.lam];
    ws[L.info + 4] = rotate ? 1.0 : 0.0;
  }
}


typedef double nyls_d4 __attribute__((ext_vector_type(4)));

// Eigenbasis Gram when the smallest retained eigenvalue is below kRotate lambda_1 (the
// kernel-space Gram would lose most digits in W^T S W) or when re-solving with FP64.
constexpr double kRotate = 1e-9;

__device__ inline bool use_eigenbasis(const double* ws, const nyls_wsl& L, int only) {
  const int rank = (int)ws[L.info + 0];
  return only || (rank > 0 && ws[L.lam + rank - 1] < kRotate * ws[L.lam]);
}

// Value of lane 16 (lane / 16) + T (the same column of this lane's point).  The builtin's
// result is returned as the double itself (one v_mov_b64_dpp with row_newbcast); inside an
// overloaded call it could be read as an integer, which nyls_dpp_f64 avoids elsewhere.
template <int T>
__device__ inline double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + T, 0xf, 0xf, false);
}

// NB = ceil((m + 2) / 16) column blocks with data; TLG: the last holds at most four columns
// and is accumulated on the VALU (nyls_gram_class_of: the instance's NYLS_DF_GRAM_TAIL flag).
template <int NB, int P, bool EX, bool TLG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_gram64_mfma(const nyls_desc* __restrict__ desc,
                                                    const int32_t* __restrict__ order,
                                                    double* __restrict__ wsbase, int only) {
  constexpr int NF = TLG ? NB - 1 : NB;  // blocks on the matrix cores
  constexpr int T = NF * (NF + 1) / 2;
  const nyls_desc& d = desc[instance_of(order)];
  if (d.p != P || d.rec != (EX ? 0 : 1) || d.m + 2 > 64 ||
      (d.flags & (NYLS_DF_GRAM_VALU | NYLS_DF_SPLIT)) || nyls_gram_class_of(d) != 2 * NB + (TLG ? 1 : 0))
    return;
  const int m = d.m, n = d.n, g = m + 2;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  // only < 0: every instance, before the eigensolver has chosen the basis (instances that
  // turn out to need the eigenbasis are redone by k_gram64_rot_mfma afterwards)
  if (only >= 0 && use_eigenbasis(ws, L, only)) return;  // k_gram64_rot_mfma
  const int lane = threadIdx.x;

  nyls_walk<NB, EX> wk;
  wk.init(d, lane);
  nyls_cpts cpt;
  cpt.init(d);
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  // what this lane's slot b carries: 0 landmark, 1 c_i, 2 r_i, 3 nothing
  int kind[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int s = 16 * b + wk.sl;
    kind[b] = s < m ? 0 : (s == m ? 1 : (s == m + 1 ? 2 : 3));
  }
  nyls_d4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = nyls_d4{0.0, 0.0, 0.0, 0.0};
  double tacc[NB][4];  // tail: sum_i q_i[16 b + sl] q_i[16 (NB - 1) + c]
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) tacc[b][c] = 0.0;

  nyls_oppoly<P> op;
  op.init(inv_s2);
  struct stage {
    double f[P][4], r[4];
  };
  auto load = [&](int i0, stage& st) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + 4 * j + wk.ph;
#pragma unroll
      for (int k = 0; k < P; ++k) st.f[k][j] = nyls_bload(fr, (k * n + i) * 8);
      st.r[j] = nyls_bload(rr, i * 8);
    }
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
    double q[NB];
    wk.chunk(
        d, i0,
        [&](int b, int j, double g, double e) {
          const double v = kind[b] == 0 ? e * nyls_horner<P>(g, cj[j])
                                         : (kind[b] == 1 ? -st.f[P - 1][j] : (kind[b] == 2 ? st.r[j] : 0.0));
          q[b] = v;
        },
        [&](int j) {
          const int i = i0 + 4 * j + wk.ph;
          const bool ok = i < n && !cpt.has(i);
#pragma unroll
          for (int b = 0; b < NB; ++b) q[b] = ok ? q[b] : 0.0;
          int t = 0;
#pragma unroll
          for (int I = 0; I < NF; ++I)
#pragma unroll
            for (int J = I; J < NF; ++J) {
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(q[I], q[J], acc[t], 0, 0, 0);
              ++t;
            }
          if (TLG) {
            const double qt = q[NB - 1];
            const double c0 = row_bcast<0>(qt), c1 = row_bcast<1>(qt), c2 = row_bcast<2>(qt),
                         c3 = row_bcast<3>(qt);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              tacc[b][0] += q[b] * c0;
              tacc[b][1] += q[b] * c1;
              tacc[b][2] += q[b] * c2;
              tacc[b][3] += q[b] * c3;
            }
          }
        });
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
  // tile (I, J): register v of lane l holds row 16 I + 4 v + l / 16, column 16 J + l % 16
  double* out = ws + L.gram;
  int t = 0;
#pragma unroll
  for (int I = 0; I < NF; ++I)
#pragma unroll
    for (int J = I; J < NF; ++J) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + 4 * v + (lane >> 4), b = 16 * J + (lane & 15);
        if (a < g && b < g) {
          out[a * g + b] = acc[t][v];
          if (I != J) out[b * g + a] = acc[t][v];
        }
      }
      ++t;
    }
  if (TLG) {
    // fold the four phases (points); phase-0 lanes own row 16 b + sl.  Entries inside the
    // tail block are written once per (row, column) by the lane of that row.
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double v = nyls_walk_fold(tacc[b][c]);
        const int a = 16 * b + wk.sl, x = 16 * (NB - 1) + c;
        if (wk.ph == 0 && a < g && x < g) {
          out[a * g + x] = v;
          if (b < NB - 1) out[x * g + a] = v;
        }
      }
  }
  if (lane == 0) ws[L.info + 4] = 0.0;
}

// Kernel-space FP64 Gram for 64 < m + 2 <= 128 on the matrix cores, four wavefronts per
// instance.  The one-wave kernel's 36 accumulator tiles would not fit one wavefront's
// registers, so the work is shared out: wavefront w forms the rows q_i for the column blocks
// 2w and 2w + 1 (the one-wave lane layout with two slot blocks, landmarks from 32 w on) and
// stores them to LDS in that same operand layout, Qt[j][b][lane] = q_(4j+ph)[16 b + sl]; after
// one workgroup barrier every wavefront reads the operands of all blocks back from its own
// lane positions and accumulates the tile pairs t = I (I + 1) / 2 + ... with t = w (mod 4)
// (at most nine, 36 accumulator doubles).  The LDS rows are double-buffered by chunk, so one
// barrier per 16-point chunk suffices.
template <int P, bool EX>
__global__ __launch_bounds__(NYLS_BLOCK) void k_gram64_mfma4(const nyls_desc* __restrict__ desc,
                                                             const int32_t* __restrict__ order,
                                                             double* __restrict__ wsbase, int only) {
  constexpr int NBW = kG4Blocks / 4;                      // slot blocks formed per wavefront
  constexpr int TMAX = kG4Blocks * (kG4Blocks + 1) / 2;   // tile pairs
  constexpr int TW = (TMAX + 3) / 4;                      // per wavefront
  __shared__ __align__(16) double Qt[2][4][kG4Blocks][64];
  const nyls_desc& d = desc[instance_of(order)];
  if (d.p != P || d.rec != (EX ? 0 : 1) || d.m + 2 <= 64 || d.m + 2 > 16 * kG4Blocks ||
      (d.flags & (NYLS_DF_GRAM_VALU | NYLS_DF_SPLIT)))
    return;
  const int m = d.m, n = d.n, g = m + 2;
  const int nbt = (g + 15) >> 4;  // blocks with data
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  // only < 0: every instance, before the eigensolver has chosen the basis (instances that
  // turn out to need the eigenbasis are redone by k_gram64); only > 0: the FP64 re-solve of
  // the flagged instances, in kernel space unless K_mm is ill-conditioned
  if (only > 0 && !((int)ws[L.info + 1] & only)) return;
  if (only >= 0 && use_eigenbasis(ws, L, 0)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s0 = 16 * NBW * w;

  nyls_walk<NBW, EX> wk;
  wk.init(d, lane, s0);
  nyls_cpts cpt;
  cpt.init(d);
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  int kind[NBW];  // 0 landmark, 1 c_i, 2 r_i, 3 nothing
#pragma unroll
  for (int b = 0; b < NBW; ++b) {
    const int sidx = s0 + 16 * b + wk.sl;
    kind[b] = sidx < m ? 0 : (sidx == m ? 1 : (sidx == m + 1 ? 2 : 3));
  }
  nyls_d4 acc[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) acc[t] = nyls_d4{0.0, 0.0, 0.0, 0.0};
  nyls_oppoly<P> op;
  op.init(inv_s2);
  struct stage {
    double f[P][4], r[4];
  };
  auto load = [&](int i0, stage& st) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + 4 * j + wk.ph;
#pragma unroll
      for (int k = 0; k < P; ++k) st.f[k][j] = nyls_bload(fr, (k * n + i) * 8);
      st.r[j] = nyls_bload(rr, i * 8);
    }
  };
  int buf = 0;
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
    double q[NBW];
    wk.chunk(
        d, i0,
        [&](int b, int j, double gg, double e) {
          q[b] = kind[b] == 0 ? e * nyls_horner<P>(gg, cj[j])
                              : (kind[b] == 1 ? -st.f[P - 1][j] : (kind[b] == 2 ? st.r[j] : 0.0));
        },
        [&](int j) {
          const int i = i0 + 4 * j + wk.ph;
          const bool ok = i < n && !cpt.has(i);
#pragma unroll
          for (int b = 0; b < NBW; ++b) Qt[buf][j][NBW * w + b][lane] = ok ? q[b] : 0.0;
        });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double qa[kG4Blocks];
#pragma unroll
      for (int I = 0; I < kG4Blocks; ++I) qa[I] = I < nbt ? Qt[buf][j][I][lane] : 0.0;
      int t = 0;
#pragma unroll
      for (int I = 0; I < kG4Blocks; ++I)
#pragma unroll
        for (int J = I; J < kG4Blocks; ++J, ++t)
          if ((t & 3) == w && J < nbt)
            acc[t >> 2] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[I], qa[J], acc[t >> 2], 0, 0, 0);
    }
    buf ^= 1;
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
  // tile (I, J): register v of lane l holds row 16 I + 4 v + l / 16, column 16 J + l % 16
  double* out = ws + L.gram;
  int t = 0;
#pragma unroll
  for (int I = 0; I < kG4Blocks; ++I)
#pragma unroll
    for (int J = I; J < kG4Blocks; ++J, ++t) {
      if ((t & 3) != w || J >= nbt) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + 4 * v + (lane >> 4), b = 16 * J + (lane & 15);
        if (a < g && b < g) {
          out[a * g + b] = acc[t >> 2][v];
          if (I != J) out[b * g + a] = acc[t >> 2][v];
        }
      }
    }
  if (threadIdx.x == 0) ws[L.info + 4] = 0.0;
}

// Eigenbasis Gram on the matrix cores: per 16-point chunk the kernel-space rows are staged in
// LDS (X[point][landmark]) and rotated, D = X U, with v_mfma_f64_16x16x4f64 (A = X in the
// operand layout row = point, k = 4 landmarks; B = U, kept in registers).  The result
// register v of lane l holds point 4 v + l / 16 and eigen-direction l % 16 of its block,
// which is again the operand layout of the Gram MFMAs with the four points of register v
// as the k dimension; columns m and m+1 take c_i and r_i before the Gram step.
template <int NB, int P, bool EX>
__global__ __launch_bounds__(64) void k_gram64_rot_mfma(const nyls_desc* __restrict__ desc,
                                                        const int32_t* __restrict__ order,
                                                        double* __restrict__ wsbase, int only) {
  constexpr int T = NB * (NB + 1) / 2;
  constexpr int KS = 4 * NB;        // k-steps of four landmarks
  constexpr int LDX = 16 * NB + 2;  // row stride of the staged rows
  __shared__ double X[16 * LDX];
  const nyls_desc& d = desc[instance_of(order)];
  if (d.p != P || d.rec != (EX ? 0 : 1) || nyls_slot_blocks(d.m + 2) != NB ||
      (d.flags & (NYLS_DF_GRAM_VALU | NYLS_DF_SPLIT)))
    return;
  const int m = d.m, n = d.n, g = m + 2;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  if (only && !((int)ws[L.info + 1] & only)) return;
  if (!use_eigenbasis(ws, L, only)) return;  // k_gram64_mfma
  const int lane = threadIdx.x;
  const int ks_end = (m + 3) >> 2;

  nyls_walk<NB, EX> wk;
  wk.init(d, lane);
  nyls_cpts cpt;
  cpt.init(d);
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  const double* U = ws + L.U;
  double ub[NB][KS];
#pragma unroll
  for (int kb = 0; kb < NB; ++kb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int s = 4 * ks + (lane >> 4), kk = 16 * kb + (lane & 15);
      ub[kb][ks] = (s < m && kk < m) ? U[s * m + kk] : 0.0;
    }
  nyls_d4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = nyls_d4{0.0, 0.0, 0.0, 0.0};

  double fj[P][4], rj[4];
  auto load = [&](int i0, double (&f)[P][4], double (&r_)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + 4 * j + wk.ph;
#pragma unroll
      for (int k = 0; k < P; ++k) f[k][j] = nyls_bload(fr, (k * n + i) * 8);
      r_[j] = nyls_bload(rr, i * 8);
    }
  };
  load(0, fj, rj);
  for (int i0 = 0; i0 < n; i0 += 16) {
    wk.advance(d, i0);
    double fn[P][4], rn[4];
    load(i0 + 16, fn, rn);
    bool okj[4];
    double q[NB];
    wk.chunk(
        d, i0,
        [&](int b, int j, double g, double e) {
          double h[P + 2];
          nyls_hfac<P>(g, inv_s2, h);
          double poly = h[P];
#pragma unroll
          for (int k = 1; k <= P; ++k) poly -= fj[k - 1][j] * h[P - k];
          q[b] = wk.lv[b] ? e * poly : 0.0;
        },
        [&](int j) {
          const int i = i0 + 4 * j + wk.ph;
          okj[j] = i < n && !cpt.has(i);
#pragma unroll
          for (int b = 0; b < NB; ++b) X[(4 * j + wk.ph) * LDX + 16 * b + wk.sl] = okj[j] ? q[b] : 0.0;
        });
    nyls_wave_lds_sync();
    nyls_d4 D[NB];
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) D[kb] = nyls_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks < ks_end) {
        const double a = X[(lane & 15) * LDX + 4 * ks + (lane >> 4)];
#pragma unroll
        for (int kb = 0; kb < NB; ++kb)
          D[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ub[kb][ks], D[kb], 0, 0, 0);
      }
    }
    nyls_wave_lds_sync();
    // columns m (c_i) and m + 1 (r_i); register v holds point 4 v + ph
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      const int kk = 16 * kb + (lane & 15);
      if (kk == m || kk == m + 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          D[kb][v] = okj[v] ? (kk == m ? -fj[P - 1][v] : rj[v]) : 0.0;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int t = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = I; J < NB; ++J) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(D[I][v], D[J][v], acc[t], 0, 0, 0);
          ++t;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int k = 0; k < P; ++k) fj[k][j] = fn[k][j];
      rj[j] = rn[j];
    }
  }
  double* out = ws + L.gram;
  int t = 0;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = I; J < NB; ++J) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + 4 * v + (lane >> 4), b = 16 * J + (lane & 15);
        if (a < g && b < g) {
          out[a * g + b] = acc[t][v];
          if (I != J) out[b * g + a] = acc[t][v];
        }
      }
      ++t;
    }
  if (lane == 0) ws[L.info + 4] = 1.0;
}

template <int NB, bool EX>
void launch_mfma_nbx(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  const dim3 grid(pv.batch), block(64);
  if (pv.p_mask & 2) hipLaunchKernelGGL((k_gram64_rot_mfma<NB, 1, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, pv.only);
  if (pv.p_mask & 4) hipLaunchKernelGGL((k_gram64_rot_mfma<NB, 2, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, pv.only);
  if (pv.p_mask & 8) hipLaunchKernelGGL((k_gram64_rot_mfma<NB, 3, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, pv.only);
  if (pv.p_mask & 16) hipLaunchKernelGGL((k_gram64_rot_mfma<NB, 4, EX>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, pv.only);
}

template <int NB>
void launch_mfma_nb(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  if (pv.rec_mask & 2) launch_mfma_nbx<NB, false>(pv, ws, st);
  if (pv.rec_mask & 1) launch_mfma_nbx<NB, true>(pv, ws, st);
}

template <int NB, bool EX, bool TLG>
void launch_ks_x(const nyls_plan_view& pv, double* ws, hipStream_t st, int only) {
  const dim3 grid(pv.batch), block(64);
  if (pv.p_mask & 2) hipLaunchKernelGGL((k_gram64_mfma<NB, 1, EX, TLG>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, only);
  if (pv.p_mask & 4) hipLaunchKernelGGL((k_gram64_mfma<NB, 2, EX, TLG>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, only);
  if (pv.p_mask & 8) hipLaunchKernelGGL((k_gram64_mfma<NB, 3, EX, TLG>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, only);
  if (pv.p_mask & 16) hipLaunchKernelGGL((k_gram64_mfma<NB, 4, EX, TLG>), grid, block, 0, st, pv.d_desc, pv.d_order, ws, only);
}

// kernel-space Grams, one launch set per column-block class present in the batch
template <int NB, bool TLG>
void launch_ks(const nyls_plan_view& pv, double* ws, hipStream_t st, int only) {
  if (!(pv.gcls_mask & (1u << (2 * NB + (TLG ? 1 : 0))))) return;
  if (pv.rec_mask & 2) launch_ks_x<NB, false, TLG>(pv, ws, st, only);
  if (pv.rec_mask & 1) launch_ks_x<NB, true, TLG>(pv, ws, st, only);
}

template <int P>
void launch_g4_p(const nyls_plan_view& pv, double* ws, hipStream_t st, int only) {
  if (!(pv.p_mask & (1u << P))) return;
  if (pv.rec_mask & 2)
    hipLaunchKernelGGL((k_gram64_mfma4<P, false>), dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, pv.d_order, ws, only);
  if (pv.rec_mask & 1)
    hipLaunchKernelGGL((k_gram64_mfma4<P, true>), dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, pv.d_order, ws, only);
}

void launch_g4_all(const nyls_plan_view& pv, double* ws, hipStream_t st, int only) {
  if (pv.maxm_narrow + 2 > 64) {  // four-wave MFMA Gram, 64 < m + 2 <= 128
    launch_g4_p<1>(pv, ws, st, only);
    launch_g4_p<2>(pv, ws, st, only);
    launch_g4_p<3>(pv, ws, st, only);
    launch_g4_p<4>(pv, ws, st, only);
  }
}

void launch_ks_all(const nyls_plan_view& pv, double* ws, hipStream_t st, int only) {
  launch_g4_all(pv, ws, st, only);
  launch_ks<1, false>(pv, ws, st, only);
  launch_ks<2, false>(pv, ws, st, only);
  launch_ks<2, true>(pv, ws, st, only);
  launch_ks<3, false>(pv, ws, st, only);
  launch_ks<3, true>(pv, ws, st, only);
  launch_ks<4, false>(pv, ws, st, only);
  launch_ks<4, true>(pv, ws, st, only);
}

}  // namespace

namespace {
size_t gram64_lds_bytes(int maxm, int TP, bool wide) {
  const int gp = (maxm + 2 + 3) & ~3;
  const int nb = gp >> 2;
  const size_t tile = (size_t)TP * gp, red = wide ? 0 : (size_t)nb * (nb + 1) / 2 * 16;
  // the rotated-row tile Q2 sits after the point flags at an offset that is independent of
  // the instance's own tile width; the reduction buffer may run into fr / tl / okp only
  const size_t base = tile * sizeof(double) + TP * (NYLS_MAX_P + 1) * sizeof(double) +
                      NYLS_MAX_M * sizeof(double) + TP * sizeof(int);
  size_t total = base + tile * sizeof(double) + (maxm <= 64 ? (size_t)maxm * maxm * sizeof(double) : 0);
  if (red * sizeof(double) > total) total = red * sizeof(double);
  return total;
}

// The LDS-tile Gram: TP = 64 for the bases up to NYLS_NARROW_MAX_M (smode 0: unsplit
// instances, one workgroup each; 1 / 2: split instances, one per chunk), TP = 32 for the wide
// bases (always split; grid z shares out the Gram's blocks).
template <int TP>
void launch_vg(const nyls_plan_view& pv, double* ws, hipStream_t st, int smode, int only) {
  constexpr bool wide = TP == 32;
  const int maxm = wide ? pv.maxm : pv.maxm_narrow;
  const bool split = smode == 1 || smode == 2;
  if (wide ? (!split || !(pv.nb_mask & (1u << 16))) : maxm == 0) return;
  if (split ? !pv.n_split : smode == 3 ? !pv.n_vks : (!pv.n_vgram && !pv.only)) return;
  const size_t lds = gram64_lds_bytes(maxm, TP, wide);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram64<TP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int gz = 1;
  if (wide) {
    const int nb = ((maxm + 2 + 3) & ~3) >> 2;
    gz = (nb * (nb + 1) / 2 + kWideBlocks - 1) / kWideBlocks;
  }
  const dim3 grid(pv.batch, split ? pv.max_chunks : 1, gz);
  hipLaunchKernelGGL(k_gram64<TP>, grid, dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order, ws, maxm,
                     only, smode);
}

// Chunk partials of the split instances (smode 1: kernel space, 2: eigenbasis where needed).
void launch_split_parts(const nyls_plan_view& pv, double* ws, hipStream_t st, int smode) {
  launch_vg<64>(pv, ws, st, smode, 0);
  launch_vg<32>(pv, ws, st, smode, 0);
}
}  // namespace

hipError_t nyls_launch_gram64_kspace(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  launch_ks_all(pv, ws, st, -1);
  launch_vg<64>(pv, ws, st, 3, 0);  // LDS-tile kernel-space Grams (m + 2 > 64, or by tuning)
  launch_split_parts(pv, ws, st, 1);
  return hipGetLastError();
}

hipError_t nyls_launch_gram64_over64(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  launch_g4_all(pv, ws, st, 0);   // kernel space on the matrix cores
  launch_vg<64>(pv, ws, st, 0, 0);  // eigenbasis where K_mm is ill-conditioned
  return hipGetLastError();
}

hipError_t nyls_launch_gram64(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  if (!pv.only) {
    launch_ks_all(pv, ws, st, 0);
    launch_split_parts(pv, ws, st, 1);
  } else {
    launch_g4_all(pv, ws, st, pv.only);  // re-solve: 64 < m + 2 <= 128 in kernel space
  }
  return nyls_launch_gram64_rest(pv, ws, st, false);
}

hipError_t nyls_launch_gram64_rest(const nyls_plan_view& pv, double* ws, hipStream_t st, bool ks_done) {
  if (pv.gnb_mask & 4) launch_mfma_nb<2>(pv, ws, st);
  if (pv.gnb_mask & 16) launch_mfma_nb<4>(pv, ws, st);
  // after nyls_launch_gram64_kspace the LDS-tile kernel-space Grams exist: only the
  // instances that need the eigenbasis are done again
  launch_vg<64>(pv, ws, st, (ks_done && !pv.only) ? 4 : 0, pv.only);
  if (pv.n_split && !pv.only) {
    launch_split_parts(pv, ws, st, 2);
    const int g = pv.maxm + 2;
    hipLaunchKernelGGL(k_gram_split_sum, dim3(pv.batch, (g * g + NYLS_BLOCK - 1) / NYLS_BLOCK),
                       dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws);
  }
  return hipGetLastError();
}
