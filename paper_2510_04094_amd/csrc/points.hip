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
// One wavefront per instance with the lane layout of nyls_walk.h: kernel values come from
// the Gaussian recurrence in registers, sums over landmarks are pre-reduced in registers and
// finished in a small LDS tile, sum_i rho_i p_i stays in registers for the whole pass.  The
// kernel is instantiated per ODE order P (only that order's Hermite factors are formed) and
// per number NB of 16-landmark slots per lane.
#include "nyls_dense.h"
#include "nyls_walk.h"

#include <type_traits>

namespace {

constexpr int NK = NYLS_MAX_M + 1 + NYLS_MAX_P;          // split instances (any basis)
constexpr int NKN = NYLS_NARROW_MAX_M + 1 + NYLS_MAX_P;  // one-wave instances

__device__ inline int instance_of(const int32_t* order, int single) {
  return single >= 0 ? single : (order ? order[blockIdx.x] : (int)blockIdx.x);
}

template <int NB, int P, bool EX, bool TL>
__global__ __launch_bounds__(64) void k_points(
    const nyls_desc* __restrict__ desc, const int32_t* __restrict__ order,
    double* __restrict__ wsbase, int refine, double* __restrict__ yhat,
    double* __restrict__ omega_out, double* __restrict__ bias_out, double* __restrict__ lambda_out,
    int32_t* __restrict__ status, int maxm, int single, double tol_stop, double tol_flag,
    int only) {
  __shared__ __align__(16) double tile[2 * 16 * NYLS_WALK_PAD];
  __shared__ double ttile[TL ? 2 * 64 : 1];
  __shared__ double bc[16];
  __shared__ double Rv[NKN], xv[NKN], zs[NYLS_NARROW_MAX_M];
  __shared__ int piv[NKN];

  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  if (d.p != P || d.rec != (EX ? 0 : 1) || nyls_slot_blocks(d.m) != NB ||
      (!EX && (d.flags & NYLS_DF_TAIL)) != TL || (d.flags & NYLS_DF_SPLIT))
    return;  // another launch handles this instance
  if (only && !((int)wsbase[d.ws + nyls_layout(d.m, P, 0).info + 1] & only)) return;
  const int m = d.m, n = d.n;
  const int N = m + 1 + P;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const double* LU = ws + L.lu;
  const int lane = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma;
  double* yo = yhat + d.goff;

  nyls_walk<NB, EX, TL> wk;
  wk.init(d, lane);
  nyls_cpts cpt;
  cpt.init(d);
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  const __amdgpu_buffer_rsrc_t yr = nyls_rsrc(yhat + d.goff, n * 8);
  double alv[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) alv[b] = wk.lv[b] ? ws[L.alpha + 16 * b + wk.sl] : 0.0;
  const int st_ = 16 * (NB - 1) + wk.tts;  // tail layout: this lane's tail landmark
  double alt = wk.tlv ? ws[L.alpha + st_] : 0.0;
  for (int e = lane; e < N; e += 64) {
    xv[e] = ws[L.x + e];
    piv[e] = (int)ws[L.piv + e];
  }
  __syncthreads();

  // One pass over the grid.  Always writes y_hat for the current (alpha, b); when refining
  // also forms rho_i = r_i - p_i^T alpha - c_i b and accumulates sum_i rho_i p_i (zacc, per
  // landmark slot and phase; zt for the lane's tail slot) and sum_i c_i rho_i (sacc, lanes
  // 0..15).
  nyls_oppoly<P> op;
  op.init(inv_s2);
  // operator data of a lane's points (f), of the point it finishes (r, c) and the previous
  // pass's y_hat of that point, loaded one chunk ahead into alternating stages
  struct stage {
    double f[P][4], ft[P];  // ft: operator data of the tail point (tail layout)
    double r, c, y;
  };
  auto pass = [&](auto REF, double b, double (&zacc)[NB], double& zt, double& sacc,
                  double& ymax, bool track, double& dmax) {
    constexpr bool refining = decltype(REF)::value;
    constexpr int Q = refining ? 2 : 1;
    auto load = [&](int i0, stage& st) {
      const int ip = i0 + (lane & 15);
      if (refining) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
          for (int j = 0; j < 4; ++j) st.f[k][j] = nyls_bload(fr, (k * n + i0 + 4 * j + wk.ph) * 8);
        st.r = nyls_bload(rr, ip * 8);
        st.c = -nyls_bload(fr, ((P - 1) * n + ip) * 8);
        if (TL)
#pragma unroll
          for (int k = 0; k < P; ++k) st.ft[k] = nyls_bload(fr, (k * n + i0 + wk.tpt) * 8);
      }
      st.y = track ? nyls_bload(yr, ip * 8) : 0.0;
    };
    auto body = [&](int i0, const stage& st) {
      wk.advance(d, i0);
      double cj[4][P];
      if (refining)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double f[P];
#pragma unroll
          for (int k = 0; k < P; ++k) f[k] = st.f[k][j];
          op.coef(f, cj[j]);
        }
      double pe[refining ? NB : 1][4];
      double acc0 = 0.0, acc1 = 0.0, pvt = 0.0;
      wk.chunk(
          d, i0,
          [&](int bb, int j, double g, double e) {
            if (refining) {
              const double pv = e * nyls_horner<P>(g, cj[j]);
              pe[refining ? bb : 0][j] = pv;
              acc1 += alv[bb] * pv;
            }
            acc0 += alv[bb] * e;
          },
          [&](int j) {
            nyls_walk_put(tile, lane, 0, j, acc0);
            if (refining) nyls_walk_put(tile, lane, 1, j, acc1);
            acc0 = acc1 = 0.0;
          },
          [&](double g, double e) {
            if (refining) {
              double ct[P];
              op.coef(st.ft, ct);
              pvt = e * nyls_horner<P>(g, ct);
              nyls_walk_put_tail(ttile, lane, 1, alt * pvt);
            }
            nyls_walk_put_tail(ttile, lane, 0, alt * e);
          });
      double tot[Q];
      if (TL) nyls_walk_sum_tail<Q>(tile, ttile, lane, tot);
      else nyls_walk_sum<Q>(tile, lane, tot);
      const int ip = i0 + (lane & 15);
      const double yv = tot[0] + b;
      if (ip < n) {
        if (lane < 16) {
          if (track) dmax = fmax(dmax, fabs(yv - st.y));
          yo[ip] = yv;
        }
        ymax = fmax(ymax, fabs(yv));
      }
      if (refining) {
        const bool okp = ip < n && !cpt.has(ip);
        const double rho = okp ? st.r - tot[Q - 1] - st.c * b : 0.0;
        if (lane < 16) sacc += st.c * rho;
        const double w1[1] = {rho};
        double rj[1][4], rt[1];
        if (TL) {
          nyls_walk_bcast_tail<1>(w1, bc, lane, rj, rt);
          zt += rt[0] * pvt;
        } else {
          nyls_walk_bcast<1>(w1, bc, lane, rj);
        }
#pragma unroll
        for (int bb = 0; bb < wk.NM; ++bb)
#pragma unroll
          for (int j = 0; j < 4; ++j) zacc[bb] += rj[0][j] * pe[refining ? bb : 0][j];
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
  };

  // Each pass writes y_hat of the current solution and, from the second on, measures how
  // far the previous correction moved it (dmax).  The iteration stops
  //  * after a solve, when the bound |d y_hat| <= |d omega|_2 + |d b| (phi(t)^T phi(t) is
  //    the Nystrom approximation of k(t, t) = 1 and never exceeds it) is below tol_stop:
  //    the y_hat just written is final;
  //  * before a solve, when the measured change is below tol_stop, or above half the
  //    previous one (the FP64 residual has reached its rounding floor): y_hat and the
  //    solution of this pass are kept.
  //  * after a solve, when the change this correction will make is predicted below
  //    tol_stop: the change just measured (of the previous correction) times the ratio of
  //    the two corrections' bounds, i.e. the contraction of the iteration seen so far.
  //    Then no further residual is formed, but the output pass still applies the correction.
  // Otherwise (or when the step limit is reached) the last correction is followed by an
  // output pass, which also measures it.
  double corr = 0.0, dprev = 0.0, ymax = 0.0, bprev = 0.0;
  bool need_output = true;
  int passes = 0;
  for (int step = 0; step < refine; ++step) {
    double zacc[NB], zt = 0.0, sacc = 0.0, dmax = 0.0;
    ymax = 0.0;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) zacc[bb] = 0.0;
    pass(std::true_type{}, xv[m], zacc, zt, sacc, ymax, step > 0, dmax);
    ++passes;
    ymax = nyls_wave_max(ymax);
    if (step > 0) {
      dmax = nyls_wave_max(dmax);
      const bool stalled = step > 1 && dmax > 0.5 * dprev;
      dprev = corr = dmax;
      if (dmax <= tol_stop * ymax || stalled) {
        need_output = false;
        break;
      }
    }
#pragma unroll
    for (int bb = 0; bb < wk.NM; ++bb) {
      const double zb = nyls_walk_fold(zacc[bb]);
      if (wk.ph == 0 && wk.lv[bb]) zs[16 * bb + wk.sl] = zb;
    }
    if (TL) {
      const double ztot = nyls_tail_fold(zt);
      if (lane < 4 && wk.tlv) zs[st_] = ztot;
    }
    const double ssum = nyls_wave_sum(sacc);
    __syncthreads();
    for (int e = lane; e < N; e += 64) {
      double val = 0.0;
      if (e < m) {
        if (e < r) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + e] * zs[s];
          val = gam * acc - xv[e];
          for (int j = 0; j < P; ++j) val -= ws[L.H + j * m + e] * xv[m + 1 + j];
        }
      } else if (e == m) {
        val = gam * ssum;
        for (int j = 0; j < P; ++j) val -= (d.cond_d[j] == 0 ? 1.0 : 0.0) * xv[m + 1 + j];
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
    for (int bb = 0; bb < NB; ++bb) {
      const int s = 16 * bb + wk.sl;
      if (wk.lv[bb]) {
        double acc = 0.0;
        for (int k = 0; k < r; ++k) acc += W[s * m + k] * xv[k];
        alv[bb] = acc;
      }
    }
    if (TL && wk.tlv) {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc += W[st_ * m + k] * xv[k];
      alt = acc;
    }
    double dsq = 0.0;
    for (int k = lane; k < r; k += 64) dsq += Rv[k] * Rv[k];
    const double bound = sqrt(nyls_wave_sum(dsq)) + fabs(Rv[m]);
    if (bound <= tol_stop * ymax) {
      corr = bound;
      need_output = false;
      break;
    }
    // predicted to be the last correction: the output pass below applies it to y_hat and
    // measures it (so y_hat, x and alpha agree, and the recorded change is a measured one)
    const double pred = step > 0 && bprev > 0.0 ? corr * (bound / bprev) : bound;
    if (pred <= tol_stop * ymax) break;
    bprev = bound;
  }
  if (need_output) {
    double zacc[NB], zt = 0.0, sacc = 0.0, dmax = 0.0;
    ymax = 0.0;
    pass(std::false_type{}, xv[m], zacc, zt, sacc, ymax, refine > 0, dmax);
    ymax = nyls_wave_max(ymax);
    corr = nyls_wave_max(dmax);
  }

  for (int e = lane; e < N; e += 64) ws[L.x + e] = xv[e];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb)
    if (wk.ph == 0 && wk.lv[bb]) ws[L.alpha + 16 * bb + wk.sl] = alv[bb];
  if (omega_out)
    for (int k = lane; k < maxm; k += 64) omega_out[(size_t)inst * maxm + k] = k < m ? xv[k] : 0.0;
  if (lambda_out && lane < NYLS_MAX_P)
    lambda_out[(size_t)inst * NYLS_MAX_P + lane] = lane < P ? xv[m + 1 + lane] : 0.0;
  if (lane == 0) {
    if (bias_out) bias_out[inst] = xv[m];
    int bits = (int)ws[L.info + 1] & ~NYLS_S_REFINE_NOCONV;
    if (only) bits |= NYLS_S_FP64_RESOLVED;
    if (!(fabs(xv[m]) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    if (refine > 0 && corr > tol_flag * ymax) bits |= NYLS_S_REFINE_NOCONV;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 3] = corr;
    ws[L.info + 5] = (double)passes;
    if (status) status[inst] = bits;
  }
}

// ---- instances split over point chunks (NYLS_DF_SPLIT) ----------------------------------
//
// The same passes with one workgroup (one wavefront) per chunk of d.chunk grid points: each
// pass writes y_hat of its points and its partial sums (sum rho_i p_i per landmark,
// sum c_i rho_i, max |y_hat|, max change of y_hat) to the instance's partial area;
// k_combine_split then adds the chunks in chunk order and takes the refinement step of
// k_points (same stopping rules), keeping the iteration's state in the instance's
// accumulator block between launches.
enum { SS_DONE = 0, SS_NEEDOUT, SS_CORR, SS_DPREV, SS_BPREV, SS_PASSES, SS_YMAX };

__global__ void k_split_init(const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const nyls_desc& d = desc[i];
  if (!(d.flags & NYLS_DF_SPLIT)) return;
  double* st = wsbase + d.ws + nyls_layout(d.m, d.p, 0).acc;
  st[SS_DONE] = 0.0;
  st[SS_NEEDOUT] = 1.0;
  st[SS_CORR] = st[SS_DPREV] = st[SS_BPREV] = st[SS_PASSES] = st[SS_YMAX] = 0.0;
}

// G = 2: wide bases (m > NYLS_NARROW_MAX_M), two wavefronts per chunk, wavefront w walking
// the landmark slots 16 NB w .. 16 NB (w + 1) - 1; the per-point sums over the landmarks are
// joined through LDS (nyls_walk_join), after which both wavefronts hold the same residuals
// and each accumulates the landmark sums of its own slots.
template <int NB, int P, bool EX, bool REF, int G = 1>
__global__ __launch_bounds__(64 * G) void k_pass_split(const nyls_desc* __restrict__ desc,
                                                       double* __restrict__ wsbase,
                                                       double* __restrict__ yhat, int track) {
  constexpr int Q = REF ? 2 : 1;
  __shared__ __align__(16) double tiles[G][2 * 16 * NYLS_WALK_PAD];
  __shared__ double bcs[G][16];
  __shared__ double xw[G > 1 ? 2 * G * Q * 16 : 1];
  const nyls_desc& d = desc[blockIdx.x];
  if (!(d.flags & NYLS_DF_SPLIT) || d.p != P || d.rec != (EX ? 0 : 1) ||
      nyls_slot_blocks(d.m) != NB * G)
    return;
  const int c = (int)blockIdx.y;
  if (c >= d.nchunks) return;
  const int m = d.m, n = d.n;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* sst = ws + L.acc;
  if (REF ? sst[SS_DONE] != 0.0 : sst[SS_NEEDOUT] == 0.0) return;
  const int lane = threadIdx.x & 63, grp = G > 1 ? (int)(threadIdx.x >> 6) : 0;
  const int s0 = 16 * NB * grp;  // first landmark slot of this wavefront
  double* const tile = tiles[grp];
  double* const bc = bcs[grp];
  const bool lead = grp == 0;  // writes the per-point outputs and scalar sums
  const int ibeg = c * d.chunk, iend = min(n, ibeg + d.chunk);
  double* yo = yhat + d.goff;

  nyls_walk<NB, EX> wk;
  wk.init(d, lane, s0);
  nyls_cpts cpt;
  cpt.init(d);
  const double inv_sigma = wk.inv_sigma, inv_s2 = inv_sigma * inv_sigma;
  const __amdgpu_buffer_rsrc_t fr = nyls_rsrc(d.f, P * n * 8), rr = nyls_rsrc(d.r, n * 8);
  const __amdgpu_buffer_rsrc_t yr = nyls_rsrc(yhat + d.goff, n * 8);
  double alv[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) alv[b] = wk.lv[b] ? ws[L.alpha + s0 + 16 * b + wk.sl] : 0.0;
  const double bias = ws[L.x + m];
  nyls_oppoly<P> op;
  op.init(inv_s2);
  double zacc[NB], sacc = 0.0, ymax = 0.0, dmax = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) zacc[b] = 0.0;
  int parity = 0;
  struct stage {
    double f[P][4];
    double r, c, y;
  };
  auto load = [&](int i0, stage& st) {
    const int ip = i0 + (lane & 15);
    if (REF) {
#pragma unroll
      for (int k = 0; k < P; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) st.f[k][j] = nyls_bload(fr, (k * n + i0 + 4 * j + wk.ph) * 8);
      st.r = nyls_bload(rr, ip * 8);
      st.c = -nyls_bload(fr, ((P - 1) * n + ip) * 8);
    }
    st.y = track ? nyls_bload(yr, ip * 8) : 0.0;
  };
  auto body = [&](int i0, const stage& st) {
    wk.advance(d, i0);
    double cj[4][P];
    if (REF)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double f[P];
#pragma unroll
        for (int k = 0; k < P; ++k) f[k] = st.f[k][j];
        op.coef(f, cj[j]);
      }
    double pe[REF ? NB : 1][4];
    double acc0 = 0.0, acc1 = 0.0;
    wk.chunk(
        d, i0,
        [&](int bb, int j, double g, double e) {
          if (REF) {
            const double pv = e * nyls_horner<P>(g, cj[j]);
            pe[REF ? bb : 0][j] = pv;
            acc1 += alv[bb] * pv;
          }
          acc0 += alv[bb] * e;
        },
        [&](int j) {
          nyls_walk_put(tile, lane, 0, j, acc0);
          if (REF) nyls_walk_put(tile, lane, 1, j, acc1);
          acc0 = acc1 = 0.0;
        });
    double tot[Q];
    nyls_walk_sum<Q>(tile, lane, tot);
    if constexpr (G > 1) {
      nyls_walk_join<G, Q>(tot, xw, lane, grp, parity);
      parity ^= 1;
    }
    const int ip = i0 + (lane & 15);
    const double yv = tot[0] + bias;
    if (ip < n) {
      if (lane < 16 && lead) {
        if (track) dmax = fmax(dmax, fabs(yv - st.y));
        yo[ip] = yv;
      }
      ymax = fmax(ymax, fabs(yv));
    }
    if (REF) {
      const bool okp = ip < n && !cpt.has(ip);
      const double rho = okp ? st.r - tot[Q - 1] - st.c * bias : 0.0;
      if (lane < 16) sacc += st.c * rho;
      const double w1[1] = {rho};
      double rj[1][4];
      nyls_walk_bcast<1>(w1, bc, lane, rj);
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
#pragma unroll
        for (int j = 0; j < 4; ++j) zacc[bb] += rj[0][j] * pe[REF ? bb : 0][j];
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
  double* part = wsbase + d.part + nyls_split_pass(m, d.nchunks, c);
  ymax = nyls_wave_max(ymax);
  dmax = nyls_wave_max(dmax);
  if (REF) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const double zb = nyls_walk_fold(zacc[bb]);
      if (wk.ph == 0 && wk.lv[bb]) part[s0 + 16 * bb + wk.sl] = zb;
    }
  }
  const double ssum = nyls_wave_sum(sacc);
  if (lane == 0 && lead) {
    part[m] = ssum;
    part[m + 1] = ymax;
    part[m + 2] = dmax;
  }
}

// One refinement step (fin == 0, step `step` of at most `refine`) or the final bookkeeping
// (fin == 1) of a split instance, one wavefront per instance.
template <int P>
__global__ __launch_bounds__(64) void k_combine_split(
    const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, int step, int refine, int fin,
    double* __restrict__ omega_out, double* __restrict__ bias_out, double* __restrict__ lambda_out,
    int32_t* __restrict__ status, int maxm, double tol_stop, double tol_flag) {
  __shared__ double Rv[NK], xv[NK], zs[NYLS_MAX_M];
  __shared__ int piv[NK];
  const int inst = (int)blockIdx.x;
  const nyls_desc& d = desc[inst];
  if (!(d.flags & NYLS_DF_SPLIT) || d.p != P) return;
  const int m = d.m, N = m + 1 + P, nc = d.nchunks;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  double* sst = ws + L.acc;
  const double* part = wsbase + d.part;
  const int lane = threadIdx.x;
  auto pmax = [&](int k) {  // max over the chunks of pass-partial entry m + k
    double v = 0.0;
    for (int c = lane; c < nc; c += 64) v = fmax(v, part[nyls_split_pass(m, nc, c) + m + k]);
    return nyls_wave_max(v);
  };
  if (fin) {
    double ymax = sst[SS_YMAX], corr = sst[SS_CORR];
    if (sst[SS_NEEDOUT] != 0.0) {  // the output pass ran: it measured the last correction
      ymax = pmax(1);
      corr = pmax(2);
    }
    const double bias = ws[L.x + m];
    if (omega_out)
      for (int k = lane; k < maxm; k += 64) omega_out[(size_t)inst * maxm + k] = k < m ? ws[L.x + k] : 0.0;
    if (lambda_out && lane < NYLS_MAX_P)
      lambda_out[(size_t)inst * NYLS_MAX_P + lane] = lane < P ? ws[L.x + m + 1 + lane] : 0.0;
    if (lane == 0) {
      if (bias_out) bias_out[inst] = bias;
      int bits = (int)ws[L.info + 1] & ~NYLS_S_REFINE_NOCONV;
      if (!(fabs(bias) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
      if (refine > 0 && corr > tol_flag * ymax) bits |= NYLS_S_REFINE_NOCONV;
      ws[L.info + 1] = (double)bits;
      ws[L.info + 3] = corr;
      ws[L.info + 5] = sst[SS_PASSES];
      if (status) status[inst] = bits;
    }
    return;
  }
  if (sst[SS_DONE] != 0.0) return;
  const double ymax = pmax(1);
  const double dmax = pmax(2);
  double corr = sst[SS_CORR], dprev = sst[SS_DPREV], bprev = sst[SS_BPREV];
  bool done = false, needout = true;
  auto save = [&]() {
    if (lane == 0) {
      sst[SS_DONE] = done ? 1.0 : 0.0;
      sst[SS_NEEDOUT] = needout ? 1.0 : 0.0;
      sst[SS_CORR] = corr;
      sst[SS_DPREV] = dprev;
      sst[SS_BPREV] = bprev;
      sst[SS_PASSES] += 1.0;
      sst[SS_YMAX] = ymax;
    }
  };
  if (step > 0) {
    const bool stalled = step > 1 && dmax > 0.5 * dprev;
    dprev = corr = dmax;
    if (dmax <= tol_stop * ymax || stalled) {
      done = true;
      needout = false;
      save();
      return;
    }
  }
  // the residual from the chunk sums (added in chunk order), as in k_points
  const int r = (int)ws[L.info + 0];
  const double* W = ws + L.W;
  for (int s = lane; s < m; s += 64) {
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) acc += part[nyls_split_pass(m, nc, c) + s];
    zs[s] = acc;
  }
  double ssum = 0.0;
  if (lane == 0)
    for (int c = 0; c < nc; ++c) ssum += part[nyls_split_pass(m, nc, c) + m];
  ssum = nyls_rdlane(ssum, 0);
  for (int e = lane; e < N; e += 64) {
    xv[e] = ws[L.x + e];
    piv[e] = (int)ws[L.piv + e];
  }
  __syncthreads();
  const double gam = d.gamma;
  for (int e = lane; e < N; e += 64) {
    double val = 0.0;
    if (e < m) {
      if (e < r) {
        double acc = 0.0;
        for (int s = 0; s < m; ++s) acc += W[s * m + e] * zs[s];
        val = gam * acc - xv[e];
        for (int j = 0; j < P; ++j) val -= ws[L.H + j * m + e] * xv[m + 1 + j];
      }
    } else if (e == m) {
      val = gam * ssum;
      for (int j = 0; j < P; ++j) val -= (d.cond_d[j] == 0 ? 1.0 : 0.0) * xv[m + 1 + j];
    } else {
      const int j = e - m - 1;
      val = d.v[j] - (d.cond_d[j] == 0 ? xv[m] : 0.0);
      for (int k = 0; k < r; ++k) val -= ws[L.H + j * m + k] * xv[k];
    }
    Rv[e] = val;
  }
  __syncthreads();
  nyls_lu_solve_w(ws + L.lu, N, N, piv, Rv);
  for (int e = lane; e < N; e += 64) {
    xv[e] += Rv[e];
    ws[L.x + e] = xv[e];
  }
  __syncthreads();
  for (int s = lane; s < m; s += 64) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * xv[k];
    ws[L.alpha + s] = acc;
  }
  double dsq = 0.0;
  for (int k = lane; k < r; k += 64) dsq += Rv[k] * Rv[k];
  const double bound = sqrt(nyls_wave_sum(dsq)) + fabs(Rv[m]);
  if (bound <= tol_stop * ymax) {
    corr = bound;
    done = true;
    needout = false;
  } else {
    const double pred = step > 0 && bprev > 0.0 ? corr * (bound / bprev) : bound;
    if (pred <= tol_stop * ymax) done = true;
    bprev = bound;
  }
  if (step + 1 >= refine) done = true;  // step limit: the output pass applies the correction
  save();
}

template <int NB, bool EX, bool TL>
void launch_nbx(const nyls_plan_view& pv, double* ws, int refine, double* yhat, double* omega,
                double* bias, double* lambda, int32_t* status, int single, double ts, double tf,
                hipStream_t st) {
  const dim3 grid(single >= 0 ? 1 : pv.batch);
  if (pv.p_mask & 2)
    hipLaunchKernelGGL((k_points<NB, 1, EX, TL>), grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws,
                       refine, yhat, omega, bias, lambda, status, pv.maxm, single, ts, tf, pv.only);
  if (pv.p_mask & 4)
    hipLaunchKernelGGL((k_points<NB, 2, EX, TL>), grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws,
                       refine, yhat, omega, bias, lambda, status, pv.maxm, single, ts, tf, pv.only);
  if (pv.p_mask & 8)
    hipLaunchKernelGGL((k_points<NB, 3, EX, TL>), grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws,
                       refine, yhat, omega, bias, lambda, status, pv.maxm, single, ts, tf, pv.only);
  if (pv.p_mask & 16)
    hipLaunchKernelGGL((k_points<NB, 4, EX, TL>), grid, dim3(64), 0, st, pv.d_desc, pv.d_order, ws,
                       refine, yhat, omega, bias, lambda, status, pv.maxm, single, ts, tf, pv.only);
}

template <int NB>
hipError_t launch_nb(const nyls_plan_view& pv, double* ws, int refine, double* yhat, double* omega,
                     double* bias, double* lambda, int32_t* status, int single, hipStream_t st) {
  // Refinement stops once the change of y_hat falls below tol_stop max|y_hat| and flags
  // instances whose last change stayed above tol_flag.  Both modes refine to the same
  // level: the adjoint's residual terms (dl/dgamma) need the forward solution to FP64
  // accuracy, whatever precision the factorisation had.
  const double ts = 1e-11, tf = 1e-8;
  if ((pv.rec_mask & 2) && (pv.ntl_mask & (1u << NB)))
    launch_nbx<NB, false, false>(pv, ws, refine, yhat, omega, bias, lambda, status, single, ts, tf, st);
  if (pv.tl_mask & (1u << NB))
    launch_nbx<NB, false, true>(pv, ws, refine, yhat, omega, bias, lambda, status, single, ts, tf, st);
  if (pv.rec_mask & 1)
    launch_nbx<NB, true, false>(pv, ws, refine, yhat, omega, bias, lambda, status, single, ts, tf, st);
  return hipGetLastError();
}

}  // namespace

namespace {
// NB: slot blocks of the instance class (16: wide bases, two wavefronts of eight blocks)
template <int NB, int P, bool EX>
void launch_pass_split(const nyls_plan_view& pv, double* ws, double* yhat, bool ref, int track,
                       hipStream_t st) {
  constexpr int G = NB > 8 ? NB / 8 : 1, NW = NB / G;
  const dim3 grid(pv.batch, pv.max_chunks), block(64 * G);
  if (ref) hipLaunchKernelGGL((k_pass_split<NW, P, EX, true, G>), grid, block, 0, st, pv.d_desc, ws, yhat, track);
  else hipLaunchKernelGGL((k_pass_split<NW, P, EX, false, G>), grid, block, 0, st, pv.d_desc, ws, yhat, track);
}

template <int NB, int P>
void launch_pass_split_p(const nyls_plan_view& pv, double* ws, double* yhat, bool ref, int track,
                         hipStream_t st) {
  if (!(pv.p_mask & (1u << P))) return;
  if (pv.rec_mask & 2) launch_pass_split<NB, P, false>(pv, ws, yhat, ref, track, st);
  if (pv.rec_mask & 1) launch_pass_split<NB, P, true>(pv, ws, yhat, ref, track, st);
}

template <int NB>
void launch_pass_split_nb(const nyls_plan_view& pv, double* ws, double* yhat, bool ref, int track,
                          hipStream_t st) {
  if (!(pv.nb_mask & (1u << NB))) return;
  launch_pass_split_p<NB, 1>(pv, ws, yhat, ref, track, st);
  launch_pass_split_p<NB, 2>(pv, ws, yhat, ref, track, st);
  launch_pass_split_p<NB, 3>(pv, ws, yhat, ref, track, st);
  launch_pass_split_p<NB, 4>(pv, ws, yhat, ref, track, st);
}

void launch_combine(const nyls_plan_view& pv, double* ws, int step, int refine, int fin, double* omega,
                    double* bias, double* lambda, int32_t* status, double ts, double tf, hipStream_t st) {
  const dim3 grid(pv.batch);
  if (pv.p_mask & 2) hipLaunchKernelGGL(k_combine_split<1>, grid, dim3(64), 0, st, pv.d_desc, ws, step, refine, fin, omega, bias, lambda, status, pv.maxm, ts, tf);
  if (pv.p_mask & 4) hipLaunchKernelGGL(k_combine_split<2>, grid, dim3(64), 0, st, pv.d_desc, ws, step, refine, fin, omega, bias, lambda, status, pv.maxm, ts, tf);
  if (pv.p_mask & 8) hipLaunchKernelGGL(k_combine_split<3>, grid, dim3(64), 0, st, pv.d_desc, ws, step, refine, fin, omega, bias, lambda, status, pv.maxm, ts, tf);
  if (pv.p_mask & 16) hipLaunchKernelGGL(k_combine_split<4>, grid, dim3(64), 0, st, pv.d_desc, ws, step, refine, fin, omega, bias, lambda, status, pv.maxm, ts, tf);
}

// The refinement and output passes of the split instances: at most `refine` (pass, step)
// pairs, then the output pass and the final bookkeeping; launches of instances that have
// stopped return at once.
void launch_split_points(const nyls_plan_view& pv, double* ws, int refine, double* yhat, double* omega,
                         double* bias, double* lambda, int32_t* status, hipStream_t st) {
  const double ts = 1e-11, tf = 1e-8;  // as in launch_nb
  hipLaunchKernelGGL(k_split_init, dim3((pv.batch + 255) / 256), dim3(256), 0, st, pv.d_desc, ws, pv.batch);
  auto pass = [&](bool ref, int track) {
    launch_pass_split_nb<2>(pv, ws, yhat, ref, track, st);
    launch_pass_split_nb<4>(pv, ws, yhat, ref, track, st);
    launch_pass_split_nb<8>(pv, ws, yhat, ref, track, st);
    launch_pass_split_nb<16>(pv, ws, yhat, ref, track, st);
  };
  for (int step = 0; step < refine; ++step) {
    pass(true, step > 0);
    launch_combine(pv, ws, step, refine, 0, omega, bias, lambda, status, ts, tf, st);
  }
  pass(false, refine > 0);
  launch_combine(pv, ws, 0, refine, 1, omega, bias, lambda, status, ts, tf, st);
}
}  // namespace

hipError_t nyls_launch_points(const nyls_plan_view& pv, double* ws, int refine, double* yhat,
                              double* omega, double* bias, double* lambda, int32_t* status,
                              int single, hipStream_t st, unsigned classes) {
  const unsigned nb = pv.nb_mask & classes;
  if (nb & 4) launch_nb<2>(pv, ws, refine, yhat, omega, bias, lambda, status, single, st);
  if (nb & 16) launch_nb<4>(pv, ws, refine, yhat, omega, bias, lambda, status, single, st);
  if (nb & 256) launch_nb<8>(pv, ws, refine, yhat, omega, bias, lambda, status, single, st);
  if ((classes & 1) && pv.n_split && single < 0 && !pv.only)
    launch_split_points(pv, ws, refine, yhat, omega, bias, lambda, status, st);
  return hipGetLastError();
}
