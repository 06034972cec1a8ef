// One-wavefront-per-instance passes over the collocation grid.
//
// Lane geometry: lane = 16 ph + sl.  A lane owns the landmarks s = 16 b + sl (b < NB) and,
// inside a chunk of 16 consecutive grid points i0 .. i0 + 15, the four points
// i0 + 4 j + ph (j < 4): it produces a 4 x NB block of (point, landmark) values per chunk.
//  * Sums over the landmarks (dot products with alpha, beta) are first reduced in registers
//    over the lane's NB landmarks, then over the 16 landmark slots through a small padded
//    LDS tile (nyls_walk_reduce); afterwards lane l holds the totals of point l & 15.
//  * Per-point scalars computed by those lanes go back to the lanes that own the point
//    (nyls_walk_bcast), and sums over the points (sum_i rho_i p_i and the like) stay in
//    registers until the pass ends, when two shuffles fold the four phases.
// A single wavefront needs no workgroup-wide synchronisation, and the LDS footprint stays
// at a few KiB, so many instances share a compute unit.
//
// Kernel values: on a uniform grid t_i - t_s = k dt with k = i - i_s.  Along one lane's
// points k advances by 4, so with a = dt / sigma
//     e(k + 4) = e(k) R(k),  R(k) = exp(-a^2 (8 k + 16)),  R(k + 4) = R(k) exp(-32 a^2),
// restarted with two exponentials every 64 points (runs of 16 values per lane).  R is
// carried as rho = R - 1 (nyls_gauss_start / nyls_gauss_step), which keeps the run's
// relative error at the level of independent roundings.  Next to e the walk carries
// g = -2 (t_i - t_s) / sigma^2, the first Hermite factor, which also advances by a constant.
#pragma once
#include "nyls_internal.h"

constexpr int NYLS_WALK_PAD = 18;  // LDS row stride (doubles) of the reduction tile

// Hermite factors h_q = (-1/sigma)^q H_q(z), q = 0..P, so that the q-th t-derivative of
// K(t, t_s) is h_q e.  With g = -2 z / sigma: h_0 = 1, h_1 = g,
// h_{q+1} = g h_q - (2 q / sigma^2) h_{q-1}.
template <int P>
__device__ inline void nyls_hfac(double g, double inv_s2, double (&h)[P + 2]) {
  h[0] = 1.0;
  h[1] = g;
#pragma unroll
  for (int q = 1; q <= P; ++q) h[q + 1] = g * h[q] - (2.0 * q * inv_s2) * h[q - 1];
}

// The same factors as polynomials in g, h_q = sum_k H[q][k] g^k (H[q][k] = 0 unless q - k is
// even), and the operator polynomial of one point,
//     h_P(g) - sum_{i=1..P} f_i h_{P-i}(g) = g^P + sum_{k<P} c_k g^k,
// so that p_i = e * poly(g) costs P multiply-adds per (point, landmark) pair (Horner).
template <int P>
struct nyls_oppoly {
  double H[P + 2][P + 2];
  double s2;

  __device__ void init(double inv_s2) {
    s2 = inv_s2;
#pragma unroll
    for (int q = 0; q <= P + 1; ++q)
#pragma unroll
      for (int k = 0; k <= P + 1; ++k) H[q][k] = 0.0;
    H[0][0] = 1.0;
    H[1][1] = 1.0;
#pragma unroll
    for (int q = 1; q <= P; ++q)
#pragma unroll
      for (int k = 0; k <= q + 1; ++k)
        if (((q + 1 - k) & 1) == 0)
          H[q + 1][k] = (k >= 1 ? H[q][k - 1] : 0.0) - (k <= q - 1 ? 2.0 * q * inv_s2 * H[q - 1][k] : 0.0);
  }

  // Monic D(g) of degree P + 2 with d/dsigma of p_i = e * (sigma / 2) * D(g):
  // with z = -sigma g / 2, -(sa / sigma + z sb) = (sigma / 2) (g sb(g) - 2 s2 sa(g)),
  // sa = sum_q q w_q h_q and sb = sum_q w_q h_{q+1} (w_P = 1, w_q = -f_{P-q}).  Returns the
  // coefficients d_0 .. d_{P+1} for the operator weights f_1 .. f_P of one point.
  __device__ void dcoef(const double (&f)[P], double (&c)[P + 2]) const {
#pragma unroll
    for (int k = 0; k <= P + 1; ++k) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q <= P; ++q) {
        if (((q - k) & 1) != 0) continue;  // both terms vanish unless q - k is even
        const double e_qk = (k >= 1 && k - 1 <= q + 1 ? H[q + 1][k - 1] : 0.0) -
                            (q > 0 && k <= q ? 2.0 * q * s2 * H[q][k] : 0.0);
        v += (q == P ? 1.0 : -f[P - q - 1]) * e_qk;
      }
      c[k] = v;
    }
  }

  // coefficients c_0 .. c_{P-1} for the operator weights f_1 .. f_P of one point
  __device__ void coef(const double (&f)[P], double (&c)[P]) const {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      double v = (((P - k) & 1) == 0) ? H[P][k] : 0.0;
#pragma unroll
      for (int i = 1; i <= P; ++i)
        if (k <= P - i && ((P - i - k) & 1) == 0) v -= f[i - 1] * H[P - i][k];
      c[k] = v;
    }
  }
};

// Monic polynomial g^D + sum_{k<D} c_k g^k by Horner's rule (D multiply-adds).
template <int D>
__device__ inline double nyls_horner(double g, const double (&c)[D]) {
  double v = g + c[D - 1];
#pragma unroll
  for (int k = D - 2; k >= 0; --k) v = fma(v, g, c[k]);
  return v;
}

// EX = false: only for instances with nyls_desc::rec == 1 (no exact-exponential path).
// TL: the last block holds nyls_walk_tail(m) landmarks and is walked in the tail layout:
// lane = 4 pt + ts takes tail slot ts (landmark 16 (NB - 1) + ts, used when below m) for the
// single chunk point i0 + pt, 16 points further each chunk:
//     e(k + 16) = e(k) R16(k),  R16(k) = exp(-a^2 (32 k + 256)),  R16(k + 16) = R16(k) exp(-512 a^2),
// (R16 carried as R16 - 1), restarted with the other runs every 64 points.  The per-lane
// arrays keep all NB blocks (the landmark data of the last block stays usable in the block
// layout).
template <int NB, bool EX, bool TL = false>
struct nyls_walk {
  static_assert(!(TL && EX), "the tail layout is for instances with rec == 1");
  static constexpr int NM = TL ? NB - 1 : NB;  // blocks walked pair by pair
  int sl, ph, n;
  bool lv[NB];
  int ls[NB];
  double ev[NB], rv[NB], gc[NB];  // e, rho = R - 1 and g of the lane's run per block
  bool exact;  // wave-uniform: this run of 64 points uses one exponential per value
  double ga4, q4, q4m1, inv_sigma, a, gk;  // gk: g per grid step k; q4m1 = q4 - 1
  __amdgpu_buffer_rsrc_t tr;  // grid times (non-uniform grids)
  int tpt, tts, tls;          // tail layout: chunk point, tail slot, landmark grid index
  bool tlv;
  double te, tr16, tg, q16, q16m1, g16;

  // s0: first landmark of the lane's slots (0, or 16 NB for the second wavefront of a wide
  // basis); slot b of the lane is landmark s0 + 16 b + sl.
  __device__ __attribute__((always_inline)) void init(const nyls_desc& d, int lane, int s0 = 0) {
    sl = lane & 15;
    ph = lane >> 4;
    n = d.n;
    inv_sigma = 1.0 / d.sigma;
    a = d.dt * inv_sigma;
    gk = -2.0 * inv_sigma * a;
    ga4 = 4.0 * gk;
    q4 = exp(-32.0 * a * a);
    q4m1 = expm1(-32.0 * a * a);
    exact = EX && !d.uniform;
    tr = nyls_rsrc(EX && !d.uniform ? d.t : nullptr, EX && !d.uniform ? n * 8 : 0);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int s = s0 + 16 * b + sl;
      lv[b] = s < d.m;
      ls[b] = lv[b] ? d.lidx[s] : 0;
      ev[b] = rv[b] = gc[b] = 0.0;
    }
    tpt = lane >> 2;
    tts = lane & 3;
    tlv = TL && 16 * (NB - 1) + tts < d.m;
    tls = tlv ? d.lidx[16 * (NB - 1) + tts] : 0;
    q16 = TL ? exp(-512.0 * a * a) : 0.0;
    q16m1 = TL ? expm1(-512.0 * a * a) : 0.0;
    g16 = 16.0 * gk;
    te = tr16 = tg = 0.0;
  }

  // Must be called before chunk(i0) for every chunk, in increasing order from i0 = 0:
  // starts a new run of the recurrence every 64 points (and decides, wave-uniformly,
  // whether that run needs one exponential per value instead).
  __device__ __attribute__((always_inline)) void advance(const nyls_desc& d, int i0) {
    if ((!EX || d.uniform) && (i0 & 63) == 0) {
      bool any = false;
      if (TL) {
        // a tail run holds four values: z falls by at most 48 a <= 12 along it, so a run
        // starting below exp(-700) while approaching stays below exp(-200) and is set to zero
        const int k0 = i0 + tpt - tls;
        const double z0 = (double)k0 * a;
        const bool far = k0 < 0 && z0 * z0 > 700.0;
        const double e0 = exp(-z0 * z0), r0 = expm1(-a * a * (32.0 * k0 + 256.0));
        te = far ? 0.0 : e0;
        tr16 = far ? -1.0 : r0;
        tg = (double)k0 * gk;
      }
#pragma unroll
      for (int b = 0; b < NM; ++b) {
        const int k0 = i0 + ph - ls[b];
        if (EX) {
          any |= nyls_gauss_start(k0, 16, 4, a, ev[b], rv[b]);
        } else {
          // rec == 1 (a <= 1/4): a run that starts below exp(-700) while approaching its
          // landmark stays below exp(-132) (z falls by at most 60 a <= 15), so it is set to
          // zero; every other run starts from normal numbers and its ratio cannot overflow.
          const double z0 = (double)k0 * a;
          const bool far = k0 < 0 && z0 * z0 > 700.0;
          const double e0 = exp(-z0 * z0), r0 = expm1(-a * a * 4.0 * (2.0 * k0 + 4.0));
          ev[b] = far ? 0.0 : e0;
          rv[b] = far ? -1.0 : r0;
        }
        gc[b] = (double)k0 * gk;
      }
      if (EX) exact = __ballot(any) != 0;
    }
  }

  // Calls emit(b, j, g, e) for every landmark slot b < NB and point j < 4 of the chunk at
  // i0: g = -2 (t_i - t_s) / sigma^2 and e = exp(-((t_i - t_s) / sigma)^2) for
  // i = i0 + 4 j + ph, then done(j) once all slots of point j were emitted.  Past the end of
  // the grid the values are meaningless (but finite); callers ignore them.
  // With TL, blocks b < NB - 1 are emitted this way and tail(g, e) is called once for the
  // lane's tail pair (point i0 + tpt, landmark 16 (NB - 1) + tts).
  template <class Emit, class Done, class Tail>
  __device__ __attribute__((always_inline)) void chunk(const nyls_desc& d, int i0, Emit emit, Done done, Tail tail) {
    if (!EX || !exact) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int b = 0; b < NM; ++b) {
          emit(b, j, gc[b], ev[b]);
          nyls_gauss_step(ev[b], rv[b], q4, q4m1);
          gc[b] += ga4;
        }
        done(j);
      }
      if (TL) {
        tail(tg, te);
        nyls_gauss_step(te, tr16, q16, q16m1);
        tg += g16;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = i0 + 4 * j + ph;
        const double ti = d.uniform ? 0.0 : nyls_bload(tr, i * 8);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double z = d.uniform ? (double)(i - ls[b]) * a
                                     : (ti - nyls_grid_t(d, ls[b])) * inv_sigma;
          emit(b, j, -2.0 * inv_sigma * z, exp(-z * z));
        }
        done(j);
      }
    }
  }

  template <class Emit, class Done>
  __device__ __attribute__((always_inline)) void chunk(const nyls_desc& d, int i0, Emit emit, Done done) {
    static_assert(!TL, "the tail layout needs a tail callback");
    chunk(d, i0, emit, done, [](double, double) {});
  }
};

// v + (v of lane l ^ 32), and v + (v of lane l ^ 16).  Both lanes of a pair add the lower
// lane's value first, so they hold bitwise equal sums.
__device__ inline double nyls_add_xor32(double v) {
  double a, b;
  nyls_pair_xor32(v, a, b);
  return a + b;
}

__device__ inline double nyls_add_xor16(double v) {
  double a, b;
  nyls_pair_xor16(v, a, b);
  return a + b;
}

// Sums over the 16 landmark slots, in two steps: every lane stores its partial (over its NB
// landmarks) of quantity q at its point j with nyls_walk_put; nyls_walk_sum then returns in
// every lane the totals of chunk point lane & 15.  tile: LDS, Q * 16 * NYLS_WALK_PAD
// doubles, 16-byte aligned.
__device__ inline void nyls_walk_put(double* tile, int lane, int q, int j, double v) {
  tile[(q * 16 + 4 * j + (lane >> 4)) * NYLS_WALK_PAD + (lane & 15)] = v;
}

template <int Q>
__device__ inline void nyls_walk_sum(const double* tile, int lane, double (&out)[Q]) {
  nyls_wave_lds_sync();
  const int pt = lane & 15, qq = lane >> 4;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double* row = tile + (q * 16 + pt) * NYLS_WALK_PAD + 4 * qq;
    const double s = (row[0] + row[1]) + (row[2] + row[3]);
    out[q] = nyls_add_xor32(nyls_add_xor16(s));
  }
  nyls_wave_lds_sync();
}

// Tail layout: lane 4 pt + ts stores its tail pair's term of quantity q (ttile: LDS,
// Q * 64 doubles); nyls_walk_sum_tail adds the four tail slots of each point to the sums.
__device__ inline void nyls_walk_put_tail(double* ttile, int lane, int q, double v) {
  ttile[q * 64 + lane] = v;
}

template <int Q>
__device__ inline void nyls_walk_sum_tail(const double* tile, const double* ttile, int lane,
                                          double (&out)[Q]) {
  nyls_wave_lds_sync();
  const int pt = lane & 15, qq = lane >> 4;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double* row = tile + (q * 16 + pt) * NYLS_WALK_PAD + 4 * qq;
    const double s = ((row[0] + row[1]) + (row[2] + row[3])) + ttile[q * 64 + 4 * pt + qq];
    out[q] = nyls_add_xor32(nyls_add_xor16(s));
  }
  nyls_wave_lds_sync();
}

// Wide bases, G wavefronts per workgroup (wavefront grp walks landmark slots
// grp * 16 NB ..): every wavefront holds in tot[q] the totals of chunk point lane & 15 over its
// own slots; afterwards every lane holds the sums over all G wavefronts, added in wavefront
// order, so all wavefronts see bitwise the same values.  xw: LDS, 2 * G * Q * 16 doubles;
// `parity` alternates between consecutive calls, so one workgroup barrier per call suffices
// (a buffer is written again only after every wavefront has passed the next call's barrier,
// i.e. finished reading it).  Every wavefront of the workgroup must make the same calls.
template <int G, int Q>
__device__ inline void nyls_walk_join(double (&tot)[Q], double* xw, int lane, int grp, int parity) {
  double* buf = xw + parity * (G * Q * 16);
  if (lane < 16)
#pragma unroll
    for (int q = 0; q < Q; ++q) buf[(grp * Q + q) * 16 + lane] = tot[q];
  __syncthreads();
  const int pt = lane & 15;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double v = buf[q * 16 + pt];
#pragma unroll
    for (int g = 1; g < G; ++g) v += buf[(g * Q + q) * 16 + pt];
    tot[q] = v;
  }
}

// Per-point values w[q] held by lanes 0..15 (for chunk point lane) are returned in every lane
// for its own points: out[q][j] = w[q] of point 4 j + ph.  buf: LDS, Q * 16 doubles.
template <int Q>
__device__ inline void nyls_walk_bcast(const double (&w)[Q], double* buf, int lane,
                                       double (&out)[Q][4]) {
  if (lane < 16)
#pragma unroll
    for (int q = 0; q < Q; ++q) buf[q * 16 + (lane & 3) * 4 + (lane >> 2)] = w[q];
  nyls_wave_lds_sync();
  const int ph = lane >> 4;
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[q][j] = buf[q * 16 + ph * 4 + j];
  nyls_wave_lds_sync();
}

// The same, also returning in tout[q] the value of the lane's tail point (chunk point lane / 4).
template <int Q>
__device__ inline void nyls_walk_bcast_tail(const double (&w)[Q], double* buf, int lane,
                                            double (&out)[Q][4], double (&tout)[Q]) {
  if (lane < 16)
#pragma unroll
    for (int q = 0; q < Q; ++q) buf[q * 16 + (lane & 3) * 4 + (lane >> 2)] = w[q];
  nyls_wave_lds_sync();
  const int ph = lane >> 4, tp = lane >> 2;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int j = 0; j < 4; ++j) out[q][j] = buf[q * 16 + ph * 4 + j];
    tout[q] = buf[q * 16 + (tp & 3) * 4 + (tp >> 2)];
  }
  nyls_wave_lds_sync();
}

// Sum of v over the 16 lanes with the same tail slot (lane & 3); every lane gets its slot's sum.
__device__ inline double nyls_tail_fold(double v) {
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  return nyls_add_xor32(nyls_add_xor16(v));
}

// Sum of v over the four phases (lanes sl, sl + 16, sl + 32, sl + 48).
__device__ inline double nyls_walk_fold(double v) { return nyls_add_xor32(nyls_add_xor16(v)); }
