// Internal declarations shared by the nyls HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nyls.h"

#define NYLS_BLOCK 256

// Bases up to this size run the one-wavefront passes (up to eight 16-slot landmark blocks
// per lane) and keep K_mm and the KKT matrix on chip; wider ones (up to NYLS_MAX_M) are
// always split over point chunks, with two wavefronts per chunk, one per half of the
// landmark slots, and factor K_mm and the KKT matrix in the workspace.
#define NYLS_NARROW_MAX_M 128
// Widest Gram (m + 2) that the four-wave MFMA kernel forms in kernel space (eight column
// blocks of 16); wider unsplit ones take the LDS-tile kernel.
#define NYLS_GRAM4_MAX_G 128

// One instance as the kernels see it (device-resident table, one entry per instance).
struct nyls_desc {
  int32_t p, n, m, uniform;
  double t0, dt;
  const double* t;       // explicit grid (uniform == 0)
  const int32_t* lidx;   // [m] landmark grid indices (plan-owned device copy)
  const double* f;       // [p][n]
  const double* r;       // [n]
  const double* v;       // [p]
  int32_t cond_d[NYLS_MAX_P];
  int32_t cond_i[NYLS_MAX_P];
  int32_t rec;           // 1: uniform grid with dt <= sigma / 4: the strided Gaussian
                         // recurrence of the one-wave passes needs no exact exponentials
  int32_t flags;         // NYLS_DF_* launch choices of the plan's tuning for this instance
  double sigma, gamma, tau;
  int64_t ws;            // first double of this instance's workspace block
  int64_t goff;          // first grid point of this instance in per-point outputs
  int32_t chunk;         // NYLS_DF_SPLIT: grid points per workgroup (multiple of 64)
  int32_t nchunks;       // NYLS_DF_SPLIT: ceil(n / chunk)
  int64_t part;          // NYLS_DF_SPLIT: first double of the instance's partial sums
};

// Partial sums of split instances (offsets in doubles from nyls_desc::part): per chunk the
// (m+2)^2 Gram partial, then per chunk the pass partial (m landmark sums, sum c rho, max |y|,
// max change of y).
__host__ __device__ inline int64_t nyls_split_gram(int m, int c) { return (int64_t)c * (m + 2) * (m + 2); }
__host__ __device__ inline int64_t nyls_split_pass(int m, int nchunks, int c) {
  return (int64_t)nchunks * (m + 2) * (m + 2) + (int64_t)c * (m + 3);
}
__host__ __device__ inline int64_t nyls_split_doubles(int m, int nchunks) {
  return (int64_t)nchunks * ((m + 2) * (m + 2) + m + 3);
}

// nyls_desc::flags: which kernel variant takes the instance (set from the plan's tuning).
enum {
  NYLS_DF_TAIL = 1,       // one-wave passes walk a last block of <= 4 landmarks in the tail layout
  NYLS_DF_GRAM_TAIL = 2,  // one-wave MFMA Gram accumulates a last block of <= 4 columns on the VALU
  NYLS_DF_GRAM_VALU = 4,  // FP64 Gram on the LDS-tile VALU kernel even when m + 2 <= 64
  NYLS_DF_SPLIT = 8       // Gram and refinement/output passes split over point chunks, one
                          // workgroup per chunk (FP64 mode; never with NYLS_DF_TAIL)
};

// Per-instance workspace block (offsets in doubles from nyls_desc::ws).
struct nyls_wsl {
  int64_t W, lam, info, gram, lu, piv, x, alpha, acc, H, mu, beta, tmp, U, aux, log, end;
};

__host__ __device__ inline nyls_wsl nyls_layout(int m, int p, int n_newton) {
  // n_newton > 0 adds the Newton state (constant Jacobian block and scratch).
  nyls_wsl L;
  const int64_t g = m + 2, nk = m + 1 + p;
  L.W = 0;                       // m*m   W[s*m + k] = U[s][k] / sqrt(lam_k), k < r
  L.lam = L.W + (int64_t)m * m;  // m     eigenvalues, descending
  L.info = L.lam + m;            // 8     [0] rank r, [1] status bits, [2] sweeps,
                                 //       [3] last refinement correction, [4] Gram basis,
                                 //       [5] refinement passes over the grid
  L.gram = L.info + 8;           // g*g   kernel-space Gram of (p_i, c_i, r_i)
  L.lu = L.gram + g * g;         // nk*nk LU factors of the KKT system (row-major)
  L.piv = L.lu + nk * nk;        // nk    pivot rows
  L.x = L.piv + nk;              // nk    (omega, b, lambda)
  L.alpha = L.x + nk;            // m     alpha = W omega
  L.acc = L.alpha + m;           // 4g    accumulators of the per-point passes
  L.H = L.acc + 4 * g;           // p*m   condition rows h_j = W^T k^(d_j)(t_{i_j})
  L.mu = L.H + (int64_t)p * m;   // nk    adjoint solution
  L.beta = L.mu + nk;            // m     W mu_omega
  L.tmp = L.beta + m;            // g*g   scratch (S W products, eigenvectors when m is large)
  L.U = L.tmp + g * g;           // m*m   all eigenvectors (sorted, signed), U[s*m + k]
  L.log = L.U + (int64_t)m * m;  // plane-rotation log of the lane-parallel QL: 2 m^2 (c, s)
                                 // entries
  L.aux = L.log + 4 * (int64_t)m * m;  // Newton: constant block (m+2)^2 + weighted Gram (m+2)^2
                                       // + the system with small-pivot points kept (m+34)^2
  L.end = L.aux + (n_newton > 0 ? 2 * g * g + (g + 32) * (g + 32) : 0);
  L.end = (L.end + 7) & ~int64_t(7);
  return L;
}

// The value of this lane and that of lane l ^ 32 (l ^ 16), as (a, b) = the lower lane's
// value and the upper lane's: the gfx950 lane-swap instructions exchange halves of the
// wavefront in the VALU (no LDS round trip), and both lanes of a pair see the same (a, b).
__device__ inline void nyls_pair_xor32(double v, double& a, double& b) {
  const long long u = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

__device__ inline void nyls_pair_xor16(double v, double& a, double& b) {
  const long long u = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// Exchange through LDS among the lanes of one wavefront (for kernels that run one
// wavefront per workgroup).  The LDS operations of a wavefront execute in program
// order, so only compiler reordering has to be prevented; a workgroup barrier would also
// wait for the outstanding global loads of the next chunk.
__device__ inline void nyls_wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Landmark time t_s and grid time t_i.
__device__ inline double nyls_grid_t(const nyls_desc& d, int i) {
  return d.uniform ? __dadd_rn(d.t0, __dmul_rn((double)i, d.dt)) : d.t[i];
}

// The condition points of an instance held in (scalar) registers for the per-point passes,
// which skip them in the residual set: read once instead of at every point.
struct nyls_cpts {
  int c[NYLS_MAX_P];
  __device__ void init(const nyls_desc& d) {
#pragma unroll
    for (int j = 0; j < NYLS_MAX_P; ++j)
      c[j] = __builtin_amdgcn_readfirstlane(j < d.p ? d.cond_i[j] : -1);
  }
  __device__ bool has(int i) const {
    bool r = false;
#pragma unroll
    for (int j = 0; j < NYLS_MAX_P; ++j) r |= (c[j] == i);
    return r;
  }
  // some condition point lies in [lo, hi) (wave-uniform for uniform lo, hi)
  __device__ bool any_in(int lo, int hi) const {
    bool r = false;
#pragma unroll
    for (int j = 0; j < NYLS_MAX_P; ++j) r |= (c[j] >= lo && c[j] < hi);
    return r;
  }
};

__device__ inline bool nyls_is_condition_point(const nyls_desc& d, int i) {
  bool c = false;
  for (int j = 0; j < d.p; ++j) c |= (d.cond_i[j] == i);
  return c;
}

// Kernel derivative values of K(t, t_s) in the first argument, all orders 0..NYLS_MAX_P:
// d^q/dt^q K = (-1/sigma)^q H_q(z) exp(-z^2), z = (t - t_s) / sigma, with the physicists'
// Hermite recurrence H_0 = 1, H_1 = 2z, H_{q+1} = 2z H_q - 2q H_{q-1}.  Every index is
// static so the values stay in registers.
__device__ inline void nyls_kderiv(double z, double inv_sigma, double (&kd)[NYLS_MAX_P + 1]) {
  const double e = exp(-z * z);
  double hm = 1.0, h = 2.0 * z, sc = -inv_sigma;
  kd[0] = e;
  kd[1] = sc * h * e;
#pragma unroll
  for (int q = 1; q < NYLS_MAX_P; ++q) {
    const double hn = 2.0 * z * h - 2.0 * q * hm;
    hm = h;
    h = hn;
    sc *= -inv_sigma;
    kd[q + 1] = sc * h * e;
  }
}

// Static selection kd[q] for a run-time q in 0..NYLS_MAX_P.
template <typename T>
__device__ inline T nyls_pick(const T (&kd)[NYLS_MAX_P + 1], int q) {
  T v = kd[0];
#pragma unroll
  for (int k = 1; k <= NYLS_MAX_P; ++k) v = (q == k) ? kd[k] : v;
  return v;
}

// Operator weights of L = d^p - sum_k f_k d^(p-k) on the derivative orders q = 0..NYLS_MAX_P:
// w[p] = 1, w[p-k] = -f_k (k = 1..p), 0 above p.  fk(k) returns f_k at the point.
template <typename T, typename F>
__device__ inline void nyls_opweights(int p, F fk, T (&w)[NYLS_MAX_P + 1]) {
#pragma unroll
  for (int q = 0; q <= NYLS_MAX_P; ++q) w[q] = (q == p) ? T(1) : (q < p ? -T(fk(p - q)) : T(0));
}

template <typename T>
__device__ inline T nyls_dot5(const T (&a)[NYLS_MAX_P + 1], const T (&b)[NYLS_MAX_P + 1]) {
  T v = T(0);
#pragma unroll
  for (int q = 0; q <= NYLS_MAX_P; ++q) v += a[q] * b[q];
  return v;
}

// Raw buffer resource over `bytes` bytes at p (gfx9 raw-buffer word 3): loads outside
// [0, bytes) return 0 through the hardware range check, so tail chunks need no clamping.
__device__ inline __amdgpu_buffer_rsrc_t nyls_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

__device__ inline double nyls_bload(__amdgpu_buffer_rsrc_t r, int off_bytes) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off_bytes, 0, 0));
}

// Start of a run of `len` uniform-grid points k0, k0 + stride, ... (offsets from a landmark,
// a = dt / sigma) for the Gaussian recurrence.  With Q = exp(-2 a^2 stride^2) and
// R(k) = exp(-a^2 stride (2 k + stride)) the exact identities are
//     e(k + stride) = e(k) R(k),   R(k + stride) = R(k) Q.
// The walk carries rho = R - 1 instead of R (from expm1), and steps with
//     e <- fma(e, rho, e),   rho <- fma(rho, Q, Q - 1)   (Q - 1 also from expm1):
// where the values matter |rho| is small, so the roundings of rho (and of Q) perturb R by
// about |rho| eps rather than eps.  Carrying R itself lets a rounding of R tilt the relative
// error of all later values of the run by the same amount, a smooth error that the
// ill-conditioned solves amplify much more than independent per-value roundings.
// Returns true when the run must use exact exponentials instead: the ratio would overflow,
// or the run starts below exp(-700) (denormal or zero, so the relative precision is gone)
// while approaching the landmark and rising above that level inside the run.  Runs that
// stay below exp(-700) keep the recurrence: their values are negligible in absolute terms.
__device__ inline bool nyls_gauss_start(int k0, int len, int stride, double a, double& ev,
                                        double& rho) {
  const double z0 = (double)k0 * a;
  const double rexp = -a * a * (double)stride * (2.0 * k0 + stride);
  if (rexp > 700.0) return true;
  const int ke = k0 + (len - 1) * stride;
  if (k0 < 0 && z0 * z0 > 700.0) {
    const double ze = (double)ke * a;
    if (ke >= 0 || ze * ze < 700.0) return true;
  }
  ev = exp(-z0 * z0);
  rho = expm1(rexp);
  return false;
}

// One step of the recurrence above: e(k + stride) and rho(k + stride) from e(k), rho(k).
__device__ inline void nyls_gauss_step(double& ev, double& rho, double q, double qm1) {
  ev = fma(ev, rho, ev);
  rho = fma(rho, q, qm1);
}

// Gaussian values over a tile of TP consecutive grid points i = i0 + pt and all landmarks:
// calls emit(pt, s, z, e) with z = (t_i - t_s)/sigma and e = exp(-z^2) (e = 0 for i >= n).
// Work is split as thread -> (landmark s, chunk of CH points).  On a uniform grid
// t_i - t_s = (i - i_s) dt, so along a chunk, with a = dt/sigma and k = i - i_s,
//     e(k+1) = e(k) R(k),  R(k) = exp(-a^2 (2k+1)),  R(k+1) = R(k) exp(-2 a^2),
// stepped as in nyls_gauss_start (two multiply-adds per value after two exponentials per
// chunk).  Chunks that nyls_gauss_start rejects use one exponential per point instead.
template <int TP, int CH, typename Emit>
__device__ inline void nyls_gauss_tile(const nyls_desc& d, int i0, const double* tl,
                                       double inv_sigma, Emit emit) {
  constexpr int NC = TP / CH;
  const int m = d.m, n = d.n;
  const double a = d.dt * inv_sigma;
  const double q2 = exp(-2.0 * a * a), q2m1 = expm1(-2.0 * a * a);
  for (int e = threadIdx.x; e < m * NC; e += NYLS_BLOCK) {
    const int s = e % m, c = e / m;
    const int ib = i0 + c * CH;
    if (d.uniform) {
      const int k0 = ib - d.lidx[s];
      double ev = 0.0, rho = 0.0;
      if (!nyls_gauss_start(k0, CH, 1, a, ev, rho)) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          emit(c * CH + j, s, (double)(k0 + j) * a, (ib + j < n) ? ev : 0.0);
          nyls_gauss_step(ev, rho, q2, q2m1);
        }
      } else {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const double z = (double)(k0 + j) * a;
          emit(c * CH + j, s, z, (ib + j < n) ? exp(-z * z) : 0.0);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int i = ib + j;
        const double z = i < n ? (d.t[i] - tl[s]) * inv_sigma : 0.0;
        emit(c * CH + j, s, z, i < n ? exp(-z * z) : 0.0);
      }
    }
  }
}

// Derivative values from z and e = exp(-z^2): kd[q] = (-1/sigma)^q H_q(z) e, q = 0..NYLS_MAX_P.
__device__ inline void nyls_kderiv_e(double z, double e, double inv_sigma,
                                     double (&kd)[NYLS_MAX_P + 1]) {
  double hm = 1.0, h = 2.0 * z, sc = -inv_sigma;
  kd[0] = e;
  kd[1] = sc * h * e;
#pragma unroll
  for (int q = 1; q < NYLS_MAX_P; ++q) {
    const double hn = 2.0 * z * h - 2.0 * q * hm;
    hm = h;
    h = hn;
    sc *= -inv_sigma;
    kd[q + 1] = sc * h * e;
  }
}

// Block-wide helpers (blockDim.x == NYLS_BLOCK).
__device__ inline double nyls_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NYLS_BLOCK / 64; ++i) s += red[i];
  return s;
}

// Optional per-kernel timing with HIP events (off unless nyls_profile_enable(1)).
void nyls_prof_begin(int kernel, hipStream_t st);
void nyls_prof_end(int kernel, hipStream_t st);
enum { NYLS_K_EIG = 0, NYLS_K_GRAM64, NYLS_K_GRAM32, NYLS_K_KKT, NYLS_K_POINTS, NYLS_K_FEATURES,
       NYLS_K_PREDICT, NYLS_K_EXPLICIT, NYLS_K_NEWTON, NYLS_K_BACKWARD, NYLS_K_COUNT };

// 16-landmark slot blocks per lane of the one-wave passes for an instance with m landmarks
// (16 for the wide bases: eight per lane in each of two wavefronts).
__host__ __device__ inline int nyls_slot_blocks(int m) {
  return m <= 32 ? 2 : (m <= 64 ? 4 : (m <= NYLS_NARROW_MAX_M ? 8 : 16));
}

// Column blocks of the kernel-space MFMA Gram (m + 2 <= 64): nbu = ceil((m + 2) / 16) blocks
// carry data, and the last of them goes to the VALU when it holds at most four columns;
// encoded as 2 nbu + (1 if so).
__host__ __device__ inline int nyls_gram_class(int m) {
  const int g = m + 2, nbu = (g + 15) >> 4;
  return 2 * nbu + ((nbu > 1 && g - 16 * (nbu - 1) <= 4) ? 1 : 0);
}

// Column-block class of the kernel-space MFMA Gram that takes instance d (its descriptor's
// NYLS_DF_GRAM_TAIL flag says whether the last block goes to the VALU).
__host__ __device__ inline int nyls_gram_class_of(const nyls_desc& d) {
  return 2 * ((d.m + 2 + 15) >> 4) + ((d.flags & NYLS_DF_GRAM_TAIL) ? 1 : 0);
}

// Landmarks in the last 16-slot block when there are at most four of them (m = 16 (NB - 1)
// + 1 .. 4, NB = nyls_slot_blocks(m) > 1), else 0.  On instances with rec == 1 the one-wave
// passes walk such a block in a tail layout (one (point, landmark) pair per lane and chunk)
// instead of pair by pair, where it would cost a quarter of the work for a few landmarks.
__host__ __device__ inline int nyls_walk_tail(int m) {
  const int nb = nyls_slot_blocks(m), t = m - 16 * (nb - 1);
  return (nb > 1 && t >= 1 && t <= 4) ? t : 0;
}

// Host launchers (defined in the .hip files; all enqueue on `stream`).
struct nyls_plan_view {
  int32_t batch, mode, maxm, maxp, maxn;
  int32_t maxm_narrow;      // largest m <= NYLS_NARROW_MAX_M (0 if none): sizes on-chip buffers
  unsigned p_mask;          // bit p set when some instance has ODE order p
  unsigned rec_mask;        // bit 1: some instance has rec == 1, bit 0: some has rec == 0
  unsigned nb_mask;         // bit b set when some instance has nyls_slot_blocks(m) == b
  unsigned gnb_mask;        // bit b set when some instance has nyls_slot_blocks(m + 2) == b
  int32_t only;             // nonzero: the Gram / KKT / refinement kernels process only the
                            // instances whose status (info[1]) has one of these bits, with
                            // the FP64 Gram in the eigenbasis (re-solve of a failed FP32 Gram)
  const nyls_desc* d_desc;
  const int32_t* d_order;   // instance order, most expensive first
  int64_t total;
  unsigned nt_mask;         // bit t set when some instance has ceil((m+2)/16) == t
  unsigned gcls_mask;       // bit nyls_gram_class(m) for the instances with m + 2 <= 64
  unsigned tl_mask;         // bit b: some rec == 1 instance of slot class b walks a tail layout
  unsigned ntl_mask;        // bit b: some instance of slot class b does not
  int32_t n_big;            // instances with m > 64
  int32_t n_split;          // instances with NYLS_DF_SPLIT
  int32_t n_vgram;          // unsplit instances whose FP64 Gram takes the LDS-tile kernel
                            // (m + 2 > 64, or NYLS_DF_GRAM_VALU)
  int32_t n_vks;            // ... and whose kernel-space Gram it forms as well
                            // (m + 2 > NYLS_GRAM4_MAX_G, or NYLS_DF_GRAM_VALU)
  int32_t max_chunks;       // largest nchunks of a split instance
  int32_t eig_ql;           // tuning: 1 QL inside one wavefront per instance
  int32_t ql_lanes;         // tuning: instances per wavefront of the lane-parallel QL
  int32_t overlap;          // tuning: FP64 kernel-space Gram beside the eigensolver
};

// `single` >= 0 restricts a launch to that one instance (one workgroup).  `parts` selects
// the instances by basis size: NYLS_EIG_NARROW (m <= 64), NYLS_EIG_BIG (m > 64); the two
// touch disjoint instances, so they may run on different streams.
#define NYLS_EIG_NARROW 1
#define NYLS_EIG_BIG 2
hipError_t nyls_launch_eig(const nyls_plan_view& pv, double* ws, int single, hipStream_t st,
                           int parts = NYLS_EIG_NARROW | NYLS_EIG_BIG);
hipError_t nyls_launch_gram64(const nyls_plan_view& pv, double* ws, hipStream_t st);
// The FP64 Grams of the unsplit bases with m + 2 > 64 only (NYLS_MIXED: the FP32 Gram takes
// the others): kernel space on the matrix cores, the eigenbasis where K_mm is
// ill-conditioned.
hipError_t nyls_launch_gram64_over64(const nyls_plan_view& pv, double* ws, hipStream_t st);
// The two halves of nyls_launch_gram64 for a solve that overlaps the Gram with the
// eigensolver: the kernel-space Grams of every instance (they read nothing the eigensolver
// writes), then, once the eigensolver is done (ks_done = true), the eigenbasis Grams that
// replace them where K_mm is ill-conditioned.
hipError_t nyls_launch_gram64_kspace(const nyls_plan_view& pv, double* ws, hipStream_t st);
hipError_t nyls_launch_gram64_rest(const nyls_plan_view& pv, double* ws, hipStream_t st, bool ks_done);
hipError_t nyls_launch_gram32(const nyls_plan_view& pv, double* ws, hipStream_t st);
hipError_t nyls_launch_kkt(const nyls_plan_view& pv, double* ws, double* kkt_out, double* rhs_out,
                           int factor, hipStream_t st);
// `classes`: the slot classes to launch (bits of nyls_plan_view::nb_mask: 4, 16, 256; the
// split instances go with bit 1); classes touch disjoint instances, so they may run on
// different streams.
hipError_t nyls_launch_points(const nyls_plan_view& pv, double* ws, int refine, double* yhat,
                              double* omega, double* bias, double* lambda, int32_t* status,
                              int single, hipStream_t st, unsigned classes = ~0u);
hipError_t nyls_launch_features(const nyls_plan_view& pv, const double* ws, const double* t_eval,
                                const int64_t* eval_off, int dmax, double* phi, double* eigval,
                                int32_t* rank, int64_t max_eval, int single, hipStream_t st);
hipError_t nyls_launch_predict(const nyls_plan_view& pv, const double* ws, const double* t_eval,
                               const int64_t* eval_off, int d, double* out, int64_t max_eval,
                               hipStream_t st);
hipError_t nyls_launch_explicit_rows(const nyls_plan_view& pv, int inst, const double* ws,
                                     const double* phi, double* rows, int n, int m,
                                     hipStream_t st);
hipError_t nyls_launch_explicit_kkt(const nyls_plan_view& pv, int inst, double* ws,
                                    const double* phi, const double* C, hipStream_t st);
