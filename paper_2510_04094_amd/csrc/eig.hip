// Nystrom basis: landmark kernel matrix K_mm, its eigendecomposition and the feature
// transform W = U_r Lambda_r^{-1/2} (App. A.2, eq32), one workgroup per instance.
//
// K_mm is at most 128 x 128, so each workgroup keeps it in LDS and diagonalises it with
// the two-sided cyclic Jacobi method in parallel (round-robin) order: every round rotates
// m/2 disjoint index pairs at once, each thread updating whole 2 x 2 blocks J_i^T A J_j.
// Eigenvectors accumulate in LDS when both matrices fit (m <= 96), else in the instance's
// global scratch block.  Afterwards eigenvalues are sorted descending, each eigenvector is
// signed so its largest-magnitude entry (first on ties) is positive, and eigenpairs with
// lambda_k <= tau * lambda_1 are dropped (the retained rank r goes to info[0]).
#include "nyls_dense.h"

namespace {

constexpr int kMaxSweeps = 40;
constexpr int kQlMaxM = 64;       // bases up to this size use k_eig_ql
constexpr int kVldsMaxM = 96;

__device__ inline int instance_of(const int32_t* order, int single) {
  return single >= 0 ? single : (order ? order[blockIdx.x] : (int)blockIdx.x);
}

template <bool VLDS>
__global__ __launch_bounds__(NYLS_BLOCK) void k_eig(const nyls_desc* __restrict__ desc,
                                                    const int32_t* __restrict__ order,
                                                    double* __restrict__ wsbase, int single) {
  extern __shared__ double sm[];
  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  const int m = d.m;
  if (m <= kQlMaxM) return;  // k_eig_ql handles it
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;
  const int ld = m + 1;
  const int npair = (m + 1) >> 1;
  const int m2 = npair << 1;

  double* A = sm;
  double* V = VLDS ? (A + m * ld) : (ws + L.tmp);
  const int vld = VLDS ? ld : m;
  double* tail = VLDS ? (A + 2 * m * ld) : (A + m * ld);
  double* cs = tail;              // [64] cosines of this round
  double* sn = cs + 64;           // [64] sines
  double* tn = sn + 64;           // [64] tangents
  double* red = tn + 64;          // [8]  reductions
  double* tl = red + 8;           // [m]  landmark times, later eigenvalues
  int* pidx = reinterpret_cast<int*>(tl + NYLS_MAX_M);
  int* qidx = pidx + 64;
  int* pos = qidx + 64;           // [m] sorted position of eigenpair k
  double* sgn = reinterpret_cast<double*>(pos + NYLS_MAX_M);  // [m]

  const double inv_sigma = 1.0 / d.sigma;
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  __syncthreads();
  for (int e = tid; e < m * m; e += NYLS_BLOCK) {
    const int a = e / m, b = e - a * m;
    const double z = (tl[a] - tl[b]) * inv_sigma;
    A[a * ld + b] = exp(-z * z);
    V[a * vld + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();

  // Cyclic sweeps until a whole sweep finds no off-diagonal entry above 1e-17 ||diag||_2
  // (the backward-error level of a dense FP64 eigensolver).
  int* rotflag = pos;  // reused below for the sort
  int sweep = 0;
  bool converged = false;
  for (; sweep < kMaxSweeps; ++sweep) {
    double dia = 0.0;
    for (int k = tid; k < m; k += NYLS_BLOCK) dia += A[k * ld + k] * A[k * ld + k];
    const double thresh = 1e-17 * sqrt(nyls_block_sum(dia, red));
    if (tid == 0) rotflag[0] = 0;
    __syncthreads();

    for (int rd = 0; rd < m2 - 1; ++rd) {
      if (tid < npair) {
        int a, b;
        if (tid == 0) { a = rd; b = m2 - 1; }
        else { a = (rd + tid) % (m2 - 1); b = (rd - tid + (m2 - 1)) % (m2 - 1); }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < m) {
          const double apq = A[p * ld + q];
          if (fabs(apq) > thresh) {
            const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            rotflag[0] = 1;
          }
        }
        pidx[tid] = p; qidx[tid] = q; cs[tid] = c; sn[tid] = s; tn[tid] = t;
      }
      __syncthreads();
      // A <- J^T A J on every 2 x 2 block (pair i rows, pair j columns).
      for (int e = tid; e < npair * npair; e += NYLS_BLOCK) {
        const int i = e / npair, j = e - i * npair;
        const int p1 = pidx[i], q1 = qidx[i], p2 = pidx[j], q2 = qidx[j];
        const bool r1 = q1 < m, r2 = q2 < m;
        const double c1 = cs[i], s1 = sn[i], c2 = cs[j], s2 = sn[j];
        const double app = A[p1 * ld + p2];
        const double apq = r2 ? A[p1 * ld + q2] : 0.0;
        const double aqp = r1 ? A[q1 * ld + p2] : 0.0;
        const double aqq = (r1 && r2) ? A[q1 * ld + q2] : 0.0;
        const double bpp = c1 * app - s1 * aqp, bpq = c1 * apq - s1 * aqq;
        const double bqp = s1 * app + c1 * aqp, bqq = s1 * apq + c1 * aqq;
        double npp = c2 * bpp - s2 * bpq, npq = s2 * bpp + c2 * bpq;
        double nqp = c2 * bqp - s2 * bqq, nqq = s2 * bqp + c2 * bqq;
        if (i == j && r1) {
          // the rotated pair is annihilated; diagonal in the accurate form a -+ t a_pq
          const double t = tn[i];
          npp = app - t * apq;
          nqq = aqq + t * apq;
          npq = 0.0;
          nqp = 0.0;
        }
        A[p1 * ld + p2] = npp;
        if (r2) A[p1 * ld + q2] = npq;
        if (r1) A[q1 * ld + p2] = nqp;
        if (r1 && r2) A[q1 * ld + q2] = nqq;
      }
      // V <- V J
      for (int e = tid; e < m * npair; e += NYLS_BLOCK) {
        const int row = e / npair, j = e - row * npair;
        const int p2 = pidx[j], q2 = qidx[j];
        if (q2 < m) {
          const double c2 = cs[j], s2 = sn[j];
          const double vp = V[row * vld + p2], vq = V[row * vld + q2];
          V[row * vld + p2] = c2 * vp - s2 * vq;
          V[row * vld + q2] = s2 * vp + c2 * vq;
        }
      }
      __syncthreads();
    }
    if (rotflag[0] == 0) { converged = true; break; }
    __syncthreads();
  }

  // Sort eigenvalues descending (ties by index) and pick each eigenvector's sign.
  for (int k = tid; k < m; k += NYLS_BLOCK) {
    const double lk = A[k * ld + k];
    int ps = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = A[j * ld + j];
      ps += (lj > lk) || (lj == lk && j < k);
    }
    pos[k] = ps;
    int jmax = 0;
    double vmax = -1.0;
    for (int s = 0; s < m; ++s) {
      const double a = fabs(V[s * vld + k]);
      if (a > vmax) { vmax = a; jmax = s; }
    }
    sgn[k] = V[jmax * vld + k] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int k = tid; k < m; k += NYLS_BLOCK) tl[pos[k]] = A[k * ld + k];
  __syncthreads();
  const double lam1 = tl[0];
  int rank = 0;
  for (int k = 0; k < m; ++k) rank += (tl[k] > d.tau * lam1) ? 1 : 0;
  // W[s][pos] = sign * U[s][k] / sqrt(lam_k) for retained positions, 0 otherwise.
  // With V in global scratch (ws + tmp) the output region ws + W does not alias it.
  for (int e = tid; e < m * m; e += NYLS_BLOCK) {
    const int s = e / m, k = e - s * m;
    const int ps = pos[k];
    const double lk = A[k * ld + k];
    ws[L.W + s * m + ps] = (ps < rank) ? sgn[k] * V[s * vld + k] / sqrt(lk) : 0.0;
    ws[L.U + s * m + ps] = sgn[k] * V[s * vld + k];
  }
  for (int k = tid; k < m; k += NYLS_BLOCK) ws[L.lam + k] = tl[k];
  if (tid == 0) {
    int bits = 0;
    if (rank < m) bits |= NYLS_S_TRUNCATED;
    if (!converged) bits |= NYLS_S_EIG_NOCONV;
    if (!(lam1 == lam1) || rank == 0) bits |= NYLS_S_NONFINITE;
    ws[L.info + 0] = (double)rank;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 2] = (double)sweep;
  }
}

// ---- one wavefront per instance, m <= 64: Householder tridiagonalisation + implicit QL ----
//
// Lane i owns row i of the landmark matrix A in LDS (odd row stride: row-per-lane accesses
// are conflict-free, a row read by all lanes at once is a broadcast) and the entries d_i, e_i
// of the tridiagonal matrix in registers.
//  1. For k = 0 .. m-3 the reflector H_k = I - beta v v^T maps A[k+1:, k] onto alpha e_1;
//     the trailing block becomes B - v w^T - w v^T with p = beta B v,
//     w = p - (beta/2)(v^T p) v.  v is kept in column k below the diagonal.
//  2. Q = H_0 ... H_{m-3} is formed in place, last reflector first: each step applies H_k
//     to the trailing block from the left and sets row and column k to e_k.
//  3. Implicit QL on (d, e) with the shift from the leading 2 x 2 block of the active part;
//     each sweep chases the bulge from the bottom of the unreduced block upwards with plane
//     rotations, applied to the columns of Z = Q as they are formed (the column shared by
//     consecutive rotations stays in a register).  The split test |e_i| <= eps (|d_i| +
//     |d_{i+1}|) is evaluated by all lanes at once; the scalar recurrences read d and e with
//     lane broadcasts and are evaluated by every lane (they are uniform).
constexpr int kQlMaxIter = 60;  // QL sweeps per eigenvalue
// Instances per wavefront of k_ql_lanes: at most 64; the plan's tuning picks the number
// (default 64: 32, 16 and 8 all measured slower on batches of thousands of m = 50 instances,
// fewer spread a small batch over more CUs).
constexpr int kQlLaneInst = 64;

__device__ inline double sel_lane(double x, int lane, int i, double v) { return lane == i ? v : x; }

// 1/sqrt(x) for normal or subnormal x > 0: the hardware estimate followed by two Newton
// steps y <- y (3 - x y^2) / 2 (each one roughly squares the relative error), so that the
// rotation c = g y, s = f y (x = f^2 + g^2) has c^2 + s^2 = 1 to a few ulp.  The dependency
// chain is far shorter than that of a square root followed by a division.
__device__ inline double nyls_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double h = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, h, y);
  }
  return y;
}

// stage: QL_FULL all steps in one wave; QL_REDUCE steps 1-2, writing d, e and Q to the
// workspace for k_ql_lanes; QL_REPLAY applies the rotations k_ql_lanes logged to Q, then
// step 4; QL_REDO = QL_FULL for the instances whose rotation log overflowed.
enum { QL_FULL = 0, QL_REDUCE = 1, QL_REPLAY = 3, QL_REDO = 4 };

__global__ __launch_bounds__(64) void k_eig_ql(const nyls_desc* __restrict__ desc,
                                               const int32_t* __restrict__ order,
                                               double* __restrict__ wsbase, int single, int lda,
                                               int stage) {
  extern __shared__ double sm[];
  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  const int m = d.m;
  if (m > kQlMaxM) return;  // k_eig handles larger bases
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  if (stage == QL_REDO && ws[L.info + 7] != 2.0) return;
  const int lane = threadIdx.x;
  double* A = sm;                   // [lda][lda] (lda >= m): K_mm, then Q, then Z
  double* vv = A + lda * lda;       // [64] reflector, broadcast copy
  double* tt = vv + 64;             // [64] column sums / sign / sorted eigenvalues
  double* tl = tt + 64;             // [64] landmark times
  double* ww = tl;                  // [64] Householder w, broadcast copy (after tl's last use)
  int* pos = reinterpret_cast<int*>(tl + 64);  // [64] sorted position
  const bool own = lane < m;
  double* Ar = A + lane * lda;

  double dl = 0.0, el = 0.0, bl = 0.0;  // d_lane, e_lane, beta_lane
  const double eps = 2.220446049250313e-16;
  int iters = 0;
  bool converged = true;
  if (stage == QL_REPLAY) {
    if (ws[L.info + 7] == 2.0) return;  // log overflow: QL_REDO recomputes this instance
    // Q and the eigenvalues from the workspace, then the logged sweeps: each is a header
    // (mm, number of rotations k) and k pairs (c, s) for columns i = mm - 1, mm - 2, ...
    if (own)
      for (int j = 0; j < m; ++j) Ar[j] = ws[L.U + lane * m + j];
    dl = own ? ws[L.lam + lane] : 0.0;
    // lanes past m read row m - 1, so every read stays inside A
    const double* Ac = A + (own ? lane : m - 1) * lda;
    iters = (int)ws[L.info + 2];
    converged = ws[L.info + 7] == 0.0;
    // Lanes past m write their (unused) results to the vv/tt/tl area, one column apart so the
    // stores do not collide; step 4 rewrites that area before reading it.  No lane mask is
    // needed in the rotation loop.
    double* Aw = own ? Ar : vv + (lane - m);
    // Each sweep's log window (its header and at most m - 1 <= 63 rotations) is one entry
    // per lane; rotation k is read from lane k + 1 with lane broadcasts.  The next sweep's
    // window is loaded while this one is applied.
    const double* lg = ws + L.log;
    const int nsw = (int)ws[L.info + 6];
    const int cap = (int)((L.aux - L.log) / 2);
    auto fetch = [&](int e0, double& a, double& b) {
      const int e = e0 + lane;
      a = e < cap ? lg[2 * e] : 0.0;
      b = e < cap ? lg[2 * e + 1] : 0.0;
    };
    double ca, cb;
    fetch(0, ca, cb);
    int hdr = 0;
    for (int sw = 0; sw < nsw; ++sw) {
      const int mm = (int)nyls_rdlane(ca, 0), nrot = (int)nyls_rdlane(cb, 0);
      const int nxt = hdr + 1 + nrot;
      double na, nb;
      fetch(nxt, na, nb);
      double carry = Ac[mm];
      int k = 0;
      // groups of four rotations: the four Z entries they read are loaded together
      for (; k + 4 <= nrot; k += 4) {
        const int i = mm - 1 - k;  // i - 3 >= mm - nrot >= 0
        double z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = Ac[i - u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double cs = nyls_rdlane(ca, k + u + 1), sn = nyls_rdlane(cb, k + u + 1);
          Aw[i - u + 1] = sn * z[u] + cs * carry;
          carry = cs * z[u] - sn * carry;
        }
      }
      for (; k < nrot; ++k) {
        const int i = mm - 1 - k;
        const double cs = nyls_rdlane(ca, k + 1), sn = nyls_rdlane(cb, k + 1);
        const double z0 = Ac[i];
        Aw[i + 1] = sn * z0 + cs * carry;
        carry = cs * z0 - sn * carry;
      }
      Aw[mm - nrot] = carry;
      ca = na;
      cb = nb;
      hdr = nxt;
    }
    nyls_wave_lds_sync();
  } else {
  const double inv_sigma = 1.0 / d.sigma;
  if (own) tl[lane] = nyls_grid_t(d, d.lidx[lane]);
  nyls_wave_lds_sync();
  if (own) {
    const double ti = tl[lane];
    for (int j = 0; j < m; ++j) {
      const double z = (ti - tl[j]) * inv_sigma;
      Ar[j] = exp(-z * z);
    }
  }
  nyls_wave_lds_sync();

  // 1. tridiagonalisation
  for (int k = 0; k + 2 < m; ++k) {
    const bool act = own && lane > k;
    const double x = act ? Ar[k] : 0.0;
    const double sig2 = nyls_wave_sum_dpp(x * x);
    const double x1 = nyls_rdlane(x, k + 1);
    dl = sel_lane(dl, lane, k, A[k * lda + k]);
    if (!(sig2 - x1 * x1 > 0.0)) {  // already tridiagonal in this column: H_k = I
      el = sel_lane(el, lane, k, x1);
      if (act) Ar[k] = 0.0;
      nyls_wave_lds_sync();
      continue;
    }
    const double alpha = x1 >= 0.0 ? -sqrt(sig2) : sqrt(sig2);
    const double beta = 1.0 / (sig2 - alpha * x1);  // 2 / v^T v
    const double v = act ? (lane == k + 1 ? x - alpha : x) : 0.0;
    el = sel_lane(el, lane, k, alpha);
    bl = sel_lane(bl, lane, k, beta);
    vv[lane] = v;
    if (act) Ar[k] = v;
    nyls_wave_lds_sync();
    double pl = 0.0;
    if (act) pl = nyls_row_dot(Ar, vv, k + 1, m);
    pl *= beta;
    const double K = 0.5 * beta * nyls_wave_sum_dpp(v * pl);
    const double w = pl - K * v;
    ww[lane] = w;
    nyls_wave_lds_sync();
    if (act) nyls_row_rank2(Ar, v, ww, w, vv, k + 1, m);
    nyls_wave_lds_sync();
  }
  {
    const double a22 = A[(m - 2) * lda + m - 2], a32 = A[(m - 1) * lda + m - 2],
                 a33 = A[(m - 1) * lda + m - 1];
    dl = sel_lane(dl, lane, m - 2, a22);
    el = sel_lane(el, lane, m - 2, a32);
    dl = sel_lane(dl, lane, m - 1, a33);
    el = sel_lane(el, lane, m - 1, 0.0);
  }
  nyls_wave_lds_sync();

  // 2. Q in place: the trailing 2 x 2 block starts as the identity
  if (own && lane >= m - 2) {
    Ar[m - 2] = lane == m - 2 ? 1.0 : 0.0;
    Ar[m - 1] = lane == m - 1 ? 1.0 : 0.0;
  }
  nyls_wave_lds_sync();
  for (int k = m - 3; k >= 0; --k) {
    const bool act = own && lane > k;
    const double v = act ? Ar[k] : 0.0;
    const double beta = nyls_rdlane(bl, k);
    if (beta != 0.0) {
      vv[lane] = v;
      nyls_wave_lds_sync();
      // t_j = sum_i v_i Q[i][j] (lane j owns column j)
      const double t = act ? nyls_col_dot(vv, A + lane, lda, k + 1, m) : 0.0;
      tt[lane] = beta * t;
      nyls_wave_lds_sync();
      if (act) nyls_row_rank1(Ar, v, tt, k + 1, m);
    }
    // row and column k of Q: e_k
    if (lane == k)
      for (int j = k; j < m; ++j) Ar[j] = j == k ? 1.0 : 0.0;
    if (act) Ar[k] = 0.0;
    nyls_wave_lds_sync();
  }

  if (stage == QL_REDUCE) {
    // d, e and Q for k_ql_lanes and the replay (W and U are written at the end)
    if (own) {
      ws[L.lam + lane] = dl;
      ws[L.W + lane] = el;
      for (int j = 0; j < m; ++j) ws[L.U + lane * m + j] = Ar[j];
    }
    return;
  }

  // 3. implicit QL on (d, e), rotations accumulated into Z (rows in A)
  for (int l = 0; l < m; ++l) {
    int it = 0;
    for (;;) {
      const double dn = __shfl_down(dl, 1);
      const bool small = lane == m - 1 ||
                         (lane >= l && lane < m - 1 && fabs(el) <= eps * (fabs(dl) + fabs(dn)));
      const unsigned long long mask = __ballot(small && lane >= l);
      const int mm = __ffsll((long long)mask) - 1;
      if (mm == l) break;
      if (++it > kQlMaxIter) { converged = false; break; }
      ++iters;
      const double dL = nyls_rdlane(dl, l), eL = nyls_rdlane(el, l);
      double g = (nyls_rdlane(dl, l + 1) - dL) / (2.0 * eL);
      double r = sqrt(g * g + 1.0);
      g = nyls_rdlane(dl, mm) - dL + eL / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, pp = 0.0;
      double carry = own ? Ar[mm] : 0.0;
      // Rotation i reads d_i, d_{i+1} and e_i, which no earlier rotation of this sweep has
      // rewritten (rotation i rewrites d_{i+1} and e_{i+1}): read them from copies taken
      // before the sweep, off the dependency chain of g, sn, cs.  The lane's Z entry of
      // column i is loaded one rotation ahead, so the LDS latency overlaps the chain.
      const double d0 = dl, e0 = el;
      double z0 = own ? Ar[mm - 1] : 0.0;
      bool split = false;
      for (int i = mm - 1; i >= l; --i) {
        const double ei = nyls_rdlane(e0, i);
        const double di = nyls_rdlane(d0, i), di1 = nyls_rdlane(d0, i + 1);
        const double f = sn * ei, b = cs * ei;
        const double x = f * f + g * g;
        if (x == 0.0) {  // exact deflation: the chase stops here
          el = sel_lane(el, lane, i + 1, 0.0);
          dl = sel_lane(dl, lane, i + 1, di1 - pp);
          el = sel_lane(el, lane, mm, 0.0);
          if (own) Ar[i + 1] = carry;
          split = true;
          break;
        }
        const double y = nyls_rsqrt(x);
        el = sel_lane(el, lane, i + 1, x * y);
        sn = f * y;
        cs = g * y;
        g = di1 - pp;
        r = (di - g) * sn + 2.0 * cs * b;
        pp = sn * r;
        dl = sel_lane(dl, lane, i + 1, g + pp);
        g = cs * r - b;
        if (own) Ar[i + 1] = sn * z0 + cs * carry;
        carry = cs * z0 - sn * carry;
        z0 = (own && i > l) ? Ar[i - 1] : 0.0;
      }
      if (split) continue;
      if (own) Ar[l] = carry;
      dl = sel_lane(dl, lane, l, nyls_rdlane(dl, l) - pp);
      el = sel_lane(el, lane, l, g);
      el = sel_lane(el, lane, mm, 0.0);
    }
  }
  nyls_wave_lds_sync();
  }  // stage != QL_REPLAY

  // 4. sort descending (ties by index), sign each eigenvector (largest |entry| positive,
  //    first on ties), cut-off, W = U_r Lambda_r^{-1/2}
  int ps = 0;
  for (int j = 0; j < m; ++j) {
    const double lj = nyls_rdlane(dl, j);
    ps += (lj > dl) || (lj == dl && j < lane);
  }
  double sg = 1.0;
  if (own) {
    int jmax = 0;
    double vmax = -1.0;
    for (int s2 = 0; s2 < m; ++s2) {
      const double a = fabs(A[s2 * lda + lane]);
      if (a > vmax) { vmax = a; jmax = s2; }
    }
    sg = A[jmax * lda + lane] < 0.0 ? -1.0 : 1.0;
    pos[lane] = ps;
    vv[lane] = sg;
    tt[ps] = dl;  // sorted eigenvalues
  }
  nyls_wave_lds_sync();
  const double lam1 = tt[0];
  int rank = 0;
  for (int k = 0; k < m; ++k) rank += (tt[k] > d.tau * lam1) ? 1 : 0;
  if (own) {
    for (int k = 0; k < m; ++k) {  // row s = lane of U and W
      const int pk = pos[k];
      const double u = vv[k] * Ar[k];
      ws[L.U + lane * m + pk] = u;
      ws[L.W + lane * m + pk] = pk < rank ? u / sqrt(tt[pk]) : 0.0;
    }
    ws[L.lam + lane] = tt[lane];
  }
  if (lane == 0) {
    int bits = 0;
    if (rank < m) bits |= NYLS_S_TRUNCATED;
    if (!converged) bits |= NYLS_S_EIG_NOCONV;
    if (!(lam1 == lam1) || rank == 0) bits |= NYLS_S_NONFINITE;
    ws[L.info + 0] = (double)rank;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 2] = (double)iters;
    ws[L.info + 6] = 0.0;  // k_ql_lanes' sweep count; the adjoint's pass count later
    ws[L.info + 7] = 0.0;
  }
}

// Implicit QL on the tridiagonal (d, e) of QL_REDUCE with one lane per instance (64
// instances per wavefront): the scalar recurrences of a sweep are a serial chain, so a
// wavefront that runs 64 of them side by side keeps its lanes busy where the one-wave
// kernel runs one chain on all 64 lanes.  The arithmetic and the order of operations are
// those of step 3 of k_eig_ql; the plane rotations are logged to the instance's workspace
// (its rotation-log region) for the replay on Q.  An instance whose log
// would overflow is marked (info[7] = 2) and redone by k_eig_ql(QL_REDO).
__global__ __launch_bounds__(64) void k_ql_lanes(const nyls_desc* __restrict__ desc,
                                                 double* __restrict__ wsbase, int batch, int ipw) {
  __shared__ double dv[kQlMaxM][64], ev[kQlMaxM][64];  // [index][lane]: conflict-free
  const int lane = threadIdx.x;
  const int inst = blockIdx.x * ipw + lane;  // ipw <= 64 instances per wavefront
  const bool act = lane < ipw && inst < batch && desc[inst < batch ? inst : 0].m <= kQlMaxM;
  const nyls_desc& d = desc[act ? inst : 0];
  const int m = act ? d.m : 0;
  const nyls_wsl L = nyls_layout(d.m, d.p, 0);
  double* ws = wsbase + d.ws;
  for (int k = 0; k < m; ++k) {
    dv[k][lane] = ws[L.lam + k];
    ev[k][lane] = ws[L.W + k];
  }
  double* lg = ws + L.log;
  const int cap = (int)((L.aux - L.log) / 2);  // log entries (pairs of doubles)
  const double eps = 2.220446049250313e-16;
  int iters = 0, pos = 0, nsw = 0;
  bool converged = true, overflow = false;
  // nx > l: the first index above l whose off-diagonal passes the split test (m - 1 counts
  // as passing), known from the last sweep or scan; otherwise unknown.  The sweep below
  // evaluates the test for every index it finalises, so a full scan is needed only at the
  // start and after an exact deflation; the chosen mm is the first passing index from l,
  // as in the plain scan.
  int nx = -1;
  for (int l = 0; l < m && !overflow; ++l) {
    int it = 0;
    for (;;) {
      int mm = l;
      if (l < m - 1 && !(fabs(ev[l][lane]) <= eps * (fabs(dv[l][lane]) + fabs(dv[l + 1][lane])))) {
        if (nx > l) {
          mm = nx;
        } else {
          mm = l + 1;
          while (mm < m - 1 && !(fabs(ev[mm][lane]) <= eps * (fabs(dv[mm][lane]) + fabs(dv[mm + 1][lane]))))
            ++mm;
          nx = mm;
        }
      }
      if (mm == l) break;
      if (++it > kQlMaxIter) { converged = false; break; }
      if (pos + 1 + (mm - l) > cap) { overflow = true; break; }
      ++iters;
      const double dL = dv[l][lane], eL = ev[l][lane];
      double g = (dv[l + 1][lane] - dL) / (2.0 * eL);
      double r = sqrt(g * g + 1.0);
      g = dv[mm][lane] - dL + eL / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, pp = 0.0;
      const int hdr = pos++;
      int nrot = 0, sm = mm;
      bool split = false;
      double ei = ev[mm - 1][lane], di = dv[mm - 1][lane], di1 = dv[mm][lane], dup = 0.0;
      for (int i = mm - 1; i >= l; --i) {
        const int ip = i > 0 ? i - 1 : 0;  // next rotation's entries (unused after the last)
        const double ein = ev[ip][lane], din = dv[ip][lane];
        const double f = sn * ei, b = cs * ei;
        const double x = f * f + g * g;
        if (x == 0.0) {  // exact deflation: the chase stops here
          ev[i + 1][lane] = 0.0;
          dv[i + 1][lane] = di1 - pp;
          ev[mm][lane] = 0.0;
          split = true;
          break;
        }
        const double y = nyls_rsqrt(x);
        const double en = x * y;
        ev[i + 1][lane] = en;
        sn = f * y;
        cs = g * y;
        g = di1 - pp;
        r = (di - g) * sn + 2.0 * cs * b;
        pp = sn * r;
        const double dn = g + pp;
        dv[i + 1][lane] = dn;
        // index i + 1 is final for this sweep (its d above was written one step earlier)
        if (i + 1 < mm && fabs(en) <= eps * (fabs(dn) + fabs(dup))) sm = i + 1;
        dup = dn;
        g = cs * r - b;
        lg[2 * pos] = cs;
        lg[2 * pos + 1] = sn;
        ++pos;
        ++nrot;
        di1 = di;
        di = din;
        ei = ein;
      }
      lg[2 * hdr] = (double)mm;
      lg[2 * hdr + 1] = (double)nrot;
      ++nsw;
      if (split) {
        nx = -1;
        continue;
      }
      dv[l][lane] -= pp;
      ev[l][lane] = g;
      ev[mm][lane] = 0.0;
      nx = sm;
    }
  }
  if (!act) return;
  for (int k = 0; k < m; ++k) ws[L.lam + k] = dv[k][lane];
  ws[L.info + 2] = (double)iters;
  ws[L.info + 6] = (double)nsw;
  ws[L.info + 7] = overflow ? 2.0 : (converged ? 0.0 : 1.0);
}

size_t eig_lds_bytes(int maxm, bool vlds) {
  const size_t mats = (size_t)(vlds ? 2 : 1) * maxm * (maxm + 1) * sizeof(double);
  const size_t tail = (64 * 3 + 8 + NYLS_MAX_M) * sizeof(double) + (64 * 2 + NYLS_MAX_M) * sizeof(int) +
                      NYLS_MAX_M * sizeof(double);
  return mats + tail;
}

}  // namespace

hipError_t nyls_launch_eig(const nyls_plan_view& pv, double* ws, int single, hipStream_t st) {
  if (pv.nb_mask & (4 | 16)) {  // some instance has m <= 64
    const int mq = pv.maxm < kQlMaxM ? pv.maxm : kQlMaxM;
    const int lda = mq | 1;
    const size_t lds = (size_t)lda * lda * sizeof(double) + 3 * 64 * sizeof(double) +
                       64 * sizeof(int);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_ql),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const dim3 grid(single >= 0 ? 1 : pv.batch);
    if (single >= 0 || pv.eig_ql) {
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_FULL);
    } else {
      const int ipw = pv.ql_lanes >= 1 && pv.ql_lanes <= kQlLaneInst ? pv.ql_lanes : kQlLaneInst;
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_REDUCE);
      hipLaunchKernelGGL(k_ql_lanes, dim3((pv.batch + ipw - 1) / ipw), dim3(64), 0, st, pv.d_desc,
                         ws, pv.batch, ipw);
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_REPLAY);
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_REDO);
    }
  }
  if (!(pv.nb_mask & 256)) return hipGetLastError();
  const bool vlds = pv.maxm <= kVldsMaxM;
  const size_t lds = eig_lds_bytes(pv.maxm, vlds);
  const int grid = single >= 0 ? 1 : pv.batch;
  if (vlds) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig<true>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_eig<true>, dim3(grid), dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order,
                       ws, single);
  } else {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig<false>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_eig<false>, dim3(grid), dim3(NYLS_BLOCK), lds, st, pv.d_desc, pv.d_order,
                       ws, single);
  }
  return hipGetLastError();
}
