// Nystrom basis: landmark kernel matrix K_mm, its eigendecomposition and the feature
// transform W = U_r Lambda_r^{-1/2} (App. A.2, eq32), one wavefront per instance.
//
// K_mm (up to 128 x 128) is kept in LDS, reduced to tridiagonal form by Householder
// reflections and diagonalised by implicit QL (k_eig_ql for m <= 64 with one row per lane,
// staged with the lane-parallel QL of k_ql_lanes for batches; k_eig_ql2 for 64 < m <= 128
// with two rows per lane; k_eig_wide for wider bases, with the matrix in the workspace).  Afterwards eigenvalues are sorted descending, each eigenvector is
// signed so its largest-magnitude entry (first on ties) is positive, and eigenpairs with
// lambda_k <= tau * lambda_1 are dropped (the retained rank r goes to info[0]).
#include "nyls_dense.h"

namespace {

constexpr int kQlMaxM = 64;  // bases up to this size use k_eig_ql, up to twice it k_eig_ql2

__device__ inline int instance_of(const int32_t* order, int single) {
  return single >= 0 ? single : (order ? order[blockIdx.x] : (int)blockIdx.x);
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
//  3. Implicit QL on (d, e) with the shift from the leading 2 x 2 block of the active part
//     (the published implicit QL method for symmetric tridiagonal matrices of Bowdler,
//     Martin, Reinsch and Wilkinson, "The QR and QL algorithms for symmetric matrices",
//     Numer. Math. 11, 1968, known as tql2: the same shift, bulge chase and split test,
//     re-organised for wavefront lanes);
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
// Fewest m > 64 instances for which the staged QL (one lane per instance) is used.
constexpr int kQlStagedMin = 32;

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
// Takes the instances with LO < m <= MAXM, at most LN per wavefront.
template <int MAXM, int LO = MAXM - kQlMaxM, int LN = 64>
__global__ __launch_bounds__(64) void k_ql_lanes(const nyls_desc* __restrict__ desc,
                                                 double* __restrict__ wsbase, int batch, int ipw) {
  __shared__ double dv[MAXM][LN], ev[MAXM][LN];  // [index][lane]: conflict-free
  const int lane = threadIdx.x;
  const int inst = blockIdx.x * ipw + lane;  // ipw <= LN instances per wavefront
  const int mi = desc[inst < batch ? inst : 0].m;
  const bool act = lane < ipw && lane < LN && inst < batch && mi <= MAXM && mi > LO;
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

// ---- one wavefront per instance, 64 < m <= 128: the steps of k_eig_ql with two rows per lane ----
//
// Lane l owns rows (and d, e entries) l and l + 64 of the same LDS layout; values indexed by
// a wave-uniform i are read from the half that holds them.  The QL sweeps need no exchange
// between the halves beyond those reads, so the whole solver stays inside one wavefront
// (about 9 m^3 flop against the tens of cyclic Jacobi sweeps of m^3 each it replaces).
__device__ inline double rd2(double v0, double v1, int i) {
  return i < 64 ? nyls_rdlane(v0, i) : nyls_rdlane(v1, i - 64);
}
__device__ inline void wr2(double& v0, double& v1, int lane, int i, double x) {
  v0 = lane == i ? x : v0;
  v1 = lane + 64 == i ? x : v1;
}

__global__ __launch_bounds__(64) void k_eig_ql2(const nyls_desc* __restrict__ desc,
                                                const int32_t* __restrict__ order,
                                                double* __restrict__ wsbase, int single, int lda,
                                                int stage) {
  extern __shared__ double sm[];
  const int inst = instance_of(order, single);
  const nyls_desc& d = desc[inst];
  const int m = d.m;
  if (m <= kQlMaxM || m > 2 * kQlMaxM) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  if (stage == QL_REDO && ws[L.info + 7] != 2.0) return;
  if (stage == QL_REPLAY && ws[L.info + 7] == 2.0) return;  // log overflow: QL_REDO
  const int lane = threadIdx.x;
  double* A = sm;                    // [lda][lda]: K_mm, then Q, then Z
  double* vv = A + lda * lda;        // [128] reflector / signs
  double* tt = vv + 128;             // [128] column products / sorted eigenvalues
  double* tl = tt + 128;             // [128] landmark times
  double* ww = tl;                   // [128] Householder w (after tl's last use)
  int* pos = reinterpret_cast<int*>(tl + 128);  // [128] sorted position
  const int j0 = lane, j1 = lane + 64;  // the lane's rows
  const bool own0 = j0 < m, own1 = j1 < m;
  double* A0 = A + j0 * lda;
  double* A1 = A + (own1 ? j1 : j0) * lda;  // lanes without a second row alias the first
  const double eps = 2.220446049250313e-16;
  double d0 = 0.0, d1 = 0.0, e0 = 0.0, e1 = 0.0, b0 = 0.0, b1 = 0.0;
  int iters = 0;
  bool converged = true;

  if (stage == QL_REPLAY) {
    // Q and the eigenvalues from the workspace, then the sweeps k_ql_lanes logged: each is a
    // header (mm, number of rotations k) and k pairs (c, s) for columns i = mm - 1, mm - 2, ...
    // A sweep's window (header and at most m - 1 <= 127 rotations) is two entries per lane;
    // the next window is loaded while this one is applied.
    for (int j = 0; j < m; ++j) A0[j] = ws[L.U + j0 * m + j];
    if (own1)
      for (int j = 0; j < m; ++j) A1[j] = ws[L.U + j1 * m + j];
    d0 = ws[L.lam + j0];
    d1 = own1 ? ws[L.lam + j1] : 0.0;
    iters = (int)ws[L.info + 2];
    converged = ws[L.info + 7] == 0.0;
    const double* lg = ws + L.log;
    const int nsw = (int)ws[L.info + 6];
    const int cap = (int)((L.aux - L.log) / 2);
    auto fetch = [&](int e0, double& a0, double& b0, double& a1, double& b1) {
      const int e = e0 + lane;
      a0 = e < cap ? lg[2 * e] : 0.0;
      b0 = e < cap ? lg[2 * e + 1] : 0.0;
      a1 = e + 64 < cap ? lg[2 * (e + 64)] : 0.0;
      b1 = e + 64 < cap ? lg[2 * (e + 64) + 1] : 0.0;
    };
    double ca0, cb0, ca1, cb1;
    fetch(0, ca0, cb0, ca1, cb1);
    int hdr = 0;
    for (int sw = 0; sw < nsw; ++sw) {
      const int mm = (int)nyls_rdlane(ca0, 0), nrot = (int)nyls_rdlane(cb0, 0);
      const int nxt = hdr + 1 + nrot;
      double na0, nb0, na1, nb1;
      fetch(nxt, na0, nb0, na1, nb1);
      double c0 = A0[mm], c1 = own1 ? A1[mm] : 0.0;
      for (int k = 0; k < nrot; ++k) {
        const int i = mm - 1 - k;
        const double cs = rd2(ca0, ca1, k + 1), sn = rd2(cb0, cb1, k + 1);
        const double z0 = A0[i];
        A0[i + 1] = sn * z0 + cs * c0;
        c0 = cs * z0 - sn * c0;
        if (own1) {
          const double z1 = A1[i];
          A1[i + 1] = sn * z1 + cs * c1;
          c1 = cs * z1 - sn * c1;
        }
      }
      A0[mm - nrot] = c0;
      if (own1) A1[mm - nrot] = c1;
      ca0 = na0;
      cb0 = nb0;
      ca1 = na1;
      cb1 = nb1;
      hdr = nxt;
    }
    nyls_wave_lds_sync();
  } else {
  const double inv_sigma = 1.0 / d.sigma;
  tl[j0] = nyls_grid_t(d, d.lidx[j0]);
  if (own1) tl[j1] = nyls_grid_t(d, d.lidx[j1]);
  nyls_wave_lds_sync();
  for (int j = 0; j < m; ++j) {
    const double tj = tl[j];
    const double z0 = (tl[j0] - tj) * inv_sigma;
    A0[j] = exp(-z0 * z0);
    if (own1) {
      const double z1 = (tl[j1] - tj) * inv_sigma;
      A1[j] = exp(-z1 * z1);
    }
  }
  nyls_wave_lds_sync();

  // 1. tridiagonalisation
  for (int k = 0; k + 2 < m; ++k) {
    const bool a0 = j0 > k, a1 = own1 && j1 > k;
    const double x0 = a0 ? A0[k] : 0.0, x1v = a1 ? A1[k] : 0.0;
    const double sig2 = nyls_wave_sum_dpp(x0 * x0 + x1v * x1v);
    const double xk1 = rd2(x0, x1v, k + 1);
    wr2(d0, d1, lane, k, A[k * lda + k]);
    if (!(sig2 - xk1 * xk1 > 0.0)) {
      wr2(e0, e1, lane, k, xk1);
      if (a0) A0[k] = 0.0;
      if (a1) A1[k] = 0.0;
      nyls_wave_lds_sync();
      continue;
    }
    const double alpha = xk1 >= 0.0 ? -sqrt(sig2) : sqrt(sig2);
    const double beta = 1.0 / (sig2 - alpha * xk1);
    const double v0 = a0 ? (j0 == k + 1 ? x0 - alpha : x0) : 0.0;
    const double v1 = a1 ? (j1 == k + 1 ? x1v - alpha : x1v) : 0.0;
    wr2(e0, e1, lane, k, alpha);
    wr2(b0, b1, lane, k, beta);
    vv[j0] = v0;
    vv[j1] = v1;
    if (a0) A0[k] = v0;
    if (a1) A1[k] = v1;
    nyls_wave_lds_sync();
    double p0 = a0 ? beta * nyls_row_dot(A0, vv, k + 1, m) : 0.0;
    double p1 = a1 ? beta * nyls_row_dot(A1, vv, k + 1, m) : 0.0;
    const double K = 0.5 * beta * nyls_wave_sum_dpp(v0 * p0 + v1 * p1);
    const double w0 = p0 - K * v0, w1 = p1 - K * v1;
    ww[j0] = w0;
    ww[j1] = w1;
    nyls_wave_lds_sync();
    if (a0) nyls_row_rank2(A0, v0, ww, w0, vv, k + 1, m);
    if (a1) nyls_row_rank2(A1, v1, ww, w1, vv, k + 1, m);
    nyls_wave_lds_sync();
  }
  {
    const double a22 = A[(m - 2) * lda + m - 2], a32 = A[(m - 1) * lda + m - 2],
                 a33 = A[(m - 1) * lda + m - 1];
    wr2(d0, d1, lane, m - 2, a22);
    wr2(e0, e1, lane, m - 2, a32);
    wr2(d0, d1, lane, m - 1, a33);
    wr2(e0, e1, lane, m - 1, 0.0);
  }
  nyls_wave_lds_sync();

  // 2. Q in place (the trailing 2 x 2 block starts as the identity)
  if (j0 >= m - 2) {
    A0[m - 2] = j0 == m - 2 ? 1.0 : 0.0;
    A0[m - 1] = j0 == m - 1 ? 1.0 : 0.0;
  }
  if (own1 && j1 >= m - 2) {
    A1[m - 2] = j1 == m - 2 ? 1.0 : 0.0;
    A1[m - 1] = j1 == m - 1 ? 1.0 : 0.0;
  }
  nyls_wave_lds_sync();
  for (int k = m - 3; k >= 0; --k) {
    const bool a0 = j0 > k, a1 = own1 && j1 > k;
    const double v0 = a0 ? A0[k] : 0.0, v1 = a1 ? A1[k] : 0.0;
    const double beta = rd2(b0, b1, k);
    if (beta != 0.0) {
      vv[j0] = v0;
      vv[j1] = v1;
      nyls_wave_lds_sync();
      // t_j = sum_i v_i Q[i][j] for the lane's columns j0 and j1
      const double t0 = a0 ? nyls_col_dot(vv, A + j0, lda, k + 1, m) : 0.0;
      const double t1 = a1 ? nyls_col_dot(vv, A + j1, lda, k + 1, m) : 0.0;
      tt[j0] = beta * t0;
      tt[j1] = beta * t1;
      nyls_wave_lds_sync();
      if (a0) nyls_row_rank1(A0, v0, tt, k + 1, m);
      if (a1) nyls_row_rank1(A1, v1, tt, k + 1, m);
    }
    if (j0 == k)
      for (int j = k; j < m; ++j) A0[j] = j == k ? 1.0 : 0.0;
    if (own1 && j1 == k)
      for (int j = k; j < m; ++j) A1[j] = j == k ? 1.0 : 0.0;
    if (a0) A0[k] = 0.0;
    if (a1) A1[k] = 0.0;
    nyls_wave_lds_sync();
  }

  if (stage == QL_REDUCE) {
    // d, e and Q for k_ql_lanes and the replay (W and U are written at the end)
    ws[L.lam + j0] = d0;
    ws[L.W + j0] = e0;
    for (int j = 0; j < m; ++j) ws[L.U + j0 * m + j] = A0[j];
    if (own1) {
      ws[L.lam + j1] = d1;
      ws[L.W + j1] = e1;
      for (int j = 0; j < m; ++j) ws[L.U + j1 * m + j] = A1[j];
    }
    return;
  }

  // 3. implicit QL on (d, e), rotations accumulated into the rows of Z.  d and e live in LDS
  //    for the sweeps (vv and tt are free until step 4): every lane runs the scalar chain on
  //    broadcast reads issued one rotation ahead, lane 0 writes the updated entries, and no
  //    lane-to-scalar moves sit on the chain.  Rotation i reads d_i, d_{i+1} and e_i, which no
  //    earlier rotation of the sweep has rewritten (rotation i rewrites d_{i+1}, e_{i+1}).
  double* dv = vv;
  double* ev = tt;
  dv[j0] = d0;
  ev[j0] = e0;
  dv[j1] = own1 ? d1 : 0.0;
  ev[j1] = own1 ? e1 : 0.0;
  nyls_wave_lds_sync();
  for (int l = 0; l < m; ++l) {
    int it = 0;
    for (;;) {
      const bool s0 = j0 >= l && (j0 == m - 1 ||
                                  (j0 < m - 1 && fabs(ev[j0]) <= eps * (fabs(dv[j0]) + fabs(dv[j0 + 1]))));
      const bool s1 = own1 && j1 >= l &&
                      (j1 == m - 1 || (j1 < m - 1 && fabs(ev[j1]) <= eps * (fabs(dv[j1]) + fabs(dv[j1 + 1]))));
      const unsigned long long mk0 = __ballot(s0), mk1 = __ballot(s1);
      const int mm = mk0 ? __ffsll((long long)mk0) - 1 : 63 + __ffsll((long long)mk1);
      if (mm == l) break;
      if (++it > kQlMaxIter) { converged = false; break; }
      ++iters;
      const double dL = dv[l], eL = ev[l];
      double g = (dv[l + 1] - dL) / (2.0 * eL);
      double r = sqrt(g * g + 1.0);
      g = dv[mm] - dL + eL / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, pp = 0.0;
      double c0 = A0[mm], c1 = own1 ? A1[mm] : 0.0;  // carries
      double z0 = A0[mm - 1], z1 = own1 ? A1[mm - 1] : 0.0;
      double ei = ev[mm - 1], di = dv[mm - 1], di1 = dv[mm];
      bool split = false;
      for (int i = mm - 1; i >= l; --i) {
        const int ip = i > 0 ? i - 1 : 0;  // next rotation's entries (unused after the last)
        const double ein = ev[ip], din = dv[ip];
        const double f = sn * ei, b = cs * ei;
        const double x = f * f + g * g;
        if (x == 0.0) {  // exact deflation: the chase stops here
          if (lane == 0) {
            ev[i + 1] = 0.0;
            dv[i + 1] = di1 - pp;
            ev[mm] = 0.0;
          }
          A0[i + 1] = c0;
          if (own1) A1[i + 1] = c1;
          split = true;
          break;
        }
        const double y = nyls_rsqrt(x);
        const double en = x * y;
        sn = f * y;
        cs = g * y;
        g = di1 - pp;
        r = (di - g) * sn + 2.0 * cs * b;
        pp = sn * r;
        if (lane == 0) {
          ev[i + 1] = en;
          dv[i + 1] = g + pp;
        }
        g = cs * r - b;
        A0[i + 1] = sn * z0 + cs * c0;
        c0 = cs * z0 - sn * c0;
        if (own1) A1[i + 1] = sn * z1 + cs * c1;
        c1 = cs * z1 - sn * c1;
        z0 = i > l ? A0[i - 1] : 0.0;
        z1 = (own1 && i > l) ? A1[i - 1] : 0.0;
        di1 = di;
        di = din;
        ei = ein;
      }
      if (!split) {
        A0[l] = c0;
        if (own1) A1[l] = c1;
        if (lane == 0) {
          dv[l] -= pp;
          ev[l] = g;
          ev[mm] = 0.0;
        }
      }
      nyls_wave_lds_sync();
    }
  }
  d0 = dv[j0];
  d1 = own1 ? dv[j1] : 0.0;
  nyls_wave_lds_sync();
  }  // stage != QL_REPLAY

  // 4. sort descending (ties by index), sign each eigenvector (largest |entry| positive,
  //    first on ties), cut-off, W = U_r Lambda_r^{-1/2}
  int ps0 = 0, ps1 = 0;
  for (int j = 0; j < m; ++j) {
    const double lj = rd2(d0, d1, j);
    ps0 += (lj > d0) || (lj == d0 && j < j0);
    ps1 += (lj > d1) || (lj == d1 && j < j1);
  }
  auto col_sign = [&](int c) {
    int jmax = 0;
    double vmax = -1.0;
    for (int s2 = 0; s2 < m; ++s2) {
      const double a = fabs(A[s2 * lda + c]);
      if (a > vmax) { vmax = a; jmax = s2; }
    }
    return A[jmax * lda + c] < 0.0 ? -1.0 : 1.0;
  };
  pos[j0] = ps0;
  vv[j0] = col_sign(j0);
  tt[ps0] = d0;
  if (own1) {
    pos[j1] = ps1;
    vv[j1] = col_sign(j1);
    tt[ps1] = d1;
  }
  nyls_wave_lds_sync();
  const double lam1 = tt[0];
  int rank = 0;
  for (int k = 0; k < m; ++k) rank += (tt[k] > d.tau * lam1) ? 1 : 0;
  for (int h = 0; h < 2; ++h) {
    const int row = h ? j1 : j0;
    if (row >= m) continue;
    const double* Ar = h ? A1 : A0;
    for (int k = 0; k < m; ++k) {
      const int pk = pos[k];
      const double u = vv[k] * Ar[k];
      ws[L.U + row * m + pk] = u;
      ws[L.W + row * m + pk] = pk < rank ? u / sqrt(tt[pk]) : 0.0;
    }
    ws[L.lam + row] = tt[row];
  }
  if (lane == 0) {
    int bits = 0;
    if (rank < m) bits |= NYLS_S_TRUNCATED;
    if (!converged) bits |= NYLS_S_EIG_NOCONV;
    if (!(lam1 == lam1) || rank == 0) bits |= NYLS_S_NONFINITE;
    ws[L.info + 0] = (double)rank;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 2] = (double)iters;
    ws[L.info + 6] = 0.0;
    ws[L.info + 7] = 0.0;
  }
}

// ---- wide bases (NYLS_NARROW_MAX_M < m <= NYLS_MAX_M): K_mm in the workspace ----
//
// The matrix no longer fits in LDS, so the steps of k_eig_ql run on the instance's U block
// (L2-resident), thread j owning column j: K_mm and every trailing block stay exactly
// symmetric (the rank-2 update adds its two products in an order-independent way), so
// column j is also row j, and every step reads and writes with coalesced accesses.  The
// column loops load eight entries before they store any (the loads of one thread would
// otherwise wait behind its own stores, one L2 round trip per entry).
//  1. (k_eig_wide, WIDE_REDUCE) Householder reduction as in step 1 of k_eig_ql, reflector k
//     kept in row k;
//  2. Q = H_0 ... H_{m-3} formed in place, then stored transposed in the T scratch
//     (ZT[c m + i] = Z[i][c]);
//  3. (k_ql_wide) implicit QL on (d, e), one wavefront per instance carrying the chain,
//     logging the rotations;
//  4. (k_eig_wide_replay) the logged rotations applied to the rows of Z: rows are
//     independent, so four workgroups per instance each hold 64 rows in LDS (one per lane);
//  5. (k_eig_wide, WIDE_FINISH) the ordering, signs, cut-off and W of step 4 of k_eig_ql.
// A rotation log that overflowed (more than 2 m^2 rotations) leaves NYLS_S_EIG_NOCONV set.
enum { WIDE_REDUCE = 0, WIDE_FINISH = 1 };
constexpr int kWideRows = 64;  // rows of Z per replay workgroup

// Entries of a thread-owned column loaded together before any is used or stored: a thread's
// loads would otherwise each wait a round trip to L2 (and behind its own earlier stores).
constexpr int kColBatch = 8;

// A[c m + j] -= delta(c) for c in [c0, m) (thread-owned column j), in batches of kColBatch
// loads issued before their stores.
template <class F>
__device__ inline void wide_col_update(double* A, int m, int j, int c0, F delta) {
  int c = c0;
  for (; c + kColBatch <= m; c += kColBatch) {
    double v[kColBatch];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) v[u] = A[(c + u) * m + j];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) A[(c + u) * m + j] = v[u] - delta(c + u);
  }
  for (; c < m; ++c) A[c * m + j] -= delta(c);
}

// sum over c in [c0, m) of A[c m + j] * x[c] (x in LDS), added in order of c
__device__ inline double wide_col_dot(const double* A, int m, int j, int c0, const double* x) {
  double acc = 0.0;
  int c = c0;
  for (; c + kColBatch <= m; c += kColBatch) {
    double v[kColBatch];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) v[u] = A[(c + u) * m + j];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) acc += v[u] * x[c + u];
  }
  for (; c < m; ++c) acc += A[c * m + j] * x[c];
  return acc;
}

// Instances with lo < m <= hi (the wide bases, or batches of 64 < m <= 128, where the
// one-wave kernel's K_mm fills half a CU's LDS); redo: leave instances whose rotation log
// overflowed to k_eig_ql2(QL_REDO).
__global__ __launch_bounds__(NYLS_BLOCK) void k_eig_wide(const nyls_desc* __restrict__ desc,
                                                         double* __restrict__ wsbase, int stage,
                                                         int lo, int hi, int redo) {
  __shared__ double vv[NYLS_MAX_M], ww[NYLS_MAX_M], tl[NYLS_MAX_M], bt[NYLS_MAX_M];
  __shared__ double dd[NYLS_MAX_M], ee[NYLS_MAX_M], red[NYLS_BLOCK / 64];
  __shared__ int pos[NYLS_MAX_M];
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m;
  if (m <= lo || m > hi) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const int j = threadIdx.x;
  const bool own = j < m;
  double* A = ws + L.U;     // [m][m] K_mm, then Q
  double* ZT = ws + L.tmp;  // [m][m] Z transposed
  if (stage == WIDE_REDUCE) {
    const double inv_sigma = 1.0 / d.sigma;
    if (own) tl[j] = nyls_grid_t(d, d.lidx[j]);
    __syncthreads();
    if (own)
      for (int c = 0; c < m; ++c) {
        const double z = (tl[c] - tl[j]) * inv_sigma;
        A[c * m + j] = exp(-z * z);
      }
    __syncthreads();
    // 1. tridiagonalisation
    for (int k = 0; k + 2 < m; ++k) {
      const bool act = own && j > k;
      const double x = act ? A[k * m + j] : 0.0;  // row k = column k below the diagonal
      const double sig2 = nyls_block_sum(x * x, red);
      const double xk1 = A[k * m + k + 1];
      if (j == 0) dd[k] = A[k * m + k];
      if (!(sig2 - xk1 * xk1 > 0.0)) {
        if (j == 0) {
          ee[k] = xk1;
          bt[k] = 0.0;
        }
        continue;  // nothing below the subdiagonal: no reflector (the next block sum syncs)
      }
      const double alpha = xk1 >= 0.0 ? -sqrt(sig2) : sqrt(sig2);
      const double beta = 1.0 / (sig2 - alpha * xk1);
      const double v = act ? (j == k + 1 ? x - alpha : x) : 0.0;
      if (j == 0) {
        ee[k] = alpha;
        bt[k] = beta;
      }
      if (own) vv[j] = v;
      __syncthreads();
      // p = beta B v (column j of B is row j)
      const double pj = act ? beta * wide_col_dot(A, m, j, k + 1, vv) : 0.0;
      const double K = 0.5 * beta * nyls_block_sum(v * pj, red);
      const double w = pj - K * v;
      if (own) ww[j] = w;
      __syncthreads();
      if (act) {
        wide_col_update(A, m, j, k + 1,
                        [&](int c) { return __dadd_rn(__dmul_rn(vv[c], w), __dmul_rn(ww[c], v)); });
        A[k * m + j] = v;  // reflector k
      }
      __syncthreads();
    }
    if (j == 0) {
      dd[m - 2] = A[(m - 2) * m + m - 2];
      ee[m - 2] = A[(m - 1) * m + m - 2];
      dd[m - 1] = A[(m - 1) * m + m - 1];
      ee[m - 1] = 0.0;
    }
    // the owners of the last two columns overwrite those entries next
    __syncthreads();
    // 2. Q in place (the trailing 2 x 2 block starts as the identity)
    if (own && j >= m - 2) {
      A[(m - 2) * m + j] = j == m - 2 ? 1.0 : 0.0;
      A[(m - 1) * m + j] = j == m - 1 ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = m - 3; k >= 0; --k) {
      const bool act = own && j > k;
      if (act) vv[j] = A[k * m + j];
      __syncthreads();
      const double beta = bt[k];
      if (act && beta != 0.0) {
        const double t = beta * wide_col_dot(A, m, j, k + 1, vv);  // (v^T Q)_j
        wide_col_update(A, m, j, k + 1, [&](int i) { return vv[i] * t; });
      }
      if (own && j >= k) A[k * m + j] = j == k ? 1.0 : 0.0;  // row k = e_k
      if (j == k)
        for (int i = k + 1; i < m; ++i) A[i * m + k] = 0.0;  // column k = e_k
      __syncthreads();
    }
    if (own) {
      ws[L.lam + j] = dd[j];
      ws[L.W + j] = ee[j];
      for (int i = 0; i < m; ++i) ZT[j * m + i] = A[i * m + j];
    }
    return;
  }

  // 5. ordering, signs, cut-off, W and U
  const int flag = (int)ws[L.info + 7];
  if (redo && flag == 2) return;  // recomputed by k_eig_ql2(QL_REDO)
  const double dj = own ? ws[L.lam + j] : 0.0;
  if (own) dd[j] = dj;
  __syncthreads();
  int ps = 0;
  double sg = 1.0;
  if (own) {
    for (int q = 0; q < m; ++q) {
      const double lq = dd[q];
      ps += (lq > dj) || (lq == dj && q < j);
    }
    // eigenvector j is column j of Z = row j of ZT: largest |entry| positive, first on ties
    int smax = 0;
    double vmax = -1.0;
    for (int s2 = 0; s2 < m; ++s2) {
      const double a = fabs(ZT[j * m + s2]);
      if (a > vmax) {
        vmax = a;
        smax = s2;
      }
    }
    sg = ZT[j * m + smax] < 0.0 ? -1.0 : 1.0;
    pos[j] = ps;
    vv[j] = sg;
    tl[ps] = dj;  // eigenvalues in descending order
  }
  __syncthreads();
  const double lam1 = tl[0];
  int rank = 0;
  for (int q = 0; q < m; ++q) rank += (tl[q] > d.tau * lam1) ? 1 : 0;
  if (own) {
    for (int q = 0; q < m; ++q) {
      const int pq = pos[q];
      const double u = vv[q] * ZT[q * m + j];  // Z[j][q]
      ws[L.U + j * m + pq] = u;
      ws[L.W + j * m + pq] = pq < rank ? u / sqrt(tl[pq]) : 0.0;
    }
    ws[L.lam + j] = tl[j];
  }
  if (j == 0) {
    int bits = 0;
    if (rank < m) bits |= NYLS_S_TRUNCATED;
    if (flag != 0) bits |= NYLS_S_EIG_NOCONV;
    if (!(lam1 == lam1) || rank == 0) bits |= NYLS_S_NONFINITE;
    ws[L.info + 0] = (double)rank;
    ws[L.info + 1] = (double)bits;
    ws[L.info + 6] = 0.0;
    ws[L.info + 7] = 0.0;
  }
}

// 3. implicit QL on (d, e) of a wide basis, logging the rotations as k_ql_lanes does (same
// shift, chase, split test and log format), one wavefront per instance with every lane
// carrying the (wave-uniform) scalar chain: d and e sit in LDS, lane 0 writes the updated
// entries and the log, and the first negligible off-diagonal of a new sweep is found with
// one ballot per 64 entries.  Uniform control flow keeps the chain free of the exec-mask
// bookkeeping of the lane-per-instance kernel, whose single active lane would carry it here.
__global__ __launch_bounds__(64) void k_ql_wide(const nyls_desc* __restrict__ desc,
                                                double* __restrict__ wsbase) {
  __shared__ double dv[NYLS_MAX_M], ev[NYLS_MAX_M];
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m;
  if (m <= NYLS_NARROW_MAX_M) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const int lane = threadIdx.x;
  for (int k = lane; k < m; k += 64) {
    dv[k] = ws[L.lam + k];
    ev[k] = ws[L.W + k];
  }
  nyls_wave_lds_sync();
  double* lg = ws + L.log;
  const int cap = (int)((L.aux - L.log) / 2);
  const double eps = 2.220446049250313e-16;
  int iters = 0, pos = 0, nsw = 0;
  bool converged = true, overflow = false;
  for (int l = 0; l < m && !overflow; ++l) {
    int it = 0;
    for (;;) {
      // first index mm >= l with a negligible e_mm (m - 1 counts as one)
      int mm = m - 1;
      for (int b0 = l; b0 < m - 1; b0 += 64) {
        const int ix = b0 + lane;
        const bool t = ix < m - 1 && fabs(ev[ix]) <= eps * (fabs(dv[ix]) + fabs(dv[ix + 1]));
        const unsigned long long mk = __ballot(t);
        if (mk) {
          mm = b0 + __ffsll((long long)mk) - 1;
          break;
        }
      }
      if (mm == l) break;
      if (++it > kQlMaxIter) { converged = false; break; }
      if (pos + 1 + (mm - l) > cap) { overflow = true; break; }
      ++iters;
      const double dL = dv[l], eL = ev[l];
      double g = (dv[l + 1] - dL) / (2.0 * eL);
      double r = sqrt(g * g + 1.0);
      g = dv[mm] - dL + eL / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, pp = 0.0;
      const int hdr = pos++;
      int nrot = 0;
      bool split = false;
      double ei = ev[mm - 1], di = dv[mm - 1], di1 = dv[mm];
      // the rotations in blocks of eight, the block's entries i - 1 .. i - 8 (not rewritten
      // by this sweep before their rotation) read together
      for (int i = mm - 1; i >= l && !split;) {
        double eb[8], db[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int ix = max(i - 1 - q, 0);  // (unused below index 0)
          eb[q] = ev[ix];
          db[q] = dv[ix];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q, --i) {
          if (i < l) break;
          const double f = sn * ei, b = cs * ei;
          const double x = f * f + g * g;
          if (x == 0.0) {  // exact deflation: the chase stops here
            if (lane == 0) {
              ev[i + 1] = 0.0;
              dv[i + 1] = di1 - pp;
              ev[mm] = 0.0;
            }
            split = true;
            break;
          }
          const double y = nyls_rsqrt(x);
          sn = f * y;
          cs = g * y;
          g = di1 - pp;
          r = (di - g) * sn + 2.0 * cs * b;
          pp = sn * r;
          if (lane == 0) {
            ev[i + 1] = x * y;
            dv[i + 1] = g + pp;
            lg[2 * pos] = cs;
            lg[2 * pos + 1] = sn;
          }
          g = cs * r - b;
          ++pos;
          ++nrot;
          di1 = di;
          di = db[q];
          ei = eb[q];
        }
      }
      if (lane == 0) {
        lg[2 * hdr] = (double)mm;
        lg[2 * hdr + 1] = (double)nrot;
        if (!split) {
          dv[l] -= pp;
          ev[l] = g;
          ev[mm] = 0.0;
        }
      }
      ++nsw;
      nyls_wave_lds_sync();
    }
  }
  for (int k = lane; k < m; k += 64) ws[L.lam + k] = dv[k];
  if (lane == 0) {
    ws[L.info + 2] = (double)iters;
    ws[L.info + 6] = (double)nsw;
    ws[L.info + 7] = overflow ? 2.0 : (converged ? 0.0 : 1.0);
  }
}

// 4. replay: workgroup (instance, y) carries rows 64 y .. 64 y + 63 of Z, lane l row 64 y + l,
// in LDS (Zs[c * 64 + l] = Z[64 y + l][c]).  The log (each sweep: header (mm, k) and k
// rotations (c, s) for columns mm - 1, mm - 2, ...) is read in windows of 64 entries, one per
// lane, the next window loaded while the current one is used; an entry comes to every lane
// with a lane read.  Rotation i writes column i + 1 and reads column i, which no earlier
// rotation of the sweep has rewritten, so the reads of eight rotations are issued together.
// One wavefront per workgroup: no barriers.
__global__ __launch_bounds__(64) void k_eig_wide_replay(const nyls_desc* __restrict__ desc,
                                                        double* __restrict__ wsbase, int lo, int hi) {
  extern __shared__ double sm[];
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m;
  if (m <= lo || m > hi) return;  // (the LDS holds hi columns)
  const int r0 = (int)blockIdx.y * kWideRows;
  if (r0 >= m) return;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  if ((int)ws[L.info + 7] == 2) return;  // log overflow: flagged in WIDE_FINISH
  const int lane = threadIdx.x;
  const int row = r0 + lane;
  const bool own = row < m;
  double* Zs = sm;  // [m][64]
  double* ZT = ws + L.tmp;
  for (int c = 0; c < m; ++c) Zs[c * kWideRows + lane] = own ? ZT[c * m + row] : 0.0;
  const double* lg = ws + L.log;
  const int cap = (int)((L.aux - L.log) / 2);
  const int nsw = (int)ws[L.info + 6];
  auto ld = [&](int e, double& a, double& b) {
    a = e < cap ? lg[2 * e] : 0.0;
    b = e < cap ? lg[2 * e + 1] : 0.0;
  };
  int wb = 0;  // first entry of the current window
  double ca, cb, na, nb;
  ld(lane, ca, cb);
  ld(64 + lane, na, nb);
  auto get = [&](int e, double& a, double& b) {  // e wave-uniform, never decreasing
    while (e >= wb + 64) {
      ca = na;
      cb = nb;
      wb += 64;
      ld(wb + 64 + lane, na, nb);
    }
    a = nyls_rdlane(ca, e - wb);
    b = nyls_rdlane(cb, e - wb);
  };
  int hdr = 0;
  for (int sw = 0; sw < nsw; ++sw) {
    double hm, hn;
    get(hdr, hm, hn);
    const int mm = (int)hm, nrot = (int)hn;
    double c0 = Zs[mm * kWideRows + lane];
    int k = 0;
    // blocks of eight rotations: their eight Z entries (columns mm - 1 - k .. mm - 8 - k, not
    // yet rewritten in this sweep) are loaded together before the block's stores
    for (; k + 8 <= nrot; k += 8) {
      double zb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) zb[u] = Zs[(mm - 1 - k - u) * kWideRows + lane];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        double cs, sn;
        get(hdr + 1 + k + u, cs, sn);
        Zs[(mm - k - u) * kWideRows + lane] = sn * zb[u] + cs * c0;
        c0 = cs * zb[u] - sn * c0;
      }
    }
    for (; k < nrot; ++k) {
      double cs, sn;
      get(hdr + 1 + k, cs, sn);
      const double z0 = Zs[(mm - 1 - k) * kWideRows + lane];
      Zs[(mm - k) * kWideRows + lane] = sn * z0 + cs * c0;
      c0 = cs * z0 - sn * c0;
    }
    Zs[(mm - nrot) * kWideRows + lane] = c0;
    hdr += 1 + nrot;
  }
  if (own)
    for (int c = 0; c < m; ++c) ZT[c * m + row] = Zs[c * kWideRows + lane];
}

}  // namespace

hipError_t nyls_launch_eig(const nyls_plan_view& pv, double* ws, int single, hipStream_t st,
                           int parts) {
  if ((parts & NYLS_EIG_NARROW) && (pv.nb_mask & (4 | 16))) {  // some instance has m <= 64
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
      hipLaunchKernelGGL(k_ql_lanes<kQlMaxM>, dim3((pv.batch + ipw - 1) / ipw), dim3(64), 0, st,
                         pv.d_desc, ws, pv.batch, ipw);
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_REPLAY);
      hipLaunchKernelGGL(k_eig_ql, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                         (int)QL_REDO);
    }
  }
  if (!(parts & NYLS_EIG_BIG)) return hipGetLastError();
  if (pv.nb_mask & (1u << 16)) {  // wide bases (never in single-instance launches)
    const int lo = NYLS_NARROW_MAX_M;
    hipLaunchKernelGGL(k_eig_wide, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, (int)WIDE_REDUCE, lo, NYLS_MAX_M, 0);
    hipLaunchKernelGGL(k_ql_wide, dim3(pv.batch), dim3(64), 0, st, pv.d_desc, ws);
    const size_t lds = (size_t)pv.maxm * kWideRows * sizeof(double);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_wide_replay),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_eig_wide_replay, dim3(pv.batch, (pv.maxm + kWideRows - 1) / kWideRows), dim3(64),
                       lds, st, pv.d_desc, ws, lo, NYLS_MAX_M);
    hipLaunchKernelGGL(k_eig_wide, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, (int)WIDE_FINISH, lo,
                       NYLS_MAX_M, 0);
  }
  if (!(pv.nb_mask & 256)) return hipGetLastError();
  // 64 < m <= 128: one wavefront per instance, two rows per lane.  With many such instances
  // the QL is staged like the m <= 64 path (the lane-parallel QL takes up to 64 instances
  // per wavefront); a few run it inside their own wavefront, where all lanes share the
  // scalar chain instead of one lane carrying it.
  const int lda = pv.maxm_narrow | 1;
  const size_t lds = (size_t)lda * lda * sizeof(double) + 3 * 128 * sizeof(double) + 128 * sizeof(int);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_ql2),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const dim3 grid(single >= 0 ? 1 : pv.batch);
  if (single >= 0 || pv.eig_ql || pv.n_big < kQlStagedMin) {
    hipLaunchKernelGGL(k_eig_ql2, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                       (int)QL_FULL);
  } else {
    // staged through the workspace: the reduction by 256 threads per instance (K_mm in the
    // workspace, many instances per CU), the lane-parallel QL, the replay on rows of Z held in
    // LDS by two workgroups per instance and the ordering; instances whose rotation log
    // overflowed are redone by the one-wave kernel
    const int ipw = pv.ql_lanes >= 1 && pv.ql_lanes <= kQlLaneInst ? pv.ql_lanes : kQlLaneInst;
    const int lo = kQlMaxM;
    hipLaunchKernelGGL(k_eig_wide, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, (int)WIDE_REDUCE, lo, 2 * kQlMaxM, 1);
    hipLaunchKernelGGL(k_ql_lanes<2 * kQlMaxM>, dim3((pv.batch + ipw - 1) / ipw), dim3(64), 0, st,
                       pv.d_desc, ws, pv.batch, ipw);
    const int mr = pv.maxm_narrow;
    const size_t rl = (size_t)mr * kWideRows * sizeof(double);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_wide_replay),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)rl);
    hipLaunchKernelGGL(k_eig_wide_replay, dim3(pv.batch, (mr + kWideRows - 1) / kWideRows), dim3(64), rl, st,
                       pv.d_desc, ws, lo, 2 * kQlMaxM);
    hipLaunchKernelGGL(k_eig_wide, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, (int)WIDE_FINISH, lo,
                       2 * kQlMaxM, 1);
    hipLaunchKernelGGL(k_eig_ql2, grid, dim3(64), lds, st, pv.d_desc, pv.d_order, ws, single, lda,
                       (int)QL_REDO);
  }
  return hipGetLastError();
}
