// Lemma 2 Newton iteration for second-order nonlinear ODEs y'' = F(t, y, y') (Sec. 3.2, and
// the appendix section on Problem 15), one workgroup per instance.
//
// Unknowns x = (omega, b, lambda_1, lambda_2, y_i), i in the residual set I (grid points
// without a condition).  y enters F through the auxiliary unknown y_i, y' through the model,
// u_i = omega^T phi'(t_i).  With alpha = W omega, k^(d)_i = d^d/dt^d k_m(t_i) (kernel space),
// rho_i = alpha^T k''_i - F_i, eta_i = y_i - alpha^T k_i - b, F_0 = dF/dy, F_1 = dF/dy' and
// F_ab the second derivatives:
//   kappa_i  = k''_i - F_1,i k'_i                         (d rho_i / d alpha)
//   Y_omega  = omega + W^T gamma sum (rho_i kappa_i - eta_i k_i) + H lambda
//   Y_b      = -gamma sum eta_i + delta^T lambda,  Y_lambda_j = h_j^T omega + delta_j b - v_j
//   Y_y,i    = gamma (-rho_i F_0,i + eta_i)
//   J_zz     = I + W^T gamma sum (kappa kappa^T + k k^T - rho F_11 k' k'^T) W, ...,
//   J_z,y_i  = c_i = -gamma (W^T kt_i, 1, 0),  kt_i = F_0,i kappa_i + rho_i F_01,i k'_i + k_i
//   J_yy     = diag(d_i),  d_i = gamma (1 + F_0,i^2 - rho_i F_00,i).
// A step eliminates the diagonal block: (J_zz - sum c_i c_i^T / d_i) dz = Y_z - sum c_i Y_y,i
// / d_i, dy_i = (Y_y,i - c_i^T dz) / d_i, x <- x - dx.  Unlike the first-order case every
// block depends on the iterate (kappa_i through F_1), so the whole weighted Gram is formed
// each step: per point the rows (W^T kappa_i | 0 | 0), (W^T k_i | 1 | 0), (W^T k'_i | 0 | 0)
// and (W^T kt_i | 1 | Y_y,i / gamma) with weights gamma, gamma, -gamma rho_i F_11,i and
// -gamma^2 / d_i, accumulated in feature space.  Passing zero second derivatives gives the
// Gauss-Newton step.
#include "nyls_dense.h"
#include "nyls_gramacc.h"

struct nyls_plan;
int64_t nyls_plan_newton_stride(const nyls_plan* pl);
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl);

namespace {

constexpr int TP = 8;      // points per tile
constexpr int CH = 4;      // points per thread in the Gaussian recurrence
constexpr int NR = 4;      // Gram rows per point
constexpr int P = 2;       // ODE order of this kernel

__host__ __device__ inline int round4(int x) { return (x + 3) & ~3; }

// Starting point and condition rows: omega = 0, lambda = 0, b = y_i = the value of the first
// condition on y itself (0 without one); h_j = W^T k^(d_j)(t_{i_j}) -> ws[H + j m].
__global__ __launch_bounds__(NYLS_BLOCK) void k_newton2_init(const nyls_desc* __restrict__ desc,
                                                             double* __restrict__ wsbase,
                                                             double* __restrict__ x, int64_t xs,
                                                             int maxm, int maxp) {
  __shared__ double kc[NYLS_MAX_P][NYLS_NARROW_MAX_M];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double inv_sigma = 1.0 / d.sigma;
  for (int e = tid; e < d.p * m; e += NYLS_BLOCK) {
    const int j = e / m, s = e - j * m;
    const double z = (nyls_grid_t(d, d.cond_i[j]) - nyls_grid_t(d, d.lidx[s])) * inv_sigma;
    double kd[NYLS_MAX_P + 1];
    nyls_kderiv(z, inv_sigma, kd);
    kc[j][s] = nyls_pick(kd, d.cond_d[j]);
  }
  __syncthreads();
  const double* W = ws + L.W;
  for (int e = tid; e < d.p * m; e += NYLS_BLOCK) {
    const int j = e / m, k = e - j * m;
    double acc = 0.0;
    if (k < r)
      for (int s = 0; s < m; ++s) acc += W[s * m + k] * kc[j][s];
    ws[L.H + j * m + k] = acc;
  }
  double b0 = 0.0;
  for (int j = d.p - 1; j >= 0; --j)
    if (d.cond_d[j] == 0) b0 = d.v[j];
  double* xi = x + (size_t)inst * xs;
  const int xoff = maxm + 1 + maxp;
  for (int k = tid; k < maxm + 1 + maxp; k += NYLS_BLOCK) xi[k] = (k == maxm) ? b0 : 0.0;
  for (int i = tid; i < n; i += NYLS_BLOCK) xi[xoff + i] = b0;
  for (int s = tid; s < m; s += NYLS_BLOCK) ws[L.alpha + s] = 0.0;
  if (tid == 0) ws[L.x + m] = b0;
}

// State values the caller evaluates F at: u[0][i] = y_i (y_hat at condition points),
// u[d][i] = alpha^T k^(d)(t_i) = y_hat^(d)(t_i) for d = 1..p-1; u is [p][total points].
__global__ __launch_bounds__(NYLS_BLOCK) void k_newton_state(const nyls_desc* __restrict__ desc,
                                                             const double* __restrict__ wsbase,
                                                             const double* __restrict__ x,
                                                             int64_t xs, int maxm, int maxp,
                                                             double* __restrict__ u, int64_t total) {
  __shared__ double al[NYLS_NARROW_MAX_M], tl[NYLS_NARROW_MAX_M];
  const nyls_desc& d = desc[blockIdx.y];
  const int m = d.m, n = d.n;
  const nyls_wsl L = nyls_layout(m, d.p, 0);
  const double* ws = wsbase + d.ws;
  for (int s = threadIdx.x; s < m; s += NYLS_BLOCK) {
    al[s] = ws[L.alpha + s];
    tl[s] = nyls_grid_t(d, d.lidx[s]);
  }
  __syncthreads();
  const double* xi = x + (size_t)blockIdx.y * xs;
  const double inv_sigma = 1.0 / d.sigma, b = xi[maxm];
  for (int i = blockIdx.x * NYLS_BLOCK + threadIdx.x; i < n; i += gridDim.x * NYLS_BLOCK) {
    const double ti = nyls_grid_t(d, i);
    double acc[NYLS_MAX_P] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < m; ++s) {
      double kd[NYLS_MAX_P + 1];
      nyls_kderiv((ti - tl[s]) * inv_sigma, inv_sigma, kd);
#pragma unroll
      for (int q = 0; q < NYLS_MAX_P; ++q) acc[q] += al[s] * kd[q];
    }
    const bool cp = nyls_is_condition_point(d, i);
    u[d.goff + i] = cp ? acc[0] + b : xi[maxm + 1 + maxp + i];
    for (int q = 1; q < d.p; ++q) u[(int64_t)q * total + d.goff + i] = acc[q];
  }
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_newton2_step(
    const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, const double* __restrict__ Fv,
    const double* __restrict__ dFv, const double* __restrict__ d2Fv, double* __restrict__ x,
    int64_t xs, double* __restrict__ step_inf, int32_t* __restrict__ status, int maxm, int maxp,
    int64_t total) {
  extern __shared__ double sm[];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n;
  const nyls_wsl L = nyls_layout(m, P, 0);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const int g = r + 2, gp = round4(g);  // feature-space Gram columns: phi (r), b, rhs
  const double gam = d.gamma, inv_sigma = 1.0 / d.sigma;
  double* xi = x + (size_t)inst * xs;
  const int xoff = maxm + 1 + maxp;
  const int64_t go = d.goff;

  // common LDS
  double* tl = sm;                        // [128] landmark times
  double* al = tl + NYLS_NARROW_MAX_M;           // [128] alpha
  double* dal = al + NYLS_NARROW_MAX_M;          // [128] W d omega
  double* lin = dal + NYLS_NARROW_MAX_M;         // [128] sum rho q - eta phi (feature space)
  double* part = lin + NYLS_NARROW_MAX_M;        // [256] partial sums
  double* red = part + NYLS_BLOCK;        // [16]
  double* rhs = red + 16;                 // [136]
  double* pd = rhs + 136;                 // [TP][8] per-point data
  int* piv = reinterpret_cast<int*>(pd + TP * 8);  // [136]
  double* big = reinterpret_cast<double*>(piv + 136);
  // tile region
  double* K = big;                        // [3][TP][maxm]  k, k', k''  (kernel space)
  double* Fz = K + 3 * TP * maxm;         // [3][TP][maxm]  phi, phi', phi''  (first r used)
  double* Q = Fz + 3 * TP * maxm;         // [NR * TP][gp]  (also the Gram reduction buffer)
  double* wr = Q + NR * TP * round4(maxm + 2);  // [NR * TP]

  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * xi[k];
    al[s] = acc;
  }
  __syncthreads();
  const double b = xi[maxm];

  // The Jacobian blocks are accumulated in feature space (rows phi^(d)_i = W^T k^(d)_i): in
  // kernel space their rounding would reach the step through W twice, amplified by
  // lambda_1 / lambda_r, and the Schur subtraction cancels most of the omega block.
  nyls_gram::Acc A;
  nyls_gram::setup(A, gp);
  double linacc = 0.0, etasum = 0.0;
  int bad = 0;
  const int ngc = NYLS_BLOCK / (r > 0 ? r : 1), cs = tid % (r > 0 ? r : 1), cg = tid / (r > 0 ? r : 1);
  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double z, double ev) {
      // k, k' = -2 z / sigma e, k'' = (4 z^2 - 2) / sigma^2 e
      K[(0 * TP + pt) * maxm + s] = ev;
      K[(1 * TP + pt) * maxm + s] = -2.0 * z * inv_sigma * ev;
      K[(2 * TP + pt) * maxm + s] = (4.0 * z * z - 2.0) * inv_sigma * inv_sigma * ev;
    });
    __syncthreads();
    for (int e = tid; e < 3 * TP * r; e += NYLS_BLOCK) {
      const int row = e / r, k = e - row * r;
      const double* kr = K + row * maxm;
      double acc = 0.0;
      for (int s = 0; s < m; ++s) acc += kr[s] * W[s * m + k];
      Fz[row * maxm + k] = acc;
    }
    __syncthreads();
    {
      constexpr int TPG = NYLS_BLOCK / TP;
      const int pt = tid / TPG, sub = tid % TPG;
      double d0 = 0.0, d2 = 0.0;
      for (int k = sub; k < r; k += TPG) {
        d0 += Fz[(0 * TP + pt) * maxm + k] * xi[k];
        d2 += Fz[(2 * TP + pt) * maxm + k] * xi[k];
      }
      for (int o = TPG / 2; o > 0; o >>= 1) {
        d0 += __shfl_xor(d0, o);
        d2 += __shfl_xor(d2, o);
      }
      if (sub == 0) {
        const int i = i0 + pt;
        const bool ok = i < n && !nyls_is_condition_point(d, i);
        double rho = 0.0, eta = 0.0, yy = 0.0, dd = 1.0, f0 = 0.0, f1 = 0.0, f01 = 0.0, f11 = 0.0;
        if (ok) {
          f0 = dFv[go + i];
          f1 = dFv[total + go + i];
          const double f00 = d2Fv[go + i];
          f01 = d2Fv[total + go + i];
          f11 = d2Fv[3 * total + go + i];
          rho = d2 - Fv[go + i];
          eta = xi[xoff + i] - d0 - b;
          yy = gam * (-rho * f0 + eta);
          dd = gam * (1.0 + f0 * f0 - rho * f00);
          if (!(fabs(dd) >= 1e-10 * gam)) bad |= 1;
          etasum += eta;
        }
        const bool use = ok && dd != 0.0 && dd == dd;
        pd[pt * 8 + 0] = ok ? rho : 0.0;
        pd[pt * 8 + 1] = ok ? eta : 0.0;
        pd[pt * 8 + 2] = f0;
        pd[pt * 8 + 3] = f1;
        pd[pt * 8 + 4] = rho * f01;
        pd[pt * 8 + 5] = yy;
        wr[NR * pt + 0] = ok ? gam : 0.0;
        wr[NR * pt + 1] = ok ? gam : 0.0;
        wr[NR * pt + 2] = ok ? -gam * rho * f11 : 0.0;
        wr[NR * pt + 3] = use ? -gam * gam / dd : 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < NR * TP * gp; e += NYLS_BLOCK) {
      const int row = e / gp, a = e - row * gp;
      const int pt = row / NR, kind = row - pt * NR;
      double v = 0.0;
      if (wr[row] != 0.0) {
        if (a < r) {
          const double p0 = Fz[(0 * TP + pt) * maxm + a], p1 = Fz[(1 * TP + pt) * maxm + a];
          const double p2 = Fz[(2 * TP + pt) * maxm + a];
          const double qv = p2 - pd[pt * 8 + 3] * p1;
          v = kind == 0 ? qv
            : kind == 1 ? p0
            : kind == 2 ? p1
            : pd[pt * 8 + 2] * qv + pd[pt * 8 + 4] * p1 + p0;
        } else if (a == r) {
          v = (kind == 1 || kind == 3) ? 1.0 : 0.0;
        } else if (a == r + 1) {
          v = kind == 3 ? pd[pt * 8 + 5] / gam : 0.0;
        }
      }
      Q[row * gp + a] = v;
    }
    if (r > 0 && cg < ngc)
      for (int pt = cg; pt < TP; pt += ngc) {
        const double qv = Fz[(2 * TP + pt) * maxm + cs] - pd[pt * 8 + 3] * Fz[(1 * TP + pt) * maxm + cs];
        linacc += pd[pt * 8 + 0] * qv - pd[pt * 8 + 1] * Fz[(0 * TP + pt) * maxm + cs];
      }
    __syncthreads();
    nyls_gram::accumulate(A, Q, gp, wr, NR * TP);
  }
  double* Sw = ws + L.gram;  // weighted Gram (feature space), g x g
  nyls_gram::finish(A, Q, Sw, g, g);
  part[tid] = (r > 0 && cg < ngc) ? linacc : 0.0;
  const double esum = nyls_block_sum(etasum, red);
  const double badf = nyls_block_sum((double)bad, red);
  __syncthreads();
  for (int k = tid; k < r; k += NYLS_BLOCK) {
    double acc = 0.0;
    for (int gi = 0; gi < ngc; ++gi) acc += part[gi * r + k];
    lin[k] = acc;
  }
  __syncthreads();

  // Schur system in (omega padded to m, b, lambda_1, lambda_2): N2 = m + 1 + P; the
  // directions k >= r of omega are identity rows.
  const int N2 = m + 1 + P, lz = N2 + 1;
  double* Z = big;
  const double* Hc = ws + L.H;
  for (int e = tid; e < N2 * N2; e += NYLS_BLOCK) {
    const int a = e / N2, c = e - a * N2;
    double val = 0.0;
    if (a < m && c < m) {
      val = (a < r && c < r) ? Sw[a * g + c] + (a == c ? 1.0 : 0.0) : (a == c ? 1.0 : 0.0);
    } else if (a < m || c < m) {
      const int k = a < m ? a : c, o = a < m ? c : a;
      if (k < r) val = (o == m) ? Sw[k * g + r] : Hc[(o - m - 1) * m + k];
    } else if (a == m && c == m) {
      val = Sw[r * g + r];
    } else if (a == m || c == m) {
      const int j = (a == m ? c : a) - m - 1;
      val = d.cond_d[j] == 0 ? 1.0 : 0.0;
    }
    Z[a * lz + c] = val;
  }
  for (int a = tid; a < N2; a += NYLS_BLOCK) {
    double val = 0.0;
    if (a < m) {
      if (a < r) {
        val = xi[a] + gam * lin[a] - Sw[a * g + r + 1];
        for (int j = 0; j < P; ++j) val += Hc[j * m + a] * xi[maxm + 1 + j];
      }
    } else if (a == m) {
      val = -gam * esum - Sw[r * g + r + 1];
      for (int j = 0; j < P; ++j) val += (d.cond_d[j] == 0 ? 1.0 : 0.0) * xi[maxm + 1 + j];
    } else {
      const int j = a - m - 1;
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc += Hc[j * m + k] * xi[k];
      val = acc + (d.cond_d[j] == 0 ? b : 0.0) - d.v[j];
    }
    rhs[a] = val;
  }
  __syncthreads();
  const int sing = nyls_lu(Z, lz, N2, piv, red);
  nyls_lu_solve(Z, lz, N2, piv, rhs);  // rhs <- dz
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * rhs[k];
    dal[s] = acc;
  }
  __syncthreads();
  // dy_i = (Y_y,i - c_i^T dz) / d_i = (Y_y,i + gamma (kt_i^T dalpha + db)) / d_i
  const double db = rhs[m];
  double dmax = 0.0;
  for (int i = tid; i < n; i += NYLS_BLOCK) {
    if (nyls_is_condition_point(d, i)) continue;
    const double ti = nyls_grid_t(d, i);
    const double f0 = dFv[go + i], f1 = dFv[total + go + i];
    double u0 = 0.0, u2 = 0.0, k0d = 0.0, k1d = 0.0, k2d = 0.0;
    for (int s = 0; s < m; ++s) {
      const double z = (ti - tl[s]) * inv_sigma;
      const double e0 = exp(-z * z);
      const double e1 = -2.0 * z * inv_sigma * e0;
      const double e2 = (4.0 * z * z - 2.0) * inv_sigma * inv_sigma * e0;
      u0 += e0 * al[s];
      u2 += e2 * al[s];
      k0d += e0 * dal[s];
      k1d += e1 * dal[s];
      k2d += e2 * dal[s];
    }
    const double rho = u2 - Fv[go + i];
    const double eta = xi[xoff + i] - u0 - b;
    const double yy = gam * (-rho * f0 + eta);
    const double dd = gam * (1.0 + f0 * f0 - rho * d2Fv[go + i]);
    const double ktd = f0 * (k2d - f1 * k1d) + rho * d2Fv[total + go + i] * k1d + k0d;
    const double dy = (dd != 0.0 && dd == dd) ? (yy + gam * (ktd + db)) / dd : 0.0;
    xi[xoff + i] -= dy;
    dmax = fmax(dmax, fabs(dy));
  }
  for (int a = tid; a < N2; a += NYLS_BLOCK) dmax = fmax(dmax, fabs(rhs[a]));
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < NYLS_BLOCK / 64; ++w) mx = fmax(mx, red[w]);
    if (step_inf) step_inf[inst] = mx;
  }
  // x <- x - dz ; alpha and b for nyls_predict / nyls_newton_state
  for (int k = tid; k < m; k += NYLS_BLOCK) xi[k] -= rhs[k];
  __syncthreads();
  for (int s = tid; s < m; s += NYLS_BLOCK) ws[L.alpha + s] = al[s] - dal[s];
  if (tid == 0) {
    xi[maxm] = b - db;
    for (int j = 0; j < P; ++j) xi[maxm + 1 + j] -= rhs[m + 1 + j];
    ws[L.x + m] = b - db;
    int bits = (int)ws[L.info + 1];
    if (badf > 0) bits |= NYLS_S_SMALL_PIVOT;
    if (sing) bits |= NYLS_S_SINGULAR;
    if (!(fabs(b - db) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    if (status) status[inst] = bits;
  }
}

}  // namespace

size_t nyls_newton2_lds_bytes(int maxm) {
  const size_t common = (4 * NYLS_NARROW_MAX_M + NYLS_BLOCK + 16 + 136 + TP * 8) * sizeof(double) +
                        136 * sizeof(int);
  const int gp = round4(maxm + 2);
  const size_t qrows = (size_t)NR * TP;
  size_t tile = (6 * (size_t)TP * maxm + qrows * gp + qrows) * sizeof(double);
  const size_t redb = (size_t)nyls_gram::red_doubles(gp) * sizeof(double);
  const size_t qoff = 6 * (size_t)TP * maxm * sizeof(double);
  if (qoff + redb > tile) tile = qoff + redb;
  const size_t schur = (size_t)(maxm + 1 + P) * (maxm + 2 + P) * sizeof(double);
  return common + (tile > schur ? tile : schur);
}

hipError_t nyls_launch_newton2_init(const nyls_plan_view& pv, double* ws, double* x, int64_t xs,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_newton2_init, dim3(pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, x, xs,
                     pv.maxm, pv.maxp);
  return hipGetLastError();
}

hipError_t nyls_launch_newton_state(const nyls_plan_view& pv, const double* ws, const double* x,
                                    int64_t xs, double* u, hipStream_t st) {
  int gx = (pv.maxn + NYLS_BLOCK - 1) / NYLS_BLOCK;
  gx = gx > 64 ? 64 : gx;
  hipLaunchKernelGGL(k_newton_state, dim3(gx, pv.batch), dim3(NYLS_BLOCK), 0, st, pv.d_desc, ws, x,
                     xs, pv.maxm, pv.maxp, u, pv.total);
  return hipGetLastError();
}

hipError_t nyls_launch_newton2_step(const nyls_plan_view& pv, double* ws, const double* F,
                                    const double* dF, const double* d2F, double* x, int64_t xs,
                                    double* step_inf, int32_t* status, hipStream_t st) {
  const size_t lds = nyls_newton2_lds_bytes(pv.maxm);
  const hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_newton2_step),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (ea != hipSuccess) return ea;
  hipLaunchKernelGGL(k_newton2_step, dim3(pv.batch), dim3(NYLS_BLOCK), lds, st, pv.d_desc, ws, F, dF,
                     d2F, x, xs, step_inf, status, pv.maxm, pv.maxp, pv.total);
  return hipGetLastError();
}
