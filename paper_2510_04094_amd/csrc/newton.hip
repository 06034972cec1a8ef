// Lemma 2 Newton iteration for first-order nonlinear ODEs y' = F(t, y) (Sec. 3.2,
// App. A.5), one workgroup per instance.
//
// Unknowns x = (omega, b, lambda, y_i), i in the residual set I.  With alpha = W omega,
// rho_i = k'_i^T alpha - F_i and eta_i = y_i - k_i^T alpha - b (k_i = k_m(t_i), k'_i its
// time derivative), the KKT residual Y = grad L and the Hessian J of App. A.5 are
//   Y1 = omega + gamma W^T sum (rho_i k'_i - eta_i k_i) + lambda phi_1
//   Y2 = -gamma sum eta_i + lambda,   Y3 = phi_1^T omega + b - v
//   Y4_i = gamma (-rho_i Fy_i + eta_i)
//   J_zz = [[I + gamma W^T (sum k'k'^T + sum kk^T) W, gamma W^T sum k_i, phi_1],
//           [.., gamma |I|, 1], [phi_1^T, 1, 0]]             (constant: built once)
//   J_zy_i = q_i = -gamma (W^T kappa_i, 1, 0),  kappa_i = Fy_i k'_i + k_i
//   J_yy = diag(d_i),  d_i = gamma (1 + Fy_i^2 - rho_i Fyy_i).
// A step eliminates the diagonal block: (J_zz - sum q_i q_i^T / d_i) dz =
// Y_z - sum q_i Y4_i / d_i, then dy_i = (Y4_i - q_i^T dz) / d_i, and x <- x - dx.
// The weighted sum over points is accumulated in kernel space as the Gram of
// (kappa_i, 1, Y4_i / gamma) with weights gamma^2 / d_i, then mapped through W.
// Points whose pivot is tiny (|d_i| < 1e-10 gamma; d_i can pass through zero at early
// iterates) are not divided out: up to kKeep of them stay in the system as unknowns,
//   [[J_zz - sum_good q q^T / d, Q_B], [Q_B^T, D_B]] [dz; dy_B] = [Y_z - sum_good q Y4 / d; Y4_B],
// which is the same Newton step without the division, solved by dense LU in the
// workspace.  More such points than kKeep set NYLS_S_PIVOT_OVERFLOW and are divided out.
#include "nyls_dense.h"
#include "nyls_gramacc.h"

struct nyls_plan;
int64_t nyls_plan_newton_stride(const nyls_plan* pl);
bool nyls_plan_first_order(const nyls_plan* pl);
int nyls_plan_common_order(const nyls_plan* pl);
nyls_plan_view nyls_plan_get_view(const nyls_plan* pl);
// second-order nonlinear path (newton_gen.hip)
hipError_t nyls_launch_newton2_init(const nyls_plan_view& pv, double* ws, double* x, int64_t xs,
                                    hipStream_t st);
hipError_t nyls_launch_newton_state(const nyls_plan_view& pv, const double* ws, const double* x,
                                    int64_t xs, double* u, hipStream_t st);
hipError_t nyls_launch_newton2_step(const nyls_plan_view& pv, double* ws, const double* F,
                                    const double* dF, const double* d2F, double* x, int64_t xs,
                                    double* step_inf, int32_t* status, hipStream_t st);

namespace {

constexpr int TP = 32;
constexpr int CH = 8;  // points per thread in the Gaussian recurrence
constexpr int kKeep = 32;  // small-pivot points kept in the dense system per step
constexpr int kNz = NYLS_NARROW_MAX_M + 2 + kKeep;  // largest dense system

__host__ __device__ inline int round4(int x) { return (x + 3) & ~3; }

// Constant blocks (kernel space, g x g in aux[0 .. g*g)):
//   C0 = [[sum k'k'^T + sum kk^T, sum k], [sum k^T, |I|]]   (rows (k'_i, 0) and (k_i, 1))
// phi_1 = W^T k_m(t_cond) -> ws[H]; starting point into x.
__global__ __launch_bounds__(NYLS_BLOCK) void k_newton_init(const nyls_desc* __restrict__ desc,
                                                            double* __restrict__ wsbase,
                                                            double* __restrict__ x, int64_t xs,
                                                            int maxm) {
  extern __shared__ double sm[];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n, g = m + 2, gp = round4(g);
  const nyls_wsl L = nyls_layout(m, d.p, 1);
  double* ws = wsbase + d.ws;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double inv_sigma = 1.0 / d.sigma;
  double* tl = sm;                          // [128]
  double* kc = tl + NYLS_NARROW_MAX_M;             // [128]
  double* okf = kc + NYLS_NARROW_MAX_M;            // [TP]
  double* Q = okf + TP;                     // [2*TP][gp], later the reduction buffer
  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  __syncthreads();
  nyls_gram::Acc A;
  nyls_gram::setup(A, gp);
  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    // rows (k_i, 1) and (k'_i, 0); zero rows at condition points and past the grid
    for (int e = tid; e < TP; e += NYLS_BLOCK) {
      const int i = i0 + e;
      const bool ok = i < n && !nyls_is_condition_point(d, i);
      okf[e] = ok ? 1.0 : 0.0;
      for (int c = m; c < gp; ++c) {
        Q[(2 * e) * gp + c] = (c == m && ok) ? 1.0 : 0.0;
        Q[(2 * e + 1) * gp + c] = 0.0;
      }
    }
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double z, double ev) {
      const double e0 = okf[pt] * ev;
      Q[(2 * pt) * gp + s] = e0;
      Q[(2 * pt + 1) * gp + s] = -2.0 * z * inv_sigma * e0;
    });
    __syncthreads();
    nyls_gram::accumulate(A, Q, gp, nullptr, 2 * TP);
  }
  nyls_gram::finish(A, Q, ws + L.aux, g, g);
  // phi_1 = W^T k_m(t_{i_1})
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    const double z = (nyls_grid_t(d, d.cond_i[0]) - tl[s]) * inv_sigma;
    kc[s] = exp(-z * z);
  }
  __syncthreads();
  const double* W = ws + L.W;
  for (int k = tid; k < m; k += NYLS_BLOCK) {
    double acc = 0.0;
    if (k < r)
      for (int s = 0; s < m; ++s) acc += W[s * m + k] * kc[s];
    ws[L.H + k] = acc;
  }
  const double v = d.v[0];
  double* xi = x + (size_t)inst * xs;
  for (int k = tid; k < maxm; k += NYLS_BLOCK) xi[k] = 0.0;
  for (int i = tid; i < n; i += NYLS_BLOCK) xi[maxm + 2 + i] = v;
  for (int s = tid; s < m; s += NYLS_BLOCK) ws[L.alpha + s] = 0.0;
  if (tid == 0) {
    xi[maxm] = v;
    xi[maxm + 1] = 0.0;
    ws[L.x + m] = v;
  }
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_newton_step(
    const nyls_desc* __restrict__ desc, double* __restrict__ wsbase, const double* __restrict__ Fv,
    const double* __restrict__ Fyv, const double* __restrict__ Fyyv, double* __restrict__ x,
    int64_t xs, double* __restrict__ step_inf, int32_t* __restrict__ status, int maxm) {
  extern __shared__ double sm[];
  const int inst = blockIdx.x;
  const nyls_desc& d = desc[inst];
  const int m = d.m, n = d.n, g = m + 2, gp = round4(g);
  const nyls_wsl L = nyls_layout(m, d.p, 1);
  double* ws = wsbase + d.ws;
  const double* W = ws + L.W;
  const int tid = threadIdx.x;
  const int r = (int)ws[L.info + 0];
  const double gam = d.gamma, inv_sigma = 1.0 / d.sigma;
  double* xi = x + (size_t)inst * xs;
  const double* F = Fv + d.goff;
  const double* Fy = Fyv + d.goff;
  const double* Fyy = Fyyv + d.goff;

  // common LDS
  double* tl = sm;                       // [128] landmark times
  double* al = tl + NYLS_NARROW_MAX_M;          // [128] alpha
  double* dal = al + NYLS_NARROW_MAX_M;         // [128] W domega
  double* lin = dal + NYLS_NARROW_MAX_M;        // [128] sum rho k' - eta k
  double* part = lin + NYLS_NARROW_MAX_M;       // [256] partial sums
  double* red = part + NYLS_BLOCK;       // [16]
  double* rhs = red + 16;                // [kNz]
  double* pd = rhs + kNz;                // [TP][8] per-point data
  int* piv = reinterpret_cast<int*>(pd + TP * 8);  // [kNz]
  int* keep = piv + kNz;                 // [kKeep + 1] kept points, then their count
  double* big = reinterpret_cast<double*>(keep + kKeep + 2);
  // pass region
  double* K0 = big;                      // [TP][m]
  double* K1 = K0 + TP * maxm;           // [TP][m]
  double* Q = K1 + TP * maxm;            // [TP][gp]   (also the Gram reduction buffer)
  double* wr = Q + TP * round4(maxm + 2);  // [TP]

  for (int s = tid; s < m; s += NYLS_BLOCK) tl[s] = nyls_grid_t(d, d.lidx[s]);
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * xi[k];
    al[s] = acc;
  }
  if (tid == 0) keep[kKeep] = 0;
  __syncthreads();
  const double b = xi[maxm], lam = xi[maxm + 1];

  nyls_gram::Acc A;
  nyls_gram::setup(A, gp);
  const int ngc = NYLS_BLOCK / m, cs = tid % m, cg = tid / m;
  double linacc = 0.0, etasum = 0.0;
  int bad = 0;
  for (int i0 = 0; i0 < n; i0 += TP) {
    __syncthreads();
    nyls_gauss_tile<TP, CH>(d, i0, tl, inv_sigma, [&](int pt, int s, double z, double ev) {
      K0[pt * m + s] = ev;
      K1[pt * m + s] = -2.0 * z * inv_sigma * ev;
    });
    __syncthreads();
    {
      constexpr int TPG = NYLS_BLOCK / TP;
      const int pt = tid / TPG, sub = tid % TPG;
      double d0 = 0.0, d1 = 0.0;
      for (int s = sub; s < m; s += TPG) {
        d0 += K0[pt * m + s] * al[s];
        d1 += K1[pt * m + s] * al[s];
      }
      for (int o = TPG / 2; o > 0; o >>= 1) {
        d0 += __shfl_xor(d0, o);
        d1 += __shfl_xor(d1, o);
      }
      if (sub == 0) {
        const int i = i0 + pt;
        const bool ok = i < n && !nyls_is_condition_point(d, i);
        double rho = 0.0, eta = 0.0, y4 = 0.0, dd = 1.0, w = 0.0, fy = 0.0;
        if (ok) {
          fy = Fy[i];
          rho = d1 - F[i];
          eta = xi[maxm + 2 + i] - d0 - b;
          y4 = gam * (-rho * fy + eta);
          dd = gam * (1.0 + fy * fy - rho * Fyy[i]);
          w = (dd != 0.0 && dd == dd) ? gam * gam / dd : 0.0;
          if (!(fabs(dd) >= 1e-10 * gam)) {
            bad |= 1;
            const int slot = dd == dd ? atomicAdd(&keep[kKeep], 1) : kKeep;
            if (slot < kKeep) {
              keep[slot] = i;  // stays in the dense system (out of the weighted Gram)
              w = 0.0;
            } else {
              bad |= 2;
            }
          }
          etasum += eta;
        }
        pd[pt * 8 + 0] = rho;
        pd[pt * 8 + 1] = eta;
        pd[pt * 8 + 2] = y4;
        pd[pt * 8 + 3] = fy;
        wr[pt] = w;
      }
    }
    __syncthreads();
    for (int e = tid; e < TP * gp; e += NYLS_BLOCK) {
      const int pt = e / gp, a = e - pt * gp;
      double v = 0.0;
      if (wr[pt] != 0.0) {
        if (a < m) v = pd[pt * 8 + 3] * K1[pt * m + a] + K0[pt * m + a];
        else if (a == m) v = 1.0;
        else if (a == m + 1) v = pd[pt * 8 + 2] / gam;
      }
      Q[pt * gp + a] = v;
    }
    if (cg < ngc)
      for (int pt = cg; pt < TP; pt += ngc) {
        const int i = i0 + pt;
        if (i < n && !nyls_is_condition_point(d, i))
          linacc += pd[pt * 8 + 0] * K1[pt * m + cs] - pd[pt * 8 + 1] * K0[pt * m + cs];
      }
    __syncthreads();
    nyls_gram::accumulate(A, Q, gp, wr, TP);
  }
  double* Sw = ws + L.aux + (int64_t)g * g;  // weighted Gram (kernel space), g x g
  nyls_gram::finish(A, Q, Sw, g, g);
  part[tid] = (cg < ngc) ? linacc : 0.0;
  const double esum = nyls_block_sum(etasum, red);
  const double badf = nyls_block_sum((bad & 1) ? 1.0 : 0.0, red);  // small pivots met
  const double ovff = nyls_block_sum((bad & 2) ? 1.0 : 0.0, red);  // ... beyond kKeep
  __syncthreads();
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int gi = 0; gi < ngc; ++gi) acc += part[gi * m + s];
    lin[s] = acc;
  }
  __syncthreads();

  // Schur system in (omega padded to m, b, lambda): N2 = m + 2.
  const double* C0 = ws + L.aux;
  const int N2 = m + 2, lz = N2 + 1;
  double* Z = big;
  double* T = ws + L.tmp;  // T = (gamma C0 - Sw)[:m,:m] W   (global scratch)
  for (int e = tid; e < m * m; e += NYLS_BLOCK) {
    const int a = e / m, k = e - a * m;
    double acc = 0.0;
    if (k < r)
      for (int s = 0; s < m; ++s) acc += (gam * C0[a * g + s] - Sw[a * g + s]) * W[s * m + k];
    T[a * m + k] = acc;
  }
  __syncthreads();
  const double* phi1 = ws + L.H;
  for (int e = tid; e < N2 * N2; e += NYLS_BLOCK) {
    const int a = e / N2, c = e - a * N2;
    double val = 0.0;
    if (a < m && c < m) {
      if (a < r && c < r) {
        double acc = 0.0;
        for (int s = 0; s < m; ++s) acc += W[s * m + a] * T[s * m + c];
        val = acc + (a == c ? 1.0 : 0.0);
      } else {
        val = a == c ? 1.0 : 0.0;
      }
    } else if (a < m || c < m) {
      const int k = a < m ? a : c, o = a < m ? c : a;
      if (k < r) {
        if (o == m) {
          double acc = 0.0;
          for (int s = 0; s < m; ++s) acc += W[s * m + k] * (gam * C0[s * g + m] - Sw[s * g + m]);
          val = acc;
        } else {
          val = phi1[k];
        }
      }
    } else if (a == m && c == m) {
      val = gam * C0[m * g + m] - Sw[m * g + m];
    } else if (a != c) {
      val = 1.0;  // dY2/dlambda = dY3/db = 1
    }
    Z[a * lz + c] = val;
  }
  for (int a = tid; a < N2; a += NYLS_BLOCK) {
    double val = 0.0;
    if (a < m) {
      if (a < r) {
        double acc = 0.0, accu = 0.0;
        for (int s = 0; s < m; ++s) {
          acc += W[s * m + a] * lin[s];
          accu += W[s * m + a] * Sw[s * g + m + 1];
        }
        val = xi[a] + gam * acc + lam * phi1[a] + accu;
      }
    } else if (a == m) {
      val = -gam * esum + lam + Sw[m * g + m + 1];
    } else {
      double acc = 0.0;
      for (int k = 0; k < r; ++k) acc += phi1[k] * xi[k];
      val = acc + b - d.v[0];
    }
    rhs[a] = val;
  }
  __syncthreads();
  const int nkeep = min(keep[kKeep], kKeep);
  int sing;
  if (nkeep == 0) {
    sing = nyls_lu(Z, lz, N2, piv, red);
    nyls_lu_solve(Z, lz, N2, piv, rhs);   // rhs <- dz
  } else {
    // the kept points in index order (their slots were taken in arbitrary order)
    if (tid == 0)
      for (int a = 1; a < nkeep; ++a) {
        const int v = keep[a];
        int c = a - 1;
        for (; c >= 0 && keep[c] > v; --c) keep[c + 1] = keep[c];
        keep[c + 1] = v;
      }
    __syncthreads();
    // [[Z, Q_B], [Q_B^T, D_B]] in the workspace, Q_B = -gamma (W^T kappa_i, 1, 0) per kept
    // point, D_B = diag(d_i); right-hand side (rhs, Y4_B)
    const int Ne = N2 + nkeep;
    double* Ze = ws + L.aux + 2 * (int64_t)g * g;  // [Ne][Ne]
    for (int e = tid; e < Ne * Ne; e += NYLS_BLOCK) {
      const int a = e / Ne, c = e - a * Ne;
      double val = 0.0;
      if (a < N2 && c < N2) val = Z[a * lz + c];
      else if (a >= N2 && c >= N2) val = 0.0;  // diagonal entries below
      Ze[e] = val;
    }
    __syncthreads();
    for (int e = tid; e < nkeep * N2; e += NYLS_BLOCK) {
      const int j = e / N2, a = e - j * N2;
      const int i = keep[j];
      const double ti = nyls_grid_t(d, i), fy = Fy[i];
      double v = 0.0;
      if (a < r) {
        for (int s = 0; s < m; ++s) {
          const double z = (ti - tl[s]) * inv_sigma;
          const double e0 = exp(-z * z);
          v += W[s * m + a] * (fy * (-2.0 * z * inv_sigma * e0) + e0);
        }
        v *= -gam;
      } else if (a == m) {
        v = -gam;
      }
      Ze[a * Ne + N2 + j] = v;
      Ze[(N2 + j) * Ne + a] = v;
    }
    for (int j = tid; j < nkeep; j += NYLS_BLOCK) {
      const int i = keep[j];
      const double ti = nyls_grid_t(d, i), fy = Fy[i];
      double d0 = 0.0, d1 = 0.0;
      for (int s = 0; s < m; ++s) {
        const double z = (ti - tl[s]) * inv_sigma;
        const double e0 = exp(-z * z);
        d0 += e0 * al[s];
        d1 += -2.0 * z * inv_sigma * e0 * al[s];
      }
      const double rho = d1 - F[i];
      const double eta = xi[maxm + 2 + i] - d0 - b;
      Ze[(N2 + j) * Ne + N2 + j] = gam * (1.0 + fy * fy - rho * Fyy[i]);
      rhs[N2 + j] = gam * (-rho * fy + eta);
    }
    __syncthreads();
    sing = nyls_lu(Ze, Ne, Ne, piv, red);
    nyls_lu_solve(Ze, Ne, Ne, piv, rhs);  // rhs <- (dz, dy_B)
  }
  for (int s = tid; s < m; s += NYLS_BLOCK) {
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += W[s * m + k] * rhs[k];
    dal[s] = acc;
  }
  __syncthreads();
  // dy_i = (Y4_i - q_i^T dz) / d_i = (Y4_i + gamma (kappa_i^T dalpha + db)) / d_i
  const double db = rhs[m];
  double dmax = 0.0;
  for (int i = tid; i < n; i += NYLS_BLOCK) {
    if (nyls_is_condition_point(d, i)) continue;
    bool kept = false;
    for (int j = 0; j < nkeep; ++j) kept |= keep[j] == i;
    if (kept) continue;  // dy_i came from the dense system
    const double ti = nyls_grid_t(d, i);
    const double fy = Fy[i];
    double d0 = 0.0, d1 = 0.0, dk = 0.0;
    for (int s = 0; s < m; ++s) {
      const double z = (ti - tl[s]) * inv_sigma;
      const double e0 = exp(-z * z);
      const double e1 = -2.0 * z * inv_sigma * e0;
      d0 += e0 * al[s];
      d1 += e1 * al[s];
      dk += (fy * e1 + e0) * dal[s];
    }
    const double rho = d1 - F[i];
    const double eta = xi[maxm + 2 + i] - d0 - b;
    const double y4 = gam * (-rho * fy + eta);
    const double dd = gam * (1.0 + fy * fy - rho * Fyy[i]);
    const double dy = (dd != 0.0 && dd == dd) ? (y4 + gam * (dk + db)) / dd : 0.0;
    xi[maxm + 2 + i] -= dy;
    dmax = fmax(dmax, fabs(dy));
  }
  for (int j = tid; j < nkeep; j += NYLS_BLOCK) {
    const double dy = rhs[N2 + j];
    xi[maxm + 2 + keep[j]] -= dy;
    dmax = fmax(dmax, fabs(dy));
  }
  for (int a = tid; a < N2; a += NYLS_BLOCK) dmax = fmax(dmax, fabs(rhs[a]));
  // block max
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < NYLS_BLOCK / 64; ++w) mx = fmax(mx, red[w]);
    if (step_inf) step_inf[inst] = mx;
  }
  // x <- x - dz ; alpha and b for nyls_predict
  for (int k = tid; k < m; k += NYLS_BLOCK) xi[k] -= rhs[k];
  __syncthreads();
  for (int s = tid; s < m; s += NYLS_BLOCK) ws[L.alpha + s] = al[s] - dal[s];
  if (tid == 0) {
    xi[maxm] = b - db;
    xi[maxm + 1] = lam - rhs[m + 1];
    ws[L.x + m] = b - db;
    int bits = (int)ws[L.info + 1];
    if (badf > 0) bits |= NYLS_S_SMALL_PIVOT;
    if (ovff > 0) bits |= NYLS_S_PIVOT_OVERFLOW;
    if (sing) bits |= NYLS_S_SINGULAR;
    if (!(fabs(b - db) <= 1.7976931348623157e308)) bits |= NYLS_S_NONFINITE;
    if (status) status[inst] = bits;
  }
}

size_t step_lds_bytes(int maxm) {
  const size_t common = (4 * NYLS_NARROW_MAX_M + NYLS_BLOCK + 16 + kNz + TP * 8) * sizeof(double) +
                        (kNz + kKeep + 2) * sizeof(int);
  const int gp = round4(maxm + 2);
  size_t pass = (2 * (size_t)TP * maxm + (size_t)TP * gp + TP) * sizeof(double);
  const size_t redb = (size_t)nyls_gram::red_doubles(gp) * sizeof(double);
  const size_t qoff = 2 * (size_t)TP * maxm * sizeof(double);
  if (qoff + redb > pass) pass = qoff + redb;
  const size_t schur = (size_t)(maxm + 2) * (maxm + 3) * sizeof(double);
  return common + (pass > schur ? pass : schur);
}

size_t init_lds_bytes(int maxm) {
  const int gp = round4(maxm + 2);
  size_t q = 2 * (size_t)TP * gp;
  const size_t redd = nyls_gram::red_doubles(gp);
  if (redd > q) q = redd;
  return (2 * NYLS_NARROW_MAX_M + TP + q) * sizeof(double);
}

__global__ __launch_bounds__(NYLS_BLOCK) void k_riccati_eval(
    const nyls_desc* __restrict__ desc, const double* __restrict__ q, const double* __restrict__ x,
    int64_t xs, int maxm, int gauss_newton, double* __restrict__ F, double* __restrict__ Fy,
    double* __restrict__ Fyy) {
  const nyls_desc& d = desc[blockIdx.y];
  const double* y = x + (size_t)blockIdx.y * xs + maxm + 2;
  for (int i = blockIdx.x * NYLS_BLOCK + threadIdx.x; i < d.n; i += gridDim.x * NYLS_BLOCK) {
    const double yi = y[i];
    F[d.goff + i] = q[d.goff + i] - yi * yi;
    Fy[d.goff + i] = -2.0 * yi;
    Fyy[d.goff + i] = gauss_newton ? 0.0 : -2.0;
  }
}

}  // namespace

extern "C" int nyls_riccati_eval(const nyls_plan* pl, const double* q, const double* x,
                                 int32_t gauss_newton, double* F, double* Fy, double* Fyy,
                                 hipStream_t stream) {
  if (!pl || !q || !x || !F || !Fy || !Fyy) return NYLS_E_NULL;
  if (!nyls_plan_first_order(pl)) return NYLS_E_NONLINEAR;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  int gx = (pv.maxn + NYLS_BLOCK - 1) / NYLS_BLOCK;
  gx = gx > 64 ? 64 : gx;
  hipLaunchKernelGGL(k_riccati_eval, dim3(gx, pv.batch), dim3(NYLS_BLOCK), 0, stream, pv.d_desc, q, x,
                     (int64_t)nyls_plan_newton_stride(pl), pv.maxm, gauss_newton, F, Fy, Fyy);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}

extern "C" int64_t nyls_newton_state_stride(const nyls_plan* pl) { return nyls_plan_newton_stride(pl); }

extern "C" int nyls_newton_init(const nyls_plan* pl, double* x, void* ws, hipStream_t stream) {
  if (!pl || !x || !ws) return NYLS_E_NULL;
  const int order = nyls_plan_common_order(pl);
  if (order != 1 && order != 2) return NYLS_E_NONLINEAR;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  double* w = static_cast<double*>(ws);
  hipError_t e = nyls_launch_eig(pv, w, -1, stream);
  if (e != hipSuccess) return NYLS_E_HIP;
  if (order == 2) {
    e = nyls_launch_newton2_init(pv, w, x, (int64_t)nyls_plan_newton_stride(pl), stream);
    return e == hipSuccess ? NYLS_OK : NYLS_E_HIP;
  }
  const size_t lds = init_lds_bytes(pv.maxm);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_newton_init),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_newton_init, dim3(pv.batch), dim3(NYLS_BLOCK), lds, stream, pv.d_desc, w, x,
                     (int64_t)nyls_plan_newton_stride(pl), pv.maxm);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}

extern "C" int nyls_newton_state(const nyls_plan* pl, const double* x, double* u, const void* ws,
                                 hipStream_t stream) {
  if (!pl || !x || !u || !ws) return NYLS_E_NULL;
  const int order = nyls_plan_common_order(pl);
  if (order != 1 && order != 2) return NYLS_E_NONLINEAR;
  if (nyls_plan_get_view(pl).maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  const hipError_t e = nyls_launch_newton_state(nyls_plan_get_view(pl), static_cast<const double*>(ws),
                                                x, (int64_t)nyls_plan_newton_stride(pl), u, stream);
  return e == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}

extern "C" int nyls_newton_step(const nyls_plan* pl, const double* F, const double* Fy,
                                const double* Fyy, double* x, double* step_inf, int32_t* status,
                                void* ws, hipStream_t stream) {
  if (!pl || !F || !Fy || !Fyy || !x || !ws) return NYLS_E_NULL;
  const int order = nyls_plan_common_order(pl);
  if (order != 1 && order != 2) return NYLS_E_NONLINEAR;
  const nyls_plan_view pv = nyls_plan_get_view(pl);
  if (pv.maxm > NYLS_NARROW_MAX_M) return NYLS_E_SIZE;
  if (order == 2) {
    nyls_prof_begin(NYLS_K_NEWTON, stream);
    const hipError_t e = nyls_launch_newton2_step(pv, static_cast<double*>(ws), F, Fy, Fyy, x,
                                                  (int64_t)nyls_plan_newton_stride(pl), step_inf,
                                                  status, stream);
    nyls_prof_end(NYLS_K_NEWTON, stream);
    return e == hipSuccess ? NYLS_OK : NYLS_E_HIP;
  }
  const size_t lds = step_lds_bytes(pv.maxm);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_newton_step),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  nyls_prof_begin(NYLS_K_NEWTON, stream);
  hipLaunchKernelGGL(k_newton_step, dim3(pv.batch), dim3(NYLS_BLOCK), lds, stream, pv.d_desc,
                     static_cast<double*>(ws), F, Fy, Fyy, x, (int64_t)nyls_plan_newton_stride(pl),
                     step_inf, status, pv.maxm);
  nyls_prof_end(NYLS_K_NEWTON, stream);
  return hipGetLastError() == hipSuccess ? NYLS_OK : NYLS_E_HIP;
}
