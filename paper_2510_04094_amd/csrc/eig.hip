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
#include "nyls_internal.h"

namespace {

constexpr int kMaxSweeps = 40;
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

size_t eig_lds_bytes(int maxm, bool vlds) {
  const size_t mats = (size_t)(vlds ? 2 : 1) * maxm * (maxm + 1) * sizeof(double);
  const size_t tail = (64 * 3 + 8 + NYLS_MAX_M) * sizeof(double) + (64 * 2 + NYLS_MAX_M) * sizeof(int) +
                      NYLS_MAX_M * sizeof(double);
  return mats + tail;
}

}  // namespace

hipError_t nyls_launch_eig(const nyls_plan_view& pv, double* ws, int single, hipStream_t st) {
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
