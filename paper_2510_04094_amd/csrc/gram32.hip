// Mixed-precision operator Gram of Lemma 1 (Sec. 3.1) on the matrix cores, in the
// eigenbasis of K_mm.
//
// The Gram of the kernel-space rows q_i = (p_i, c_i, r_i) cannot be formed in FP32 and
// mapped through W afterwards: p_i's components along the small-eigenvalue directions of
// K_mm are tiny, FP32 rounding of the squared sum swamps them, and the system becomes too
// inexact for refinement to converge.  Each row is therefore rotated first,
//     g^_i = U^T p_i      (U: all eigenvectors of K_mm, FP32 copy),
// and the Gram of (g^_i, c_i, r_i) is accumulated; the KKT kernel applies Lambda^{-1/2}.
//
// One wavefront per instance.  Per step of 16 points:
//   * rotation on v_mfma_f32_16x16x4f32: A = kernel values (lane l: point l%16, landmark
//     4k + l/16, computed in registers: exp, Hermite factors, contraction with f_k),
//     B = U from LDS; the 16 x (16 NT) result stays in the accumulators;
//   * columns m and m+1 of the result are replaced by c_i and r_i;
//   * the result registers feed the Gram MFMAs directly as both operands (register v of
//     lane l holds point 4(l/16)+v, column l%16 + 16 X, which is exactly the operand
//     layout of k-step v), accumulating only the NT(NT+1)/2 upper-triangle tiles;
//   * FP32 accumulators are flushed into per-lane FP64 accumulators every CHUNK steps
//     (registers for up to 4 tile rows, LDS beyond), so long sums keep FP64 precision.
// Instances whose tile count differs from the template's NT leave immediately; the
// launcher issues one launch per tile count present in the batch.
#include "nyls_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int CHUNK = 4;  // 16-point steps between FP64 flushes

template <int NT>
__global__ __launch_bounds__(64) void k_gram32_rot(const nyls_desc* __restrict__ desc,
                                                   double* __restrict__ wsbase, int maxmk) {
  constexpr int T = NT * (NT + 1) / 2;
  constexpr int RN = 16 * NT;
  constexpr bool REG = T <= 15;  // FP64 accumulators in registers when they fit
  extern __shared__ double sm[];
  const nyls_desc& d = desc[blockIdx.x];
  const int m = d.m, p = d.p, n = d.n, g = m + 2;
  if ((g + 15) / 16 != NT) return;
  const int mk = (m + 3) & ~3;
  const nyls_wsl L = nyls_layout(m, p, 0);
  double* ws = wsbase + d.ws;
  const int lane = threadIdx.x;
  const int col = lane & 15, quad = lane >> 4;
  double* tlv = sm;                                              // [maxmk] landmark times
  float* U32 = reinterpret_cast<float*>(tlv + maxmk);            // [maxmk][RN]
  double* acc64 = reinterpret_cast<double*>(U32 + maxmk * RN);   // [T][4][64] unless REG
  double accr[REG ? T : 1][4];
#pragma unroll
  for (int t = 0; t < (REG ? T : 1); ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) accr[t][v] = 0.0;
  if (!REG)
    for (int e = lane; e < T * 256; e += 64) acc64[e] = 0.0;
  const double* U = ws + L.U;
  for (int e = lane; e < mk * RN; e += 64) {
    const int s = e / RN, k = e - s * RN;
    U32[e] = (s < m && k < m) ? (float)U[s * m + k] : 0.f;
  }
  for (int s = lane; s < mk; s += 64) tlv[s] = s < m ? nyls_grid_t(d, d.lidx[s]) : 0.0;
  __syncthreads();

  const double inv_sigma = 1.0 / d.sigma;
  const float isf = (float)inv_sigma;
  floatx4 accS[T];
#pragma unroll
  for (int t = 0; t < T; ++t) accS[t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int steps = (n + 15) / 16;
  for (int st = 0; st < steps; ++st) {
    // this lane's point for the rotation operand
    const int ia = 16 * st + col;
    const bool oka = ia < n && !nyls_is_condition_point(d, ia);
    float w[NYLS_MAX_P + 1];
    double ta = 0.0;
    if (oka) {
      nyls_opweights(p, [&](int k) { return (float)d.f[(size_t)(k - 1) * n + ia]; }, w);
      ta = nyls_grid_t(d, ia);
    } else {
#pragma unroll
      for (int q = 0; q <= NYLS_MAX_P; ++q) w[q] = 0.f;
    }
    floatx4 accG[NT];
#pragma unroll
    for (int X = 0; X < NT; ++X) accG[X] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < mk / 4; ++kk) {
      const int s = 4 * kk + quad;
      float v = 0.f;
      if (oka && s < m) {
        const float z = (float)((ta - tlv[s]) * inv_sigma);
        const float e = __expf(-z * z);
        float kd[NYLS_MAX_P + 1];
        float hm = 1.f, h = 2.f * z, sc = -isf;
        kd[0] = e;
        kd[1] = sc * h * e;
#pragma unroll
        for (int q = 1; q < NYLS_MAX_P; ++q) {
          const float hn = 2.f * z * h - 2.f * (float)q * hm;
          hm = h; h = hn;
          sc *= -isf;
          kd[q + 1] = sc * h * e;
        }
        v = nyls_dot5(w, kd);
      }
      const float* urow = U32 + s * RN + col;
#pragma unroll
      for (int X = 0; X < NT; ++X)
        accG[X] = __builtin_amdgcn_mfma_f32_16x16x4f32(v, urow[16 * X], accG[X], 0, 0, 0);
    }
    // columns m (c_i) and m+1 (r_i): lane holds points 16 st + 4 quad + v
#pragma unroll
    for (int X = 0; X < NT; ++X) {
      const int cidx = 16 * X + col;
      if (cidx == m || cidx == m + 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * st + 4 * quad + v;
          float val = 0.f;
          if (i < n && !nyls_is_condition_point(d, i))
            val = (cidx == m) ? -(float)d.f[(size_t)(p - 1) * n + i] : (float)d.r[i];
          accG[X][v] = val;
        }
      }
    }
    int t = 0;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = I; J < NT; ++J) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          accS[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(accG[I][v], accG[J][v], accS[t], 0, 0, 0);
        ++t;
      }
    if ((st + 1) % CHUNK == 0 || st + 1 == steps) {
#pragma unroll
      for (int tt = 0; tt < T; ++tt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (REG) accr[REG ? tt : 0][v] += (double)accS[tt][v];
          else acc64[(tt * 4 + v) * 64 + lane] += (double)accS[tt][v];
        }
        accS[tt] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  // tile (I, J): register v of lane l holds C[4 (l/16) + v][l % 16]
  double* out = ws + L.gram;
  int t = 0;
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int J = I; J < NT; ++J) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + 4 * quad + v, b = 16 * J + col;
        const double val = REG ? accr[REG ? t : 0][v] : acc64[(t * 4 + v) * 64 + lane];
        if (a < g && b < g) {
          out[a * g + b] = val;
          if (I != J) out[b * g + a] = val;
        }
      }
      ++t;
    }
}

template <int NT>
hipError_t launch_nt(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  constexpr int T = NT * (NT + 1) / 2;
  const int maxmk = (pv.maxm + 3) & ~3;
  const size_t lds = (T <= 15 ? 0 : (size_t)T * 256 * sizeof(double)) +
                     (size_t)maxmk * 16 * NT * sizeof(float) + (size_t)maxmk * sizeof(double);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram32_rot<NT>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_gram32_rot<NT>, dim3(pv.batch), dim3(64), lds, st, pv.d_desc, ws, maxmk);
  return hipGetLastError();
}

}  // namespace

hipError_t nyls_launch_gram32(const nyls_plan_view& pv, double* ws, hipStream_t st) {
  // bases with m + 2 > 64 take the FP64 Gram (nyls_launch_gram64_over64)
  const unsigned mask = pv.nt_mask & 0x1f;
  hipError_t e = hipSuccess;
  if ((mask >> 1) & 1) e = launch_nt<1>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 2) & 1)) e = launch_nt<2>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 3) & 1)) e = launch_nt<3>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 4) & 1)) e = launch_nt<4>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 5) & 1)) e = launch_nt<5>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 6) & 1)) e = launch_nt<6>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 7) & 1)) e = launch_nt<7>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 8) & 1)) e = launch_nt<8>(pv, ws, st);
  if (e == hipSuccess && ((mask >> 9) & 1)) e = launch_nt<9>(pv, ws, st);
  return e;
}
