// Online stage (Algorithm 3): M(theta) = H_1(theta_1) ... H_dt(theta_dt) with
// H_j = G_{d+j} x_2 q^p_j(theta_j), batched over theta samples, and its
// derivative dM/dtheta_j, obtained by replacing q^p_j with d q^p_j / d theta_j.
// The parameter cores are held in the Chebyshev coefficient basis, so
// q_k = T_k(t(theta)) and dq_k/dtheta = T_k'(t) dt/dtheta, with T_k' from the
// differentiated three-term recurrence T'_{k+1} = 2 T_k + 2 t T'_k - T'_{k-1}.
// Work is O(dt (n r^2 + r^3)) per theta, independent of N (Section 3.2).
// Everything is accumulated in double precision and rounded once on store.
#include "ttk_internal.h"

namespace ttk {

namespace {

struct OnlineArgs {
  const double* G[2];
  int r0[2], n[2], r1[2];
  double lo[2], hi[2];
  int dt;
};

// H_j(theta) (r0 x r1, column-major) or its derivative into out.
__device__ void form_factor(const OnlineArgs& oa, int j, double th, bool deriv, double* out, double* tk) {
  const int n = oa.n[j], r0 = oa.r0[j], r1 = oa.r1[j];
  const double lo = oa.lo[j], hi = oa.hi[j];
  if (threadIdx.x == 0) {
    const double t = (2.0 * th - (lo + hi)) / (lo - hi);
    const double dtdth = 2.0 / (lo - hi);
    double tm = 1.0, tc = t, dm = 0.0, dc = 1.0;
    tk[0] = deriv ? 0.0 : 1.0;
    if (n > 1) tk[1] = deriv ? dtdth : t;
    for (int k = 2; k < n; ++k) {
      const double tn = 2.0 * t * tc - tm;
      const double dn = 2.0 * tc + 2.0 * t * dc - dm;
      tm = tc; tc = tn; dm = dc; dc = dn;
      tk[k] = deriv ? dn * dtdth : tn;
    }
  }
  __syncthreads();
  const double* G = oa.G[j];
  for (int e = threadIdx.x; e < r0 * r1; e += blockDim.x) {
    const int a = e % r0, b = e / r0;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += G[a + (int64_t)k * r0 + (int64_t)b * r0 * n] * tk[k];
    out[a + (int64_t)b * r0] = s;
  }
  __syncthreads();
}

// C (m x n) = A (m x k) B (k x n), column-major, whole block.
__device__ void block_gemm(const double* A, const double* B, double* C, int m, int k, int n) {
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e % m, j = e / m;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += A[i + (int64_t)q * m] * B[q + (int64_t)j * k];
    C[e] = s;
  }
  __syncthreads();
}

template <class TT, class T>
__global__ void k_online(OnlineArgs oa, const TT* theta, int B, T* M, T* dM, double* work, size_t wstride) {
  __shared__ double tk[MAXN];
  double* w = work + (size_t)blockIdx.x * wstride;
  const int rs = oa.r0[0];
  const int rt = oa.r1[oa.dt - 1];
  const size_t msz = (size_t)rs * rt;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const double th0 = (double)theta[(int64_t)b * oa.dt + 0];
    if (oa.dt == 1) {
      double* H = w;
      form_factor(oa, 0, th0, false, H, tk);
      for (size_t e = threadIdx.x; e < msz; e += blockDim.x) M[b * msz + e] = (T)H[e];
      if (dM) {
        form_factor(oa, 0, th0, true, H, tk);
        for (size_t e = threadIdx.x; e < msz; e += blockDim.x) dM[b * msz + e] = (T)H[e];
      }
      __syncthreads();
    } else {
      const double th1 = (double)theta[(int64_t)b * oa.dt + 1];
      const int rm = oa.r1[0];
      double* H1 = w;
      double* H2 = H1 + (size_t)rs * rm;
      double* C = H2 + (size_t)rm * rt;
      double* E = C + msz;
      form_factor(oa, 0, th0, false, H1, tk);
      form_factor(oa, 1, th1, false, H2, tk);
      block_gemm(H1, H2, C, rs, rm, rt);
      for (size_t e = threadIdx.x; e < msz; e += blockDim.x) M[b * msz + e] = (T)C[e];
      if (dM) {
        form_factor(oa, 0, th0, true, E, tk);          // dH1 H2
        block_gemm(E, H2, C, rs, rm, rt);
        for (size_t e = threadIdx.x; e < msz; e += blockDim.x) dM[(size_t)b * 2 * msz + e] = (T)C[e];
        form_factor(oa, 1, th1, true, E, tk);          // H1 dH2
        block_gemm(H1, E, C, rs, rm, rt);
        for (size_t e = threadIdx.x; e < msz; e += blockDim.x) dM[(size_t)b * 2 * msz + msz + e] = (T)C[e];
      }
      __syncthreads();
    }
  }
}

// per-block workspace: H_1, H_2, the product and one derivative factor
size_t online_stride(const ParamCore* pc, int dt) {
  const size_t rs = pc[0].r0, rt = pc[dt - 1].r1;
  if (dt == 1) return rs * rt;
  const size_t rm = pc[0].r1;
  return rs * rm + rm * rt + rs * rt + std::max(rs * rm, rm * rt);
}

}  // namespace

void online_core_mixed(int theta_dtype, int out_dtype, const ParamCore* pc, int dt, const void* theta, int B,
                       void* M, void* dM, double* work, hipStream_t st) {
  if (B <= 0) return;
  OnlineArgs oa{};
  oa.dt = dt;
  size_t wstride = 0;
  for (int j = 0; j < dt; ++j) {
    oa.G[j] = pc[j].Ghat;
    oa.r0[j] = pc[j].r0;
    oa.n[j] = pc[j].n;
    oa.r1[j] = pc[j].r1;
    oa.lo[j] = pc[j].lo;
    oa.hi[j] = pc[j].hi;
  }
  wstride = online_stride(pc, dt);
  const int nblk = std::min(B, 256);
  const bool tf = theta_dtype == TTK_FP32, of = out_dtype == TTK_FP32;
  if (tf && of)
    hipLaunchKernelGGL((k_online<float, float>), dim3(nblk), dim3(256), 0, st, oa, static_cast<const float*>(theta),
                       B, static_cast<float*>(M), static_cast<float*>(dM), work, wstride);
  else if (tf)
    hipLaunchKernelGGL((k_online<float, double>), dim3(nblk), dim3(256), 0, st, oa,
                       static_cast<const float*>(theta), B, static_cast<double*>(M), static_cast<double*>(dM), work,
                       wstride);
  else if (of)
    hipLaunchKernelGGL((k_online<double, float>), dim3(nblk), dim3(256), 0, st, oa,
                       static_cast<const double*>(theta), B, static_cast<float*>(M), static_cast<float*>(dM), work,
                       wstride);
  else
    hipLaunchKernelGGL((k_online<double, double>), dim3(nblk), dim3(256), 0, st, oa,
                       static_cast<const double*>(theta), B, static_cast<double*>(M), static_cast<double*>(dM), work,
                       wstride);
}

void online_core(int dtype, const ParamCore* pc, int dt, const void* theta, int B, void* M, void* dM,
                 double* work, hipStream_t st) {
  online_core_mixed(dtype, dtype, pc, dt, theta, B, M, dM, work, st);
}

size_t online_work_doubles(const ParamCore* pc, int dt, int B) {
  return online_stride(pc, dt) * (size_t)std::min(std::max(B, 1), 256);
}

}  // namespace ttk
